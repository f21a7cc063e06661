"""Host-side checks of the batched-level scheduler (no GPU): every column of
every patch is an output lane exactly once, lanes of a strip are contiguous
with their ghost columns, no patch is split across jobs, pass rows cover the
patches, and packing uses fewer wavefront-rows than one strip per wavefront."""
import numpy as np
import pytest

from paper_1605_05320_amd import inputs as I


@pytest.fixture(scope="module")
def S():
    from paper_1605_05320_amd import swe
    swe.lib()
    return swe


def decode(lanes):
    idle = lanes < 0
    patch = np.where(idle, -1, lanes >> 32)
    role = np.where(idle, 0, (lanes >> 16) & 0xffff)
    col = np.where(idle, 0, (lanes & 0xffff) - 32768)
    return patch, role, col


@pytest.mark.parametrize("chunk", [0, 16])
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("seed", [4, 5])
def test_schedule_covers_every_cell_once(S, kind, seed, chunk):
    ps = I.patches(400, seed=seed)
    tab, ncells = S.patch_table(ps.nx, ps.ny, ps.dx)
    lanes, rows, jp, row0 = S.level_schedule(tab, kind, chunk)
    npass = len(rows)
    assert lanes.shape == (npass * 64,) and jp[0] == 0 and jp[-1] == npass
    patch, role, col = decode(lanes)
    spans = {}
    job_of_patch = {}
    for j in range(len(jp) - 1):
        for q in range(jp[j], jp[j + 1]):
            sl = slice(q * 64, (q + 1) * 64)
            if chunk:
                assert rows[q] <= chunk
            for l in range(64):
                p = int(patch[sl][l])
                if p < 0:
                    continue
                if not chunk:
                    assert job_of_patch.setdefault(p, j) == j      # one job per patch
                    assert row0[q] == 0 and rows[q] >= ps.ny[p]
                else:
                    assert 0 <= row0[q] < ps.ny[p] and row0[q] + rows[q] <= ps.ny[p]
                if role[sl][l] & 1:
                    c = int(col[sl][l])
                    assert 0 <= c < ps.nx[p]
                    spans.setdefault((p, c), []).append((int(row0[q]), int(min(row0[q] + rows[q], ps.ny[p]))))
                    # two ghost columns on each side of every output lane
                    for d in (-2, -1, 1, 2):
                        assert 0 <= l + d < 64 and patch[sl][l + d] == p and col[sl][l + d] == c + d
                if role[sl][l] & 2:
                    assert 0 <= int(col[sl][l]) <= ps.nx[p]
    assert len(spans) == int(sum(ps.nx))
    for (p, c), sp in spans.items():
        sp.sort()
        # the row ranges of a column tile [0, ny) exactly once
        assert sp[0][0] == 0 and sp[-1][1] == ps.ny[p]
        assert all(a[1] == b[0] for a, b in zip(sp, sp[1:]))


def test_packing_saves_wavefront_rows(S):
    ps = I.patches(3000, seed=4)
    tab, _ = S.patch_table(ps.nx, ps.ny, ps.dx)
    cost = []
    for kind in (0, 1):
        lanes, rows, jp, _ = S.level_schedule(tab, kind)
        cost.append(float((rows + 2.5).sum()))
    assert cost[1] < 0.8 * cost[0]


def test_schedule_rejects_bad_input(S):
    tab, _ = S.patch_table([1], [8], [100.0])
    with pytest.raises(S.SweError):
        S.level_schedule(tab, 1)
    tab, _ = S.patch_table([8, 8], [8, 8], [100.0, 100.0])
    S.level_schedule(tab, 1)
    tab[1].bc[2] = 2      # neither wall nor extrapolation
    with pytest.raises(S.SweError, match="bc"):
        S.level_schedule(tab, 1)
