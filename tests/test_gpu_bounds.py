"""Exact zero-region skipping in the flag pass: the adjoint is exactly zero
outside the domain of dependence of the target (Sec. 4), so a snapshot
contributes |<q, 0>| = 0 wherever it is zero.  adj_frame_bounds records each
snapshot's box of non-zero cells; flag passes given the boxes skip the
snapshots that are zero at a cell.  The results must be the same in every
bit with and without the boxes."""
import numpy as np
import pytest

from paper_1605_05320_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_05320_amd import swe
    swe.lib()
    return swe


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def np_bounds(frames):
    """(i_lo, i_hi, j_lo, j_hi) of the non-zero cells of each snapshot."""
    out = []
    for f in frames:
        nz = np.any(f != 0.0, axis=0)
        jj, ii = np.nonzero(nz)
        ny, nx = nz.shape
        out.append([ii.min(), ii.max(), jj.min(), jj.max()] if len(ii) else [nx, -1, ny, -1])
    return np.array(out, np.int32)


def adjoint_frames(S, n, K, shape, seed=3, T=3600.0):
    """Snapshots of an adjoint run of the basin.  With the disk target (the
    indicator of Sec. 6) they are exactly zero outside a region that grows by
    at most one cell per sub-step; a Gaussian target is non-zero wherever its
    exponential does not underflow."""
    b = I.basin(n, seed)
    g = S.Grid(n, n, b.grid.dx, b.grid.dy)
    p = S.Params()
    Bd = dev(b.B)
    frames = torch.zeros(K + 1, 3, n, n, dtype=torch.float64, device=DEV)
    q = [frames[0, c] for c in range(3)]
    S.adj_target(g, p, Bd, b.target[0], b.target[1], 30e3, shape, q)
    wa = [torch.empty(n, n, dtype=torch.float64, device=DEV) for _ in range(3)]
    wb = [torch.empty(n, n, dtype=torch.float64, device=DEV) for _ in range(3)]
    ds = T / K
    nsub = int(np.ceil(ds / (0.9 * b.grid.dx / np.sqrt(9.81 * 4000.0))))
    for k in range(1, K + 1):
        cur = [frames[k - 1, c] for c in range(3)]
        for s_ in range(nsub):
            dst = [frames[k, c] for c in range(3)] if s_ == nsub - 1 else (wa if s_ % 2 == 0 else wb)
            S.adj_step(g, p, Bd, cur, dst, ds / nsub)
            cur = dst
    torch.cuda.synchronize()
    return b, g, Bd, frames


def test_frame_bounds_match_numpy(S):
    rng = np.random.default_rng(4)
    ny, nx, K = 70, 130, 5
    frames = np.zeros((K + 1, 3, ny, nx))
    frames[1, 0, 10:20, 30:41] = rng.normal(size=(10, 11))
    frames[2, 2, 5, 7] = 1e-300                       # one tiny value in one plane
    frames[3, 1, :, :] = rng.normal(size=(ny, nx))    # everything
    frames[4, 0, 69, 0] = np.nan                      # a NaN counts as non-zero
    frames[5, 1, 33, 129] = -0.0                      # a negative zero does not
    g = S.Grid(nx, ny, 100.0, 100.0)
    bd = torch.full((4 * (K + 1),), 12345, dtype=torch.int32, device=DEV)
    S.adj_frame_bounds(g, dev(frames), K, bd)
    torch.cuda.synchronize()
    got = host(bd).reshape(K + 1, 4)
    assert np.array_equal(got, np_bounds(frames)), got
    assert list(got[0]) == [nx, -1, ny, -1] and list(got[5]) == [nx, -1, ny, -1]


@pytest.mark.parametrize("shape", ["disk", "gauss"])
@pytest.mark.parametrize("interp", [False, True])
def test_flags_with_bounds_bit_identical(S, interp, shape):
    n, K, tol = 160, 12, 1e-4
    b, g, Bd, frames = adjoint_frames(S, n, K, S.DISK if shape == "disk" else S.GAUSS)
    fr = host(frames)
    bd = torch.empty(4 * (K + 1), dtype=torch.int32, device=DEV)
    S.adj_frame_bounds(g, frames, K, bd)
    torch.cuda.synchronize()
    bnp = host(bd).reshape(K + 1, 4)
    assert np.array_equal(bnp, np_bounds(fr))
    areas = [(r[1] - r[0] + 1) * (r[3] - r[2] + 1) if r[1] >= 0 else 0 for r in bnp]
    assert areas[0] > 0
    if shape == "disk":
        assert areas[0] < n * n // 20 and areas[1] < n * n // 4, areas    # the last snapshots are compact
        assert areas == sorted(areas), areas
    noise = np.random.default_rng(2).uniform(-0.05, 0.05, b.B.shape)
    if interp:
        # forward grid twice as fine as the snapshots'
        nf = 2 * n
        bf = I.basin(nf, 3)
        gf = S.Grid(nf, nf, bf.grid.dx, bf.grid.dy)
        h = np.maximum(0.0, bf.eta0 + np.repeat(np.repeat(noise, 2, 0), 2, 1) - bf.B)
        q = [dev(h), dev(0.3 * h), dev(-0.2 * h)]
        Bf = dev(bf.B)
    else:
        h = np.maximum(0.0, b.eta0 + noise - b.B)
        q = [dev(h), dev(0.3 * h), dev(-0.2 * h)]
    outs = {}
    for use in (False, True):
        shape = (2 * n, 2 * n) if interp else (n, n)
        fl = torch.empty(shape, dtype=torch.int8, device=DEV)
        m = torch.empty(shape, dtype=torch.float64, device=DEV)
        acc = torch.zeros(shape, dtype=torch.int8, device=DEV)
        macc = torch.zeros(shape, dtype=torch.float64, device=DEV)
        for (lo, hi) in [(0, K), (0, 2), (4, 9), (K, K)]:
            if interp:
                S.adj_flag_interp(gf, S.Params(), Bf, q, g, Bd, frames, K, lo, hi, tol, fl, m, acc, macc,
                                  bounds=bd if use else None)
            else:
                S.adj_flag(g, S.Params(), Bd, q, frames, K, lo, hi, tol, fl, m, acc, macc, bounds=bd if use else None)
            torch.cuda.synchronize()
            outs[(use, lo, hi)] = (host(fl), host(m))
        outs[use] = (host(acc), host(macc))
    for key in [(0, K), (0, 2), (4, 9), (K, K)]:
        f0, m0 = outs[(False,) + key]
        f1, m1 = outs[(True,) + key]
        assert np.array_equal(f0, f1) and np.array_equal(m0.view(np.int64), m1.view(np.int64)), key
    assert np.array_equal(outs[False][0], outs[True][0])
    assert np.array_equal(outs[False][1].view(np.int64), outs[True][1].view(np.int64))
    assert outs[True][0].any()


@pytest.mark.parametrize("shape", ["disk", "gauss"])
def test_run_with_and_without_skipping_bit_identical(S, shape):
    """swe_run with the snapshots' boxes (default) and reading every snapshot
    in full (full_frames = 1): every output equal in every bit."""
    n, K, tol = 128, 16, 1e-4
    b = I.basin(n, 3)
    g = S.Grid(n, n, b.grid.dx, b.grid.dy)
    res = {}
    for full in (0, 1):
        frames = torch.zeros(K + 1, 3, n, n, dtype=torch.float64, device=DEV)
        q = [torch.zeros(n, n, dtype=torch.float64, device=DEV) for _ in range(3)]
        fat = torch.zeros(K + 1, n, n, dtype=torch.int8, device=DEV)
        acc = torch.zeros(n, n, dtype=torch.int8, device=DEV)
        macc = torch.zeros(n, n, dtype=torch.float64, device=DEV)
        pb = S.make_problem(g, S.Params(), dev(b.B), dev(b.eta0), b.target, 0.0, 3600.0, 7200.0, K, tol, frames, q,
                            fat, acc, macc, flag_every=1, full_frames=full,
                            shape=S.DISK if shape == "disk" else S.GAUSS)
        ws = torch.empty(S.swe_run_workspace_bytes(pb) // 8 + 64, dtype=torch.float64, device=DEV)
        r = S.swe_run(pb, ws)
        res[full] = ([host(x) for x in [frames, *q, macc]], [host(fat), host(acc)],
                     (r.n_fwd_steps, r.n_flag_calls, r.t_end))
    assert res[0][2] == res[1][2]
    for x, y in zip(res[0][0], res[1][0]):
        assert np.array_equal(x.view(np.int64), y.view(np.int64))
    for x, y in zip(res[0][1], res[1][1]):
        assert np.array_equal(x, y)
    assert res[0][1][1].any()


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("interp", [False, True])
def test_random_boxes_bit_identical(S, seed, interp):
    """Snapshots that are non-zero only in random rectangles (single cells,
    whole rows, the grid's corners and edges, empty snapshots), on a ragged
    grid: flags and m with the boxes equal those without, for random windows."""
    rng = np.random.default_rng(100 + seed)
    nx, ny, K = int(rng.integers(70, 200)), int(rng.integers(40, 130)), 9
    ax, ay = (nx // 2 + 3, ny // 2 + 2) if interp else (nx, ny)
    frames = np.zeros((K + 1, 3, ay, ax))
    for k in range(K + 1):
        kind = rng.integers(0, 5)
        if kind == 0:
            continue                                            # zero everywhere
        if kind == 1:
            i, j = int(rng.integers(0, ax)), int(rng.integers(0, ay))
            frames[k, int(rng.integers(0, 3)), j, i] = rng.normal()    # one cell, one plane
            continue
        i0, j0 = int(rng.integers(0, ax)), int(rng.integers(0, ay))
        i1, j1 = int(rng.integers(i0, ax)) + 1, int(rng.integers(j0, ay)) + 1
        if kind == 3:
            i0, i1 = 0, ax                                       # whole rows
        frames[k, :, j0:j1, i0:i1] = rng.normal(size=(3, j1 - j0, i1 - i0))
    b = I.basin(max(nx, ny), seed)
    B = b.B[:ny, :nx]
    h = np.maximum(0.0, b.eta0[:ny, :nx] + rng.uniform(-0.05, 0.05, (ny, nx)) - B)
    q = [dev(h), dev(0.3 * h), dev(-0.2 * h)]
    g = S.Grid(nx, ny, 1000.0, 1000.0)
    fr = dev(frames)
    bd = torch.empty(4 * (K + 1), dtype=torch.int32, device=DEV)
    ga = S.Grid(ax, ay, 2000.0, 2000.0)
    S.adj_frame_bounds(ga if interp else g, fr, K, bd)
    Bd = dev(B)
    Ba = dev(np.full((ay, ax), -1000.0))
    for lo, hi in [(0, K), (int(rng.integers(0, K)), K), (3, 3), (K, K - 1)]:
        res = []
        for use in (None, bd):
            fl = torch.empty(ny, nx, dtype=torch.int8, device=DEV)
            m = torch.empty(ny, nx, dtype=torch.float64, device=DEV)
            if interp:
                S.adj_flag_interp(g, S.Params(), Bd, q, ga, Ba, fr, K, lo, hi, 1e-3, fl, m, bounds=use)
            else:
                S.adj_flag(g, S.Params(), Bd, q, fr, K, lo, hi, 1e-3, fl, m, bounds=use)
            torch.cuda.synchronize()
            res.append((host(fl), host(m)))
        assert np.array_equal(res[0][0], res[1][0]), (lo, hi)
        assert np.array_equal(res[0][1].view(np.int64), res[1][1].view(np.int64)), (lo, hi)
