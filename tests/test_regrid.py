"""Regridding without a GPU: the oracle's clustering against what clustering
must satisfy (coverage, disjointness, efficiency or indivisibility, size
limits, the exact boxes of simple shapes), injection conserving mass and a
lake at rest, and the library's clustering (host code) box for box equal to
the oracle's on random and on adjoint-flag fields."""
import numpy as np
import pytest

from oracle import regrid as R
from paper_1605_05320_amd import inputs as I


def _check_boxes(flags, boxes, eff, min_side, max_side):
    f = np.asarray(flags) != 0
    cover = np.zeros(f.shape, np.int32)
    for (i, j, nx, ny) in boxes:
        assert nx >= 1 and ny >= 1 and i >= 0 and j >= 0
        assert i + nx <= f.shape[1] and j + ny <= f.shape[0]
        cover[j:j + ny, i:i + nx] += 1
        sub = f[j:j + ny, i:i + nx]
        # tight: every edge row/column of a box holds a flag
        assert sub[0].any() and sub[-1].any() and sub[:, 0].any() and sub[:, -1].any()
        efficient = sub.sum() >= eff * nx * ny
        if efficient:
            assert nx <= max_side and ny <= max_side
        else:
            # not efficient: no hole and no admissible cut was left
            assert not (sub.sum(axis=0)[1:] == 0).any() and not (sub.sum(axis=1)[1:] == 0).any()
            assert nx < 2 * min_side and ny < 2 * min_side
    assert cover.max() <= 1, "boxes overlap"
    assert (cover[f] == 1).all(), "a flagged cell is not covered"


def test_simple_shapes():
    f = np.zeros((20, 30), np.int8)
    assert R.cluster(f, 0.7, 2, 16) == []
    f[3:9, 4:14] = 1
    assert R.cluster(f, 0.7, 2, 16) == [(4, 3, 10, 6)]
    f[12:18, 20:27] = 1                                   # a second, separate block
    assert R.cluster(f, 0.7, 2, 16) == [(4, 3, 10, 6), (20, 12, 7, 6)]
    g = np.zeros((20, 30), np.int8)
    g[2:5, 2:20] = 1                                      # an L: horizontal bar ...
    g[2:18, 2:5] = 1                                      # ... and vertical bar
    boxes = R.cluster(g, 0.9, 2, 32)
    _check_boxes(g, boxes, 0.9, 2, 32)
    assert len(boxes) == 2 and sum(nx * ny for (_, _, nx, ny) in boxes) == int(g.sum())
    # an efficient block larger than max_side is bisected
    h = np.ones((10, 40), np.int8)
    assert R.cluster(h, 0.7, 2, 16) == [(0, 0, 10, 10), (10, 0, 10, 10), (20, 0, 10, 10), (30, 0, 10, 10)]


@pytest.mark.parametrize("seed", range(6))
def test_random_fields_satisfy_the_rules(seed):
    rng = np.random.default_rng(seed)
    ny, nx = 48, 64
    f = np.zeros((ny, nx), np.int8)
    for _ in range(rng.integers(1, 6)):                  # a few blobs of random density
        cy, cx = rng.integers(0, ny), rng.integers(0, nx)
        r = rng.integers(3, 12)
        Y, X = np.mgrid[0:ny, 0:nx]
        f |= (((Y - cy) ** 2 + (X - cx) ** 2 < r * r) & (rng.random((ny, nx)) < rng.uniform(0.3, 1.0))).astype(np.int8)
    for eff, mn, mx in [(0.7, 2, 16), (0.5, 4, 32), (0.9, 1, 8)]:
        _check_boxes(f, R.cluster(f, eff, mn, mx), eff, mn, mx)


def test_injection_conserves_and_keeps_rest():
    rng = np.random.default_rng(1)
    B = -rng.uniform(100.0, 4000.0, (12, 16))
    h = -B.copy()
    hu = rng.normal(0, 1, B.shape)
    boxes = [(2, 3, 5, 4), (9, 0, 7, 6)]
    for r in (1, 2, 4):
        for (box, (hf, huf, Bf)) in zip(boxes, R.prolong([h, hu, B], boxes, r)):
            i, j, nx, ny = box
            assert hf.shape == (ny * r, nx * r)
            assert np.isclose(huf.sum(), r * r * hu[j:j + ny, i:i + nx].sum(), rtol=1e-14)
            assert np.array_equal(hf + Bf, np.zeros_like(hf))


# --------------------------------------------------------------------------
# the library's clustering equals the oracle's (host code, no GPU needed)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def S():
    from paper_1605_05320_amd import swe
    swe.lib()
    return swe


@pytest.mark.parametrize("seed", range(8))
def test_library_clustering_equals_oracle(S, seed):
    rng = np.random.default_rng(100 + seed)
    ny, nx = int(rng.integers(20, 90)), int(rng.integers(20, 90))
    dens = rng.uniform(0.02, 0.6)
    f = (rng.random((ny, nx)) < dens).astype(np.int8)
    f[:, : nx // 3] &= (rng.random((ny, nx // 3)) < 0.2).astype(np.int8)   # uneven density
    for eff, mn, mx in [(0.7, 2, 16), (0.8, 4, 32), (0.5, 1, 64)]:
        assert S.cluster(f, eff, mn, mx) == R.cluster(f, eff, mn, mx)


def test_library_clustering_of_adjoint_flags(S, oracle):
    """On a real flag field: the accumulated adjoint flags of a basin run."""
    O = oracle
    b = I.basin(96, 3)
    g = O.Grid(96, 96, b.grid.dx, b.grid.dy)
    r = O.run(g, O.Params(), O.NONLINEAR, b.B, b.eta0, (b.target[0], b.target[1], 60e3), 0.0, 1800.0, 3600.0,
              6, 1e-4, flag_every=3)
    f = r.flags_at[3]
    assert f.any()
    for eff, mn, mx in [(0.7, 2, 16), (0.85, 4, 32)]:
        boxes = S.cluster(f, eff, mn, mx)
        assert boxes == R.cluster(f, eff, mn, mx)
        _check_boxes(f, boxes, eff, mn, mx)


def test_library_clustering_rejects_bad_arguments(S):
    f = np.ones((4, 4), np.int8)
    for args in [(0.0, 2, 8), (1.5, 2, 8), (0.7, 0, 8), (0.7, 4, 7)]:
        with pytest.raises(S.SweError):
            S.cluster(f, *args)
