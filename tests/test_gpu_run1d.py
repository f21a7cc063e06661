"""One-dimensional runs with each phase in one workgroup (the default for
grids of up to 3840 cells) against the same runs launched step by step
(launch_per_step = 1): every output equal in every bit.  The step-by-step
runs are compared with the oracle elsewhere; this covers ragged strips, the
largest grid that fits, the first that does not, both boundary kinds, dry
cells, order 1, a flag cadence, an adjoint grid of its own, and segments
long enough to take many rounds of attempts."""
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


def run(S, n, K, tf, tol, per_step, flag_every=1, order=2, bc_lo=0, land=0, adj_n=0, seed=0, ts=0.0):
    s = I.shelf1d(n, seed=seed)
    B = s.B.copy()
    if land:
        B[-land:] = 5.0                                    # dry land at the shore
    g = S.Grid(n, 1, s.dx, 1.0, s.x_lo, bc=(bc_lo, 0, 0, 0))
    prm = S.Params(model=S.LINEAR, order=order)
    an = adj_n or n
    frames = torch.zeros(K + 1, 2, 1, an, dtype=torch.float64, device=DEV)
    q = [torch.zeros(1, n, dtype=torch.float64, device=DEV) for _ in range(2)]
    fat = torch.zeros(K + 1, 1, n, dtype=torch.int8, device=DEV)
    sfl = torch.zeros(K + 1, 1, n, dtype=torch.int8, device=DEV)
    acc = torch.zeros(1, n, dtype=torch.int8, device=DEV)
    macc = torch.zeros(1, n, dtype=torch.float64, device=DEV)
    kw = {}
    if adj_n:
        sa = I.shelf1d(adj_n, seed=seed)
        Ba = sa.B.copy()
        if land:
            Ba[sa.x_lo + (np.arange(adj_n) + 0.5) * sa.dx > s.x_lo + (n - land) * s.dx] = 5.0
        kw = dict(adj_grid=S.Grid(adj_n, 1, sa.dx, 1.0, sa.x_lo, bc=(bc_lo, 0, 0, 0)), adj_B=dev(Ba.reshape(1, -1)))
    pb = S.make_problem(g, prm, dev(B.reshape(1, n)), dev(s.eta0.reshape(1, n)), s.target, 0.0, ts, tf, K, tol,
                        frames, q, fat, acc, macc, flag_every=flag_every, surface_tol=0.02, surface_flags_at=sfl,
                        launch_per_step=per_step, **kw)
    ws = torch.empty(S.swe_run_workspace_bytes(pb) // 8 + 64, dtype=torch.float64, device=DEV)
    r = S.swe_run(pb, ws)
    torch.cuda.synchronize()
    res = (r.n_adj_steps, r.n_sub, r.n_fwd_steps, r.n_rejected, r.n_flag_calls, r.n_clamped, r.dt_adj, r.t_end)
    return res, [host(frames), host(q[0]), host(q[1]), host(macc)], [host(fat), host(sfl), host(acc)]


CASES = [
    # n, K, tf, tol, extra
    (2000, 60, 10800.0, 1e-3, {}),                       # the 3 h shelf with 60 snapshots
    (8, 4, 1800.0, 1e-3, {}),                            # one strip, mostly halo lanes
    (60, 6, 1800.0, 1e-3, {"flag_every": 2, "ts": 600.0}),   # exactly one full strip
    (61, 8, 1800.0, 1e-3, {}),
    (119, 8, 1800.0, 1e-3, {"bc_lo": 1}),
    (121, 8, 1800.0, 1e-3, {"order": 1}),
    (1999, 12, 3600.0, 1e-3, {"flag_every": 3, "land": 40}),
    (3840, 6, 1800.0, 1e-3, {"ts": 900.0}),              # the largest grid of one workgroup
    (3841, 6, 1800.0, 1e-3, {}),                         # launched step by step either way
    (2000, 2, 10800.0, 1e-3, {}),                        # ~6000 attempts per segment: many rounds
    (1200, 10, 3600.0, 1e-3, {"adj_n": 600, "land": 20}),   # adjoint on a grid of its own
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}_K{c[1]}_{'_'.join(c[4])}" for c in CASES])
def test_one_workgroup_equals_launch_per_step(S, case):
    n, K, tf, tol, kw = case
    r0, f0, i0 = run(S, n, K, tf, tol, 0, **kw)
    r1, f1, i1 = run(S, n, K, tf, tol, 1, **kw)
    assert r0 == r1, (r0, r1)
    for x, y in zip(f0, f1):
        assert np.array_equal(x.view(np.int64), y.view(np.int64))
    for x, y in zip(i0, i1):
        assert np.array_equal(x, y)
    if n >= 60:
        assert i0[2].any()


@pytest.mark.parametrize("seed", range(6))
def test_random_problems_one_workgroup_equals_launch_per_step(S, seed):
    """Random sizes (including the largest grid of one workgroup), boundaries,
    orders, land, cadences, windows and adjoint grids."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.choice([int(rng.integers(2, 130)), int(rng.integers(130, 3841)), 3840]))
    kw = dict(flag_every=int(rng.integers(1, 4)), order=int(rng.integers(1, 3)), bc_lo=int(rng.integers(0, 2)),
              land=int(rng.integers(0, n // 4 + 1)), ts=float(rng.choice([0.0, 600.0])), seed=int(rng.integers(0, 8)))
    if n >= 16 and rng.random() < 0.4:
        kw["adj_n"] = int(rng.integers(8, n // 2 + 2))
    K, tf = int(rng.integers(1, 13)), float(rng.choice([900.0, 1800.0]))
    r0, f0, i0 = run(S, n, K, tf, 1e-3, 0, **kw)
    r1, f1, i1 = run(S, n, K, tf, 1e-3, 1, **kw)
    assert r0 == r1, (n, K, kw, r0, r1)
    for x, y in zip(f0, f1):
        assert np.array_equal(x.view(np.int64), y.view(np.int64)), (n, K, kw)
    for x, y in zip(i0, i1):
        assert np.array_equal(x, y), (n, K, kw)
