"""swe_run_static (the allocation-free driver) through the C ABI against
swe_run with a workspace of the caller's: two calls in a row, the second on a
smaller grid (the library's array keeps the first call's contents), each
bit-identical to swe_run on the same problem."""
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


def problem(S, n, seed, K=8, ts=1800.0, tf=3600.0, tol=1e-4):
    b = I.basin(n, seed)
    g = S.Grid(n, n, b.grid.dx, b.grid.dy)
    out = {
        "frames": torch.full((K + 1, 3, n, n), float("nan"), dtype=torch.float64, device=DEV),
        "q": [torch.full((n, n), float("nan"), dtype=torch.float64, device=DEV) for _ in range(3)],
        "flags_at": torch.full((K + 1, n, n), 7, dtype=torch.int8, device=DEV),
        "acc": torch.zeros(n, n, dtype=torch.int8, device=DEV),
        "macc": torch.zeros(n, n, dtype=torch.float64, device=DEV),
    }
    pb = S.make_problem(g, S.Params(), dev(b.B), dev(b.eta0), (b.target[0], b.target[1], 60e3), 0.0, ts, tf, K,
                        tol, out["frames"], out["q"], out["flags_at"], out["acc"], out["macc"], flag_every=2)
    return pb, out


def results(out, res):
    t = [out["frames"], *out["q"], out["flags_at"], out["acc"], out["macc"]]
    return [x.cpu().numpy() for x in t], (res.n_adj_steps, res.n_sub, res.n_fwd_steps, res.n_rejected,
                                          res.n_flag_calls, res.n_clamped, res.dt_adj, res.t_end)


@pytest.mark.parametrize("sizes", [((160, 3), (72, 5))])
def test_static_workspace_matches_swe_run(S, sizes):
    for n, seed in sizes:
        print(f"swe_run_static: {n}^2 basin seed {seed}", flush=True)
        pb, out = problem(S, n, seed)
        assert S.swe_run_workspace_bytes(pb) <= S.STATIC_WORKSPACE_BYTES
        ws = torch.empty(S.swe_run_workspace_bytes(pb) // 8 + 64, dtype=torch.float64, device=DEV)
        ref, rcount = results(out, S.swe_run(pb, ws))
        pb2, out2 = problem(S, n, seed)
        got, gcount = results(out2, S.swe_run_static(pb2))
        assert gcount == rcount
        for x, y in zip(got, ref):
            assert np.array_equal(x, y, equal_nan=False)
        assert ref[-2].any(), "some cell must be flagged"


def problem1d(S, n, seed, K=12, tf=3600.0, tol=1e-3):
    s = I.shelf1d(n, seed=seed)
    g = S.Grid(n, 1, s.dx, 1.0, s.x_lo)
    out = {
        "frames": torch.full((K + 1, 2, 1, n), float("nan"), dtype=torch.float64, device=DEV),
        "q": [torch.full((1, n), float("nan"), dtype=torch.float64, device=DEV) for _ in range(2)],
        "flags_at": torch.full((K + 1, 1, n), 7, dtype=torch.int8, device=DEV),
        "acc": torch.zeros(1, n, dtype=torch.int8, device=DEV),
        "macc": torch.zeros(1, n, dtype=torch.float64, device=DEV),
    }
    pb = S.make_problem(g, S.Params(model=S.LINEAR), dev(s.B.reshape(1, n)), dev(s.eta0.reshape(1, n)), s.target,
                        0.0, 0.0, tf, K, tol, out["frames"], out["q"], out["flags_at"], out["acc"], out["macc"])
    return pb, out


@pytest.mark.parametrize("sizes", [((2000, 0), (1000, 1))])
def test_static_workspace_matches_swe_run_1d(S, sizes):
    """The same for 1D runs, whose phases run in one workgroup with their
    recorded states in the workspace."""
    for n, seed in sizes:
        print(f"swe_run_static: 1D {n} cells seed {seed}", flush=True)
        pb, out = problem1d(S, n, seed)
        assert S.swe_run_workspace_bytes(pb) <= S.STATIC_WORKSPACE_BYTES
        ws = torch.empty(S.swe_run_workspace_bytes(pb) // 8 + 64, dtype=torch.float64, device=DEV)
        ref, rcount = results(out, S.swe_run(pb, ws))
        pb2, out2 = problem1d(S, n, seed)
        got, gcount = results(out2, S.swe_run_static(pb2))
        assert gcount == rcount
        for x, y in zip(got, ref):
            assert np.array_equal(x, y, equal_nan=False)
        assert ref[-2].any(), "some cell must be flagged"
