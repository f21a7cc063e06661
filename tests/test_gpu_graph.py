"""HIP-graph capture of the device-controlled stepping (the form the headline
step is timed in), of the same with device-scheduled flag passes, of
adjoint steps, and of a batched level's advance (launch per attempt, and the one persistent launch):
a graph of
K attempts, captured once, is replayed several times with eager work and
synchronisations in between, and the state and control block after every
replay equal, bit for bit, those of the same attempts issued eagerly."""
import numpy as np
import pytest

from paper_1605_05320_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F64 = dict(dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_05320_amd import swe
    swe.lib()
    return swe


def current(S, ctl, a, b):
    c = S.read_ctl(ctl)
    q = b if c.s.cur else a
    return [x.cpu().numpy().copy() for x in q], (c.s.t, c.s.dt, c.s.n_accepted, c.s.n_rejected, c.cfl_bits)


def capture(fn):
    """fn(stream) recorded into a graph on a side stream."""
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(graph, stream=gs):
            fn(gs)
    torch.cuda.current_stream().wait_stream(gs)
    torch.cuda.synchronize()
    return graph


def check_replays(S, run_eager, run_in_graph, ctl_e, ctl_g, ea, eb, ga, gb, reps=3):
    graph = capture(run_in_graph)
    scratch = torch.randn(1 << 16, **F64)
    for r in range(reps):
        run_eager()
        torch.cuda.synchronize()
        want_q, want_c = current(S, ctl_e, ea, eb)
        graph.replay()
        # the program's own eager work between replays
        scratch.mul_(1.0001).add_(float(r))
        torch.cuda.synchronize()
        got_q, got_c = current(S, ctl_g, ga, gb)
        print(f"replay {r}: t = {got_c[0]:.3f}, accepted {got_c[2]}, rejected {got_c[3]}")
        assert got_c == want_c, (r, got_c, want_c)
        for x, y in zip(got_q, want_q):
            assert np.array_equal(x, y), r


@pytest.mark.parametrize("n,ny,K", [(200, 150, 7), (1024, 1024, 10)])
def test_advance_graph_replays_match_eager(S, n, ny, K):
    b = I.basin(n, 2, ny=ny)
    g = S.Grid(n, ny, b.grid.dx, b.grid.dy)
    p = S.Params()
    B = torch.tensor(b.B, **F64)
    q0 = [torch.empty(ny, n, **F64) for _ in range(3)]
    S.swe_init(g, p, B, torch.tensor(b.eta0 * 20.0, **F64), q0)
    spd = torch.zeros(1, dtype=torch.int64, device="cuda")
    S.swe_max_speed(g, p, B, q0, 0, spd)
    dt0 = 1.2 * p.cfl_desired / float(spd.view(torch.float64).item())   # the first attempt is rejected
    ea = [x.clone() for x in q0]
    eb = [torch.empty_like(x) for x in q0]
    ga = [x.clone() for x in q0]
    gb = [torch.empty_like(x) for x in q0]
    ctl_e, ctl_g = S.new_ctl(), S.new_ctl()
    S.swe_ctl_set(ctl_e, 0.0, dt0, 1.0e30, 0)
    S.swe_ctl_set(ctl_g, 0.0, dt0, 1.0e30, 0)
    torch.cuda.synchronize()
    check_replays(S, lambda: S.swe_advance(g, p, B, ea, eb, ctl_e, K),
                  lambda st: S.swe_advance(g, p, B, ga, gb, ctl_g, K, stream=st),
                  ctl_e, ctl_g, ea, eb, ga, gb)
    assert S.read_ctl(ctl_g).s.n_rejected >= 1


@pytest.mark.parametrize("persistent", [0, 1])
def test_level_graph_replays_match_eager(S, persistent):
    """The level's advance of 5 attempts in 16-row chunks, one launch per
    attempt or one persistent (cooperative) launch, captured once."""
    ps = I.patches(200, seed=4)
    tab, ncell = S.patch_table(ps.nx, ps.ny, ps.dx)
    B = torch.tensor(np.concatenate([x.ravel() for x in ps.B]), **F64)
    eta = torch.tensor(np.concatenate([x.ravel() for x in ps.eta0]), **F64) * 20.0
    p = S.Params()
    q0 = [torch.empty(ncell, **F64) for _ in range(3)]
    spd = torch.zeros(1, dtype=torch.int64, device="cuda")
    for k in range(len(tab)):
        o, m = tab[k].offset, tab[k].nx * tab[k].ny
        gk = S.Grid(tab[k].nx, tab[k].ny, tab[k].dx, tab[k].dy)
        qk = [x[o:o + m] for x in q0]
        S.swe_init(gk, p, B[o:o + m], eta[o:o + m], qk)
        S.swe_max_speed(gk, p, B[o:o + m], qk, 0, spd)
    dt0 = p.cfl_desired / float(spd.view(torch.float64).item())
    lv = S.Level(tab, S.SCHED_PACKED, chunk_rows=16)
    ea = [x.clone() for x in q0]
    eb = [torch.empty_like(x) for x in q0]
    ga = [x.clone() for x in q0]
    gb = [torch.empty_like(x) for x in q0]
    ctl_e, ctl_g = S.new_ctl(), S.new_ctl()
    S.swe_ctl_set(ctl_e, 0.0, dt0, 1.0e30, 0)
    S.swe_ctl_set(ctl_g, 0.0, dt0, 1.0e30, 0)
    torch.cuda.synchronize()
    check_replays(S, lambda: S.level_advance(lv, p, B, ea, eb, ctl_e, 5, persistent),
                  lambda st: S.level_advance(lv, p, B, ga, gb, ctl_g, 5, persistent, stream=st),
                  ctl_e, ctl_g, ea, eb, ga, gb)
    assert int(lv.sync_t[2].item()) == 0


def test_advance_flagged_graph_replays_match_eager(S):
    """swe_advance_flagged captured once (7 attempts, a flag pass after every
    second accepted one, decided on the device from the control block): every
    replay leaves the state, control block and flag accumulators equal to
    those of the same attempts issued eagerly."""
    n, ny, K = 200, 150, 6
    b = I.basin(n, 3, ny=ny)
    g = S.Grid(n, ny, b.grid.dx, b.grid.dy)
    p = S.Params()
    B = torch.tensor(b.B, **F64)
    q0 = [torch.empty(ny, n, **F64) for _ in range(3)]
    S.swe_init(g, p, B, torch.tensor(b.eta0 * 20.0, **F64), q0)
    spd = torch.zeros(1, dtype=torch.int64, device="cuda")
    S.swe_max_speed(g, p, B, q0, 0, spd)
    dt0 = p.cfl_desired / float(spd.view(torch.float64).item())
    rng = np.random.default_rng(8)
    frames = torch.tensor(rng.normal(0.0, 1e-2, (K + 1, 3, ny, n)), **F64)
    t0, ts, tf, tol = 0.0, 10.0 * dt0, 40.0 * dt0, 1e-2
    bufs = {}
    for side in ("e", "g"):
        bufs[side] = dict(a=[x.clone() for x in q0], b=[torch.empty_like(x) for x in q0], ctl=S.new_ctl(),
                          acc=torch.zeros(ny, n, dtype=torch.int8, device="cuda"),
                          macc=torch.zeros(ny, n, **F64))
        S.swe_ctl_set(bufs[side]["ctl"], 0.0, dt0, 1.0e30, 0)
    torch.cuda.synchronize()

    def run(side, stream=None):
        d = bufs[side]
        S.swe_advance_flagged(g, p, B, d["a"], d["b"], d["ctl"], 7, frames, K, 2, t0, ts, tf, tol,
                              flag_acc=d["acc"], maxip_acc=d["macc"], stream=stream)

    graph = capture(lambda st: run("g", st))
    scratch = torch.randn(1 << 16, **F64)
    for r in range(3):
        run("e")
        torch.cuda.synchronize()
        want_q, want_c = current(S, bufs["e"]["ctl"], bufs["e"]["a"], bufs["e"]["b"])
        graph.replay()
        scratch.mul_(1.0001).add_(float(r))
        torch.cuda.synchronize()
        got_q, got_c = current(S, bufs["g"]["ctl"], bufs["g"]["a"], bufs["g"]["b"])
        calls = (S.read_ctl(bufs["g"]["ctl"]).n_flag_calls, S.read_ctl(bufs["e"]["ctl"]).n_flag_calls)
        print(f"replay {r}: t = {got_c[0]:.3f}, accepted {got_c[2]}, flag passes {calls[0]}, "
              f"flagged {int(bufs['g']['acc'].sum().item())}")
        assert got_c == want_c and calls[0] == calls[1], r
        for x, y in zip(got_q, want_q):
            assert np.array_equal(x, y), r
        assert torch.equal(bufs["g"]["acc"], bufs["e"]["acc"]), r
        assert torch.equal(bufs["g"]["macc"], bufs["e"]["macc"]), r
    assert calls[0] >= 6 and bufs["g"]["acc"].any()


def test_adjoint_steps_graph_replays_match_eager(S):
    """Six adjoint steps (ping-pong between two plane sets) captured once:
    every replay, restarted from the same target data with eager work in
    between, equals the same steps issued eagerly, bit for bit."""
    n, ny = 300, 200
    b = I.basin(n, 3, ny=ny)
    g = S.Grid(n, ny, b.grid.dx, b.grid.dy)
    p = S.Params()
    B = torch.tensor(b.B, **F64)
    phi = [torch.zeros(ny, n, **F64) for _ in range(3)]
    S.adj_target(g, p, B, b.target[0], b.target[1], 60e3, S.GAUSS, phi)
    ea, eb = [x.clone() for x in phi], [torch.empty_like(x) for x in phi]
    ga, gb = [x.clone() for x in phi], [torch.empty_like(x) for x in phi]
    # a Courant number of 0.8 at the deepest cell
    dt = 0.8 * min(b.grid.dx, b.grid.dy) / float(np.sqrt(9.81 * max(-b.B.min(), 1.0)))

    def steps(a, bb, stream=None):
        for k in range(6):
            src, dst = (a, bb) if k % 2 == 0 else (bb, a)
            S.adj_step(g, p, B, src, dst, dt, stream=stream)

    graph = capture(lambda st: steps(ga, gb, st))
    scratch = torch.randn(1 << 16, **F64)
    for r in range(3):
        for x, y, z in zip(ea, ga, phi):
            x.copy_(z)
            y.copy_(z)
        steps(ea, eb)
        torch.cuda.synchronize()
        graph.replay()
        scratch.mul_(1.0001).add_(float(r))
        torch.cuda.synchronize()
        for x, y in zip(ga, ea):
            assert torch.equal(x, y), r
    assert bool(torch.isfinite(ea[0]).all()) and not torch.equal(ea[0], phi[0])
