"""Serving through swe_serve: a scenario's results are identical whether it
runs alone or in a mix with others in flight; they match the oracle's run
(a 1D request beside 2D ones too); admission never exceeds the arena or the
slot count; a request larger than
the arena is refused without blocking the rest; realtime admission waits
for each arrival; and a request that fails (a non-finite state) leaves the
others' results as they are alone."""
import numpy as np
import pytest

from paper_1605_05320_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL = 1e-12
K, T0, TS, TF, TOL, FLAG_EVERY, R_TARGET = 8, 0.0, 1800.0, 3600.0, 1e-4, 2, 60e3


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_05320_amd import swe
    swe.lib()
    return swe


def make_request(S, n, seed, arrival=0.0):
    b = I.basin(n, seed)
    g = S.Grid(b.grid.nx, b.grid.ny, b.grid.dx, b.grid.dy, b.grid.x_lo, b.grid.y_lo)
    target = (b.target[0], b.target[1], R_TARGET)
    print(f"request n={n} seed={seed} arrival={arrival:.3f}", flush=True)
    return S.Request(g, S.Params(), b.B, b.eta0, target, T0, TS, TF, K, TOL, flag_every=FLAG_EVERY,
                     arrival=arrival), b


def outputs(r):
    return [r.flag_acc.copy(), r.maxip_acc.copy()] + [q.copy() for q in r.q]


def arena_for(S, reqs, copies=1):
    nbytes = max(S.serve_footprint(r) for r in reqs) * copies
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def trace(S, n_req=8, nmin=48, nmax=128):
    return [make_request(S, a.n, a.seed)[0] for a in I.arrivals(n_req, 50.0, nmin, nmax, seed=5)]


def test_mix_equals_alone(S):
    reqs = trace(S)
    alone = []
    for r in reqs:
        arena = arena_for(S, [r])
        _, st = S.serve([r], arena, 1)
        assert st[0]["status"] == 0
        alone.append((outputs(r), st[0]))
        r.flag_acc[:] = 0
        r.maxip_acc[:] = 0
        for q in r.q:
            q[:] = 0
    arena = arena_for(S, reqs, copies=4)
    _, st = S.serve(reqs, arena, 4)
    slots = {s["slot"] for s in st}
    assert len(slots) > 1, "the mix never used two slots"
    # at least two requests were in flight together: their admitted..finished
    # intervals overlap (the mix really ran side by side)
    spans = sorted((s["admitted"], s["finished"]) for s in st)
    overlaps = sum(1 for k in range(len(spans)) for m in range(k + 1, len(spans))
                   if spans[m][0] < spans[k][1] and spans[k][0] < spans[m][1])
    print(f"mix: {len(slots)} slots, {overlaps} overlapping pairs of requests")
    assert overlaps >= 1, "no two requests were in flight at the same time"
    for r, s, (ref, s1) in zip(reqs, st, alone):
        assert s["status"] == 0
        assert s["n_fwd_steps"] == s1["n_fwd_steps"] and s["n_adj_steps"] == s1["n_adj_steps"]
        for x, y in zip(outputs(r), ref):
            assert np.array_equal(x, y)
    assert any(r.flag_acc.any() for r in reqs)


def test_served_matches_oracle(oracle, S):
    O = oracle
    for n, seed in [(64, 1001), (77, 1002)]:
        r, b = make_request(S, n, seed)
        arena = arena_for(S, [r])
        _, st = S.serve([r], arena, 1)
        go = O.Grid(n, n, b.grid.dx, b.grid.dy, b.grid.x_lo, b.grid.y_lo, (0, 0, 0, 0))
        rc = O.run(go, O.Params(), O.NONLINEAR, b.B, b.eta0, (b.target[0], b.target[1], R_TARGET),
                   T0, TS, TF, K, TOL, flag_every=FLAG_EVERY)
        assert st[0]["n_fwd_steps"] == rc.n_fwd_steps and st[0]["n_adj_steps"] == rc.n_adj_steps
        eta_g, eta_c = r.q[0] + b.B, rc.q[0] + b.B
        assert np.abs(eta_g - eta_c).max() <= REL * (np.abs(eta_c).max() + 1.0)
        for c in (1, 2):
            assert np.abs(r.q[c] - rc.q[c]).max() <= REL * np.abs(rc.q[c]).max()
        assert np.abs(r.maxip_acc - rc.maxip_acc).max() <= REL * np.abs(rc.maxip_acc).max()
        band = np.abs(rc.maxip_acc - TOL) <= 1e-12 * TOL
        assert np.array_equal(r.flag_acc[~band], rc.flag_acc[~band])
        print(f"served {n}: bit-exact={all(np.array_equal(x, y) for x, y in zip(r.q, rc.q))}")


def test_admission_respects_arena_and_slots(S):
    reqs = trace(S, n_req=6, nmin=96, nmax=128)
    big, _ = make_request(S, 200, 77)
    reqs.insert(3, big)
    arena = arena_for(S, reqs[:3] + reqs[4:], copies=2)
    cap = arena.numel()
    assert S.serve_footprint(big) > cap
    rc, st = S.serve(reqs, arena, 3, check=False)
    assert rc == S.E_NOMEM
    assert st[3]["status"] == S.E_NOMEM and st[3]["slot"] == -1
    for k, s in enumerate(st):
        if k != 3:
            assert s["status"] == 0 and s["slot"] >= 0
    events = sorted({s["admitted"] for k, s in enumerate(st) if k != 3})
    for t in events:
        live = [s for k, s in enumerate(st) if k != 3 and s["admitted"] <= t < s["finished"]]
        assert sum(s["bytes"] for s in live) <= cap
        assert len(live) <= 3


def test_realtime_admission_waits_for_arrival(S):
    reqs = [make_request(S, 64, 1000 + k, arrival=0.15 * k)[0] for k in range(4)]
    arena = arena_for(S, reqs, copies=4)
    _, st = S.serve(reqs, arena, 4, realtime=True)
    for r, s in zip(reqs, st):
        assert s["status"] == 0
        assert s["admitted"] >= r.c.arrival
        assert abs(s["latency"] - (s["finished"] - r.c.arrival)) < 1e-9


def test_on_done_reports_every_request_once(S):
    import threading
    reqs = trace(S, n_req=6, nmin=48, nmax=96)
    arena = arena_for(S, reqs, copies=3)
    seen, lock = [], threading.Lock()

    def done(k):
        with lock:
            seen.append(k)

    _, st = S.serve(reqs, arena, 3, on_done=done)
    assert sorted(seen) == list(range(len(reqs)))
    # completion order: each report comes after that request finished
    fin = [st[k]["finished"] for k in seen]
    assert all(f > 0.0 for f in fin)


def test_shoreline_thin_layer_scenario_completes(S):
    """Basin seed 1114 on a 1414^2 grid with the serving workload's
    parameters: after ~1800 steps the drawdown at the shoreline wall leaves a
    millimetre-thin layer moving at hundreds of m/s.  With the cells' own
    speeds in the Courant number the time step shrinks while the layer drains
    and the run completes (with Roe edge speeds alone it blew up); a request
    served beside it completes as well."""
    import time
    b = I.basin(1414, 1114)
    g = S.Grid(1414, 1414, b.grid.dx, b.grid.dy)
    thin = S.Request(g, S.Params(), b.B, b.eta0, b.target, 0.0, 3600.0, 7200.0, 32, 1e-4, flag_every=4)
    good, _ = make_request(S, 96, 1003)
    arena = arena_for(S, [thin, good], copies=2)
    t = time.perf_counter()
    rc, st = S.serve([thin, good], arena, 2, check=False)
    el = time.perf_counter() - t
    print(f"thin-layer scenario: status {st[0]['status']}, {st[0]['n_fwd_steps']} forward steps, "
          f"{el:.1f} s; beside it: {st[1]['status']}")
    assert rc == 0 and st[0]["status"] == 0 and st[1]["status"] == 0
    assert st[0]["n_fwd_steps"] > 2000
    assert el < 60.0


def test_failing_request_leaves_the_mix_intact(S):
    """One request of a mix has a NaN in the initial surface of a wet cell:
    it ends with SWE_E_NONFINITE (the call returns that status), and every
    other request gives the results it gives alone."""
    arr = I.arrivals(6, 50.0, 48, 128, seed=7)
    reqs, alone = [], []
    for k, a in enumerate(arr):
        r, b = make_request(S, a.n, a.seed)
        if k == 2:
            eta0 = b.eta0.copy()
            j, i = np.argwhere(b.B < -100.0)[0]
            eta0[j, i] = np.nan
            g = S.Grid(b.grid.nx, b.grid.ny, b.grid.dx, b.grid.dy, b.grid.x_lo, b.grid.y_lo)
            r = S.Request(g, S.Params(), b.B, eta0, (b.target[0], b.target[1], R_TARGET), T0, TS, TF, K, TOL,
                          flag_every=FLAG_EVERY)
        else:
            _, st = S.serve([r], arena_for(S, [r]), 1)
            assert st[0]["status"] == 0
            alone.append(outputs(r))
            r.flag_acc[:] = 0
            r.maxip_acc[:] = 0
            for q in r.q:
                q[:] = 0
        reqs.append(r)
    rc, st = S.serve(reqs, arena_for(S, reqs, copies=3), 3, check=False)
    assert rc == S.E_NONFINITE and st[2]["status"] == S.E_NONFINITE
    good = [k for k in range(len(reqs)) if k != 2]
    for k, ref in zip(good, alone):
        assert st[k]["status"] == 0
        for x, y in zip(outputs(reqs[k]), ref):
            assert np.array_equal(x, y)
    print(f"mix with a failing request: {len(good)} others as alone")


def test_served_1d_request_beside_2d_matches_oracle(oracle, S):
    """A one-dimensional request (the 2000-cell shelf, linear model, 20
    snapshots over an hour) served beside two 2D basins: its results match
    the oracle's run, and the 2D requests give the results they give alone."""
    O = oracle
    n, K1, tf1, tol1 = 2000, 20, 3600.0, 1e-3
    s = I.shelf1d(n, seed=0)
    g1 = S.Grid(n, 1, s.dx, 1.0, s.x_lo)
    r1d = S.Request(g1, S.Params(model=S.LINEAR), s.B.reshape(1, n), s.eta0.reshape(1, n), s.target,
                    0.0, 0.0, tf1, K1, tol1)
    twod = [make_request(S, 64, 1010)[0], make_request(S, 96, 1011)[0]]
    alone = []
    for r in twod:
        _, st = S.serve([r], arena_for(S, [r]), 1)
        assert st[0]["status"] == 0
        alone.append(outputs(r))
        r.flag_acc[:] = 0
        r.maxip_acc[:] = 0
        for q in r.q:
            q[:] = 0
    reqs = [twod[0], r1d, twod[1]]
    rc_, st = S.serve(reqs, arena_for(S, reqs, copies=3), 3)
    assert all(x["status"] == 0 for x in st)
    for r, ref in zip(twod, alone):
        for x, y in zip(outputs(r), ref):
            assert np.array_equal(x, y)
    go = O.Grid(n, 1, s.dx, 1.0, s.x_lo, 0.0, (0, 0, 0, 0))
    rc = O.run(go, O.Params(), O.LINEAR, s.B, s.eta0, s.target, 0.0, 0.0, tf1, K1, tol1)
    assert st[1]["n_fwd_steps"] == rc.n_fwd_steps and st[1]["n_adj_steps"] == rc.n_adj_steps
    for c in (0, 1):
        ref = rc.q[c].ravel()
        assert np.abs(r1d.q[c].ravel() - ref).max() <= REL * np.abs(ref).max()
    macc = rc.maxip_acc.ravel()
    assert np.abs(r1d.maxip_acc.ravel() - macc).max() <= REL * np.abs(macc).max()
    band = np.abs(macc - tol1) <= 1e-12 * tol1
    assert np.array_equal(r1d.flag_acc.ravel()[~band], rc.flag_acc.ravel()[~band])
    assert rc.flag_acc.any()
    print(f"served 1D beside 2D: {st[1]['n_fwd_steps']} forward steps, "
          f"bit-exact={all(np.array_equal(r1d.q[c].ravel(), rc.q[c].ravel()) for c in (0, 1))}")
