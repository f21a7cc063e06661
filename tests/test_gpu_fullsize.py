"""GPU parity at the full sizes of the benchmark workloads, through the C ABI:

* the 1D shelf (2000 cells, 3 h, 60 snapshot intervals, flags every step,
  tol 1e-3, the whole run as target window);
* the 512^2 adjoint-flagged basin run (64 snapshot intervals, target window
  [3600, 7200] s, tol 1e-4, flags every step): all 65 flag grids at the
  output times, the snapshots and the final state;
* the 1024^2 nonlinear step, 2000 device-controlled attempts replayed from
  HIP graphs of 100 attempts (the headline benchmark's launch configuration),
  against the oracle's run stored in tests/golden/step_nl_1024_2000.json
  (written by tests/golden/make_step_nl_1024_2000.py, which calls only the
  oracle): a hash of every element of the final state, 1024 sampled cells to
  1e-12, and the step counts and times;
* the 3000-patch batched level (10 attempts of the level-wide control rule),
  patch by patch.

Each flag grid is compared outside the band of cells whose max inner product
of the same flag pass lies within 1e-12 of the tolerance.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1605_05320_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"
REL = 1e-12
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "step_nl_1024_2000.json")


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


def close(a, b, scale=None):
    a, b = np.asarray(a), np.asarray(b)
    scale = np.abs(b).max() if scale is None else scale
    return np.abs(a - b).max() <= REL * max(scale, 1e-300)


def band_ok(fg, fc, m, tol):
    fg, fc, m = np.ravel(fg), np.ravel(fc), np.ravel(m)
    band = np.abs(m - tol) <= 1e-12 * tol
    return np.array_equal(fg[~band], fc[~band]), int(band.sum())


def run_gpu(S, gs, model, B, eta0, target, t0, ts, tf, K, tol, flag_every=1):
    ncomp = 3 if gs.ny > 1 else 2
    ny, nx = gs.ny, gs.nx
    frames = torch.zeros(K + 1, ncomp, ny, nx, dtype=torch.float64, device=DEV)
    q_out = [torch.zeros(ny, nx, dtype=torch.float64, device=DEV) for _ in range(ncomp)]
    flags_at = torch.full((K + 1, ny, nx), 7, dtype=torch.int8, device=DEV)
    acc = torch.zeros(ny, nx, dtype=torch.int8, device=DEV)
    macc = torch.zeros(ny, nx, dtype=torch.float64, device=DEV)
    pb = S.make_problem(gs, S.Params(model=model), dev(B.reshape(ny, nx)), dev(eta0.reshape(ny, nx)), target,
                        t0, ts, tf, K, tol, frames, q_out, flags_at, acc, macc, flag_every=flag_every)
    ws = torch.empty(S.swe_run_workspace_bytes(pb) // 8 + 64, dtype=torch.float64, device=DEV)
    res = S.swe_run(pb, ws)
    return res, host(frames), [host(x) for x in q_out], host(flags_at), host(acc), host(macc)


def check_run(rc, res, frames, q, flags_at, acc, macc, tol, B=None):
    assert res.n_sub == rc.n_sub and res.n_adj_steps == rc.n_adj_steps
    assert res.n_fwd_steps == rc.n_fwd_steps and res.n_rejected == rc.n_rejected
    assert res.n_flag_calls == rc.n_flag_calls and res.t_end == rc.t_end
    assert close(frames, rc.frames)
    if B is not None:
        assert close(q[0] + B, rc.q[0] + B, np.abs(rc.q[0] + B).max() + 1.0)
        others = list(zip(q[1:], rc.q[1:]))
    else:
        others = list(zip(q, rc.q))
    for x, y in others:
        assert close(x, y)
    assert close(macc, rc.maxip_acc)
    ok, nb = band_ok(acc, rc.flag_acc, rc.maxip_acc, tol)
    assert ok
    n_band = nb
    for j in range(rc.flags_at.shape[0]):
        ok, nb = band_ok(flags_at[j], rc.flags_at[j], rc.maxip_at[j], tol)
        assert ok, f"flags at output {j}"
        n_band += nb
    exact = (np.array_equal(frames, rc.frames) and all(np.array_equal(x, y) for x, y in zip(q, rc.q))
             and np.array_equal(flags_at, rc.flags_at) and np.array_equal(macc, rc.maxip_acc))
    return exact, n_band


def test_full_1d_shelf_run(oracle, S):
    """2000 cells on [-400, 0] km, T = 3 h, K = 60 (n_sub = 199), flags every
    step over the whole run (ts = t0), tol 1e-3."""
    O = oracle
    s = I.shelf1d(2000, seed=0)
    print("1D shelf: 2000 cells, T = 10800 s, K = 60", flush=True)
    go = O.Grid(2000, 1, s.dx, 1.0, s.x_lo)
    gs = S.Grid(2000, 1, s.dx, 1.0, s.x_lo)
    rc = O.run(go, O.Params(), O.LINEAR, s.B, s.eta0, s.target, 0.0, 0.0, 10800.0, 60, 1e-3)
    assert rc.n_sub == 199
    res, frames, q, flags_at, acc, macc = run_gpu(S, gs, S.LINEAR, s.B, s.eta0, s.target, 0.0, 0.0, 10800.0,
                                                  60, 1e-3)
    exact, nb = check_run(rc, res, frames.reshape(rc.frames.shape), [x.ravel() for x in q],
                          flags_at.reshape(rc.flags_at.shape), acc.ravel(), macc.ravel(), 1e-3)
    print(f"1D shelf: {res.n_fwd_steps} forward steps, {res.n_flag_calls} flag passes, "
          f"{int(rc.flag_acc.sum())} cells flagged, band cells {nb}, bit-exact={exact}")
    # over the whole 3 h window every cell gets flagged at some time, but not at every output time
    assert rc.flag_acc.any() and not rc.flags_at.all()


@pytest.mark.timeout(600)
def test_full_512_adjoint_flagged_run(oracle, S):
    """The 512^2 basin (seed 3, 2 km cells): adjoint from the Gaussian target
    (R = 20 km) with 64 snapshot intervals (n_sub = 13), forward run with
    flags every step in the window [3600, 7200] s, tol 1e-4."""
    O = oracle
    n, K, tol = 512, 64, 1e-4
    b = I.basin(n, 3)
    print("512^2 adjoint-flagged run: K = 64, window [3600, 7200] s, tol 1e-4", flush=True)
    go = O.Grid(n, n, b.grid.dx, b.grid.dy)
    gs = S.Grid(n, n, b.grid.dx, b.grid.dy)
    res, frames, q, flags_at, acc, macc = run_gpu(S, gs, S.NONLINEAR, b.B, b.eta0, b.target, 0.0, 3600.0,
                                                  7200.0, K, tol)
    rc = O.run(go, O.Params(), O.NONLINEAR, b.B, b.eta0, b.target, 0.0, 3600.0, 7200.0, K, tol)
    assert rc.n_sub == 13 and rc.status == 0
    exact, nb = check_run(rc, res, frames, q, flags_at, acc, macc, tol, B=b.B)
    per_out = [int(f.sum()) for f in rc.flags_at]
    print(f"512^2: {res.n_adj_steps} adjoint + {res.n_fwd_steps} forward steps, {res.n_flag_calls} flag "
          f"passes, flagged cells at output times {per_out[::8]}, band cells {nb}, bit-exact={exact}")
    assert any(per_out) and rc.flag_acc.any()


def test_full_1024_step_2000_attempts_graph_replays(S):
    """The headline workload: 2000 device-controlled step attempts on the
    1024^2 basin (seed 2) from its initial state, as 20 replays of a HIP graph
    of 100 attempts."""
    with open(GOLDEN) as f:
        gold = json.load(f)
    n = 1024
    b = I.basin(n, 2)
    print("1024^2 step: 2000 controlled attempts in 20 graph replays", flush=True)
    grid = S.Grid(n, n, b.grid.dx, b.grid.dy)
    prm = S.Params()
    B = dev(b.B)
    qa = [torch.empty(n, n, dtype=torch.float64, device=DEV) for _ in range(3)]
    qb = [torch.empty(n, n, dtype=torch.float64, device=DEV) for _ in range(3)]
    S.swe_init(grid, prm, B, dev(b.eta0), qa)
    spd = torch.zeros(1, dtype=torch.int64, device=DEV)
    S.swe_max_speed(grid, prm, B, qa, 0, spd)
    dt0 = prm.cfl_desired / float(spd.view(torch.float64).item())
    ctl = S.new_ctl()
    S.swe_ctl_set(ctl, 0.0, dt0, 1.0e30, 0)
    stream = torch.cuda.current_stream()
    gs = torch.cuda.Stream()
    gs.wait_stream(stream)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(gs):
        with torch.cuda.graph(graph, stream=gs):
            S.swe_advance(grid, prm, B, qa, qb, ctl, 100, stream=gs)
    stream.wait_stream(gs)
    torch.cuda.synchronize()
    for _ in range(20):
        graph.replay()
    torch.cuda.synchronize()
    c = S.read_ctl(ctl)
    cur = qa if c.s.cur == 0 else qb
    got = [host(x) for x in cur]
    assert (c.s.n_accepted, c.s.n_rejected) == (gold["accepted"], gold["rejected"])
    assert c.s.t == float.fromhex(gold["t"]) and c.s.dt == float.fromhex(gold["dt_next"])
    smp = gold["samples"]
    jj, ii = np.array(smp["j"]), np.array(smp["i"])
    for comp in range(3):
        want = np.array([float.fromhex(v) for v in smp["values"][comp]])
        have = got[comp][jj, ii]
        if comp == 0:
            want, have = want + b.B[jj, ii], have + b.B[jj, ii]
            scale = float.fromhex(gold["max_abs_eta"]) + 1.0
        else:
            scale = float.fromhex(gold["max_abs"][comp])
        assert np.abs(have - want).max() <= REL * scale, comp
    hashes = [hashlib.sha256(np.ascontiguousarray(x, dtype="<f8").tobytes()).hexdigest() for x in got]
    print(f"1024^2: {c.s.n_accepted} accepted, {c.s.n_rejected} rejected, t = {c.s.t:.3f} s, "
          f"every element equal to the oracle's: {hashes == gold['sha256']}")
    assert hashes == gold["sha256"]


def _oracle_level(O, ps, q, dt, n_steps, cfl_d=0.9, cfl_max=1.0):
    """The level-wide control rule over the oracle's patch steps (no output time)."""
    p = O.Params(cfl_desired=cfl_d, cfl_max=cfl_max)
    t, acc, rej = 0.0, 0, 0
    grids = [O.Grid(int(ps.nx[k]), int(ps.ny[k]), ps.dx[k], ps.dx[k]) for k in range(len(ps.nx))]
    for _ in range(n_steps):
        new, cfl = [], 0.0
        for k, g in enumerate(grids):
            h, hu, hv, c, _ = O.swe_step(g, p, ps.B[k], *q[k], dt)
            new.append([h, hu, hv])
            cfl = max(cfl, c)
        if cfl > cfl_max:
            rej += 1
            dt = dt * cfl_d / cfl
        else:
            acc += 1
            q = new
            t = t + dt
            dt = dt * cfl_d / cfl
    return q, t, dt, acc, rej


@pytest.mark.timeout(300)
@pytest.mark.parametrize("kind,chunk,persistent", [(1, 16, 0), (1, 0, 1), (1, 16, 1)])
def test_full_level_3000_patches(oracle, S, kind, chunk, persistent):
    """The benchmark's level (3000 patches of 8..64 cells a side, seed 4): the
    packed schedule in 16-row chunks with one launch per attempt and with one
    persistent launch (more jobs than resident wavefronts), and the persistent
    launch of whole packed patches, 10 attempts, every patch."""
    O = oracle
    ps = I.patches(3000, seed=4)
    print(f"3000-patch level: kind={kind} chunk={chunk} persistent={persistent}", flush=True)
    q0, dts = [], []
    for k in range(len(ps.nx)):
        g = O.Grid(int(ps.nx[k]), int(ps.ny[k]), ps.dx[k], ps.dx[k])
        qk = O.init_state(g, O.Params(), O.NONLINEAR, ps.B[k], ps.eta0[k])
        q0.append(qk)
        d = O.dt0(g, O.Params(), O.NONLINEAR, ps.B[k], *qk)
        if d > 0:
            dts.append(d)
    dt0 = min(dts)
    O.set_threads(1)            # 3000 tiny grids: one thread each is fastest
    try:
        qc, t, dt, acc, rej = _oracle_level(O, ps, q0, dt0, 10)
    finally:
        O.set_threads(os.cpu_count() or 1)
    tab, ncell = S.patch_table(ps.nx, ps.ny, ps.dx)
    lvl = S.Level(tab, kind, chunk_rows=chunk)
    Bd = dev(np.concatenate([x.ravel() for x in ps.B]))
    a = [dev(np.concatenate([qq[c].ravel() for qq in q0])) for c in range(3)]
    bb = [torch.full_like(x, float("nan")) for x in a]
    ctl = S.new_ctl()
    S.swe_ctl_set(ctl, 0.0, dt0, 1.0e300, 0)
    S.level_advance(lvl, S.Params(), Bd, a, bb, ctl, 10, persistent)
    torch.cuda.synchronize()
    assert int(lvl.sync_t[2].item()) == 0
    c = S.read_ctl(ctl)
    assert (c.n_accepted, c.n_rejected, c.t, c.dt) == (acc, rej, t, dt)
    got = [host(x) for x in (a if c.cur == 0 else bb)]
    off, exact = 0, True
    for k in range(len(ps.nx)):
        m = int(ps.nx[k]) * int(ps.ny[k])
        for comp in range(3):
            g_ = got[comp][off:off + m].reshape(qc[k][comp].shape)
            r_ = qc[k][comp]
            if comp == 0:
                g_, r_ = g_ + ps.B[k], r_ + ps.B[k]
            scale = np.abs(r_).max() + (1.0 if comp == 0 else 0.0)
            assert np.abs(g_ - r_).max() <= REL * max(scale, 1e-300), (k, comp)
            exact &= np.array_equal(got[comp][off:off + m], qc[k][comp].ravel())
        off += m
    print(f"3000-patch level: {acc} accepted, {rej} rejected, bit-exact={exact}")
