"""GPU parity of the batched AMR level (both schedules, per-step and
persistent launches) against the oracle stepping each patch, with the
level-wide time step of the device-side control rule (rejection included)."""
import numpy as np
import pytest

from paper_1605_05320_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_05320_amd import swe
    swe.lib()
    return swe


def oracle_level(O, ps, B, q, dt, n_steps, cfl_d=0.9, cfl_max=1.0, t_out=1e30, bcs=None):
    """Host mirror of the control rule with the Courant number of the level
    (bcs: each patch's four boundary codes, walls if not given)."""
    p = O.Params(cfl_desired=cfl_d, cfl_max=cfl_max)
    t, fin, acc, rej = 0.0, False, 0, 0
    if dt >= t_out - t:
        dt, fin = t_out - t, True
    for _ in range(n_steps):
        new, cfl = [], 0.0
        for k in range(len(ps.nx)):
            g = O.Grid(int(ps.nx[k]), int(ps.ny[k]), ps.dx[k], ps.dx[k], 0.0, 0.0,
                       (0, 0, 0, 0) if bcs is None else tuple(bcs[k]))
            h, hu, hv, c, _ = O.swe_step(g, p, B[k], *q[k], dt)
            new.append([h, hu, hv])
            cfl = max(cfl, c)
        if cfl > cfl_max:
            rej += 1
            dt = dt * cfl_d / cfl
        else:
            acc += 1
            q = new
            t = t_out if fin else t + dt
            dt = dt * cfl_d / cfl
        fin = False
        if dt >= t_out - t:
            dt, fin = t_out - t, True
    return q, t, dt, acc, rej


@pytest.fixture(scope="module")
def setup(oracle):
    O = oracle
    ps = I.patches(48, seed=5)
    ps.nx[0], ps.ny[0] = 64, 37          # a patch of two strips
    ps.nx[1], ps.ny[1] = 61, 8
    ps = I.PatchSet(nx=ps.nx, ny=ps.ny, dx=ps.dx, x_lo=ps.x_lo, y_lo=ps.y_lo, B=None, eta0=None)
    bp = I.basin_params(5)
    B, q = [], []
    for k in range(len(ps.nx)):
        g = I.Grid2D(int(ps.nx[k]), int(ps.ny[k]), ps.dx[k], ps.dx[k], ps.x_lo[k], ps.y_lo[k])
        X, Y = g.centres()
        b = I.bathymetry(X, Y, bp)
        e = 30.0 * I.source_surface(X, Y, bp) + 0.2 * np.sin(X / 3e3) * np.cos(Y / 4e3)
        B.append(b)
        og = O.Grid(g.nx, g.ny, g.dx, g.dy)
        qk = O.init_state(og, O.Params(), O.NONLINEAR, b, e)
        if k in (2, 5):
            # a supercritical jet through the middle rows of two patches
            r0, r1 = g.ny // 3, max(g.ny // 3 + 1, 2 * g.ny // 3)
            h = qk[0][r0:r1]
            qk[1][r0:r1] = np.where(h > 1e-3, 2.5 * h * np.sqrt(9.81 * h), 0.0)
        q.append(qk)
    dts = [O.dt0(O.Grid(int(ps.nx[k]), int(ps.ny[k]), ps.dx[k], ps.dx[k]), O.Params(), O.NONLINEAR, B[k], *q[k])
           for k in range(len(ps.nx))]
    return ps, B, q, min(d for d in dts if d > 0)


def to_arena(arrs):
    return np.concatenate([a.ravel() for a in arrs])


@pytest.mark.parametrize("kind,persistent,chunk", [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (1, 0, 16),
                                                    (1, 0, 12), (0, 0, 9), (1, 0, 1), (1, 1, 16), (0, 1, 9),
                                                    (1, 1, 1)])
def test_level_parity(oracle, S, setup, kind, persistent, chunk):
    ps, B, q, dt0 = setup
    n_steps = 7
    qc, t, dt, acc, rej = oracle_level(oracle, ps, B, q, 1.6 * dt0, n_steps)
    assert rej >= 1 and acc >= 1
    tab, ncell = S.patch_table(ps.nx, ps.ny, ps.dx)
    lvl = S.Level(tab, kind, chunk_rows=chunk)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    Bd = dev(to_arena(B))
    a = [dev(to_arena([qq[c] for qq in q])) for c in range(3)]
    b = [torch.full_like(x, float("nan")) for x in a]
    ctl = S.new_ctl()
    S.swe_ctl_set(ctl, 0.0, 1.6 * dt0, 1e30, 0)
    S.level_advance(lvl, S.Params(), Bd, a, b, ctl, n_steps, persistent)
    torch.cuda.synchronize()
    assert int(lvl.sync_t[2].item()) == 0
    c = S.read_ctl(ctl)
    assert (c.n_accepted, c.n_rejected, c.t, c.dt) == (acc, rej, t, dt)
    cur = a if c.cur == 0 else b
    got = [x.cpu().numpy() for x in cur]
    off = 0
    exact = True
    for k in range(len(ps.nx)):
        n = int(ps.nx[k]) * int(ps.ny[k])
        for comp in range(3):
            g_ = got[comp][off:off + n].reshape(qc[k][comp].shape)
            r_ = qc[k][comp]
            if comp == 0:
                g_, r_ = g_ + B[k], r_ + B[k]
            scale = np.abs(r_).max() + (1.0 if comp == 0 else 0.0)
            assert np.abs(g_ - r_).max() <= 1e-12 * max(scale, 1e-300), (k, comp)
            exact &= np.array_equal(got[comp][off:off + n], qc[k][comp].ravel())
        off += n
    print(f"level kind={kind} persistent={persistent} chunk={chunk}: bit-exact={exact}")


@pytest.mark.parametrize("persistent,chunk", [(0, 0), (1, 16), (0, 3)])
def test_level_parity_mixed_boundaries(oracle, S, setup, persistent, chunk):
    """Each patch with its own mix of walls and extrapolating sides (the
    level keeps them per lane as one bit word), against the oracle stepping
    each patch with its own boundary conditions."""
    ps, B, q, dt0 = setup
    rng = np.random.default_rng(17)
    bcs = [tuple(int(v) for v in rng.integers(0, 2, 4)) for _ in range(len(ps.nx))]
    assert len(set(bcs)) > 4
    n_steps = 5
    qc, t, dt, acc, rej = oracle_level(oracle, ps, B, q, 1.6 * dt0, n_steps, bcs=bcs)
    assert rej >= 1 and acc >= 1
    tab, ncell = S.patch_table(ps.nx, ps.ny, ps.dx)
    for k, bc in enumerate(bcs):
        for side in range(4):
            tab[k].bc[side] = bc[side]
    lvl = S.Level(tab, S.SCHED_PACKED, chunk_rows=chunk)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    Bd = dev(to_arena(B))
    a = [dev(to_arena([qq[c] for qq in q])) for c in range(3)]
    b = [torch.full_like(x, float("nan")) for x in a]
    ctl = S.new_ctl()
    S.swe_ctl_set(ctl, 0.0, 1.6 * dt0, 1e30, 0)
    S.level_advance(lvl, S.Params(), Bd, a, b, ctl, n_steps, persistent)
    torch.cuda.synchronize()
    assert int(lvl.sync_t[2].item()) == 0
    c = S.read_ctl(ctl)
    assert (c.n_accepted, c.n_rejected, c.t, c.dt) == (acc, rej, t, dt)
    got = [x.cpu().numpy() for x in (a if c.cur == 0 else b)]
    off, exact = 0, True
    for k in range(len(ps.nx)):
        n = int(ps.nx[k]) * int(ps.ny[k])
        for comp in range(3):
            g_ = got[comp][off:off + n].reshape(qc[k][comp].shape)
            r_ = qc[k][comp]
            if comp == 0:
                g_, r_ = g_ + B[k], r_ + B[k]
            scale = np.abs(r_).max() + (1.0 if comp == 0 else 0.0)
            assert np.abs(g_ - r_).max() <= 1e-12 * max(scale, 1e-300), (k, comp, bcs[k])
            exact &= np.array_equal(got[comp][off:off + n], qc[k][comp].ravel())
        off += n
    print(f"level mixed boundaries persistent={persistent} chunk={chunk}: bit-exact={exact}")


@pytest.mark.parametrize("chunk", [2, 5])
def test_persistent_row_chunks_match_per_step(S, setup, chunk):
    """Row chunks of one patch on different wavefronts of the persistent
    launch: the halo rows each chunk reads were stored by other wavefronts in
    the previous attempt.  The result equals the launch-per-step run of the
    same schedule bit for bit, with the same accepted and rejected attempts."""
    ps, B, q, dt0 = setup
    tab, ncell = S.patch_table(ps.nx, ps.ny, ps.dx)
    lvl = S.Level(tab, 1, chunk_rows=chunk)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    Bd = dev(to_arena(B))
    res = []
    for persistent in (0, 1):
        a = [dev(to_arena([qq[c] for qq in q])) for c in range(3)]
        b = [torch.full_like(x, float("nan")) for x in a]
        ctl = S.new_ctl()
        S.swe_ctl_set(ctl, 0.0, 1.6 * dt0, 1e30, 0)
        S.level_advance(lvl, S.Params(), Bd, a, b, ctl, 9, persistent)
        torch.cuda.synchronize()
        assert int(lvl.sync_t[2].item()) == 0
        c = S.read_ctl(ctl)
        res.append(((c.n_accepted, c.n_rejected, c.t, c.dt), [x.cpu().numpy() for x in (a if c.cur == 0 else b)]))
    assert res[0][0] == res[1][0] and res[0][0][1] >= 1
    for x, y in zip(res[0][1], res[1][1]):
        assert np.array_equal(x.view(np.int64), y.view(np.int64))
    print(f"chunk={chunk}: {lvl.c.n_jobs} jobs, persistent equals per-step")

@pytest.mark.parametrize("seed,n,kind,chunk", [(11, 3, 1, 0), (12, 5, 0, 4), (13, 120, 1, 7), (14, 400, 0, 16),
                                               (15, 400, 1, 3)])
def test_persistent_random_levels_match_per_step(oracle, S, seed, n, kind, chunk):
    """Random patch sets (from a single workgroup with idle wavefronts to
    more passes than resident wavefronts), both schedules, whole patches and
    row chunks, waves on every wet cell and a first dt that gets rejected:
    the persistent launch equals the launch per attempt bit for bit."""
    O = oracle
    ps = I.patches(n, seed=seed)
    rng = np.random.default_rng(seed)
    q, dts = [], []
    for k in range(n):
        g = O.Grid(int(ps.nx[k]), int(ps.ny[k]), ps.dx[k], ps.dx[k])
        e = 20.0 * ps.eta0[k] + rng.uniform(-0.05, 0.05, ps.B[k].shape)
        qk = O.init_state(g, O.Params(), O.NONLINEAR, ps.B[k], e)
        q.append(qk)
        d = O.dt0(g, O.Params(), O.NONLINEAR, ps.B[k], *qk)
        if d > 0:
            dts.append(d)
    dt0 = 1.6 * min(dts)
    tab, ncell = S.patch_table(ps.nx, ps.ny, ps.dx)
    lvl = S.Level(tab, kind, chunk_rows=chunk)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    Bd = dev(to_arena(ps.B))
    res = []
    for persistent in (0, 1):
        a = [dev(to_arena([qq[c] for qq in q])) for c in range(3)]
        b = [torch.full_like(x, float("nan")) for x in a]
        ctl = S.new_ctl()
        S.swe_ctl_set(ctl, 0.0, dt0, 1e30, 0)
        S.level_advance(lvl, S.Params(), Bd, a, b, ctl, 8, persistent)
        torch.cuda.synchronize()
        assert int(lvl.sync_t[2].item()) == 0
        c = S.read_ctl(ctl)
        res.append(((c.n_accepted, c.n_rejected, c.t, c.dt, c.n_clamped, c.n_nonfinite),
                    [x.cpu().numpy() for x in (a if c.cur == 0 else b)]))
    assert res[0][0] == res[1][0] and res[0][0][1] >= 1 and res[0][0][0] >= 1
    for x, y in zip(res[0][1], res[1][1]):
        assert np.array_equal(x.view(np.int64), y.view(np.int64))
    print(f"seed={seed}: {n} patches, {lvl.c.n_passes} passes, persistent equals per-step")


def _shoreline_patch(seed, nx=70, ny=24):
    """2 m of water west, a thin layer (2..20 mm) draining westward from a dry
    beach east of column 40: large steps drive some of its cells below zero."""
    rng = np.random.default_rng(seed)
    B = np.full((ny, nx), -2.0)
    B[:, 40:] = 1.0
    h = np.maximum(0.0, -B)
    h[:, 30:40] = rng.uniform(0.002, 0.02, (ny, 10))
    B[:, 30:40] = -h[:, 30:40]
    hu = np.zeros_like(h)
    hv = np.zeros_like(h)
    hu[:, 30:40] = -h[:, 30:40] * rng.uniform(0.5, 3.0, (ny, 10))
    hv[:, 30:40] = h[:, 30:40] * rng.uniform(-1.0, 1.0, (ny, 10))
    return B, [h, hu, hv]


@pytest.mark.parametrize("kind,chunk", [(1, 0), (1, 8), (0, 5)])
def test_level_counts_clamps_of_accepted_attempts(oracle, S, kind, chunk):
    """Three shoreline patches under the level's control rule (desired Courant
    number 1.2, rejected above 1.25): clamped cells are counted for the
    accepted attempts only, as the oracle stepping each patch counts them,
    with the launch per attempt and with the persistent launch (whose
    workgroups add their wavefronts' counts before one set of atomics); the
    states equal the oracle's bit for bit."""
    O = oracle
    pats = [_shoreline_patch(s) for s in (3, 4, 5)]
    po = O.Params(cfl_desired=1.2, cfl_max=1.25)
    grid = O.Grid(70, 24, 10.0, 10.0)
    q = [list(p[1]) for p in pats]
    dt, t, acc, rej, ncl_acc, ncl_rej = 4.0, 0.0, 0, 0, 0, 0
    for _ in range(12):
        new, cfl, ncl = [], 0.0, 0
        for (B, _), qk in zip(pats, q):
            h, hu, hv, c, n = O.swe_step(grid, po, B, *qk, dt)
            new.append([h, hu, hv])
            cfl, ncl = max(cfl, c), ncl + n
        if cfl > po.cfl_max:
            rej, ncl_rej = rej + 1, ncl_rej + ncl
            dt = dt * po.cfl_desired / cfl
        else:
            acc, ncl_acc = acc + 1, ncl_acc + ncl
            q, t = new, t + dt
            if cfl > 0.0:
                dt = dt * po.cfl_desired / cfl
    assert rej >= 1 and ncl_acc >= 1 and ncl_rej >= 1
    tab, ncell = S.patch_table([70] * 3, [24] * 3, [10.0] * 3)
    lvl = S.Level(tab, kind, chunk_rows=chunk)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    Bd = dev(to_arena([p[0] for p in pats]))
    ps = S.Params(cfl_desired=1.2, cfl_max=1.25)
    for persistent in (0, 1):
        a = [dev(to_arena([p[1][c] for p in pats])) for c in range(3)]
        b = [torch.full_like(x, float("nan")) for x in a]
        ctl = S.new_ctl()
        S.swe_ctl_set(ctl, 0.0, 4.0, 1.0e30, 0)
        S.level_advance(lvl, ps, Bd, a, b, ctl, 12, persistent)
        torch.cuda.synchronize()
        assert int(lvl.sync_t[2].item()) == 0
        c = S.read_ctl(ctl)
        assert (c.n_accepted, c.n_rejected, c.t, c.dt) == (acc, rej, t, dt)
        assert c.n_clamped == ncl_acc and c.n_nonfinite == 0, (persistent, c.n_clamped, ncl_acc)
        cur = a if c.cur == 0 else b
        for comp in range(3):
            assert np.array_equal(cur[comp].cpu().numpy(), to_arena([qk[comp] for qk in q]))
    print(f"level clamp count: {ncl_acc} (accepted attempts), {ncl_rej} in rejected ones not counted")


def _tuner_setup(S, n=200, seed=4):
    F64 = dict(dtype=torch.float64, device="cuda")
    ps = I.patches(n, seed=seed)
    tab, ncell = S.patch_table(ps.nx, ps.ny, ps.dx)
    B = torch.tensor(np.concatenate([x.ravel() for x in ps.B]), **F64)
    eta = torch.tensor(np.concatenate([x.ravel() for x in ps.eta0]), **F64) * 20.0
    p = S.Params()
    init = [torch.empty(ncell, **F64) for _ in range(3)]
    spd = torch.zeros(1, dtype=torch.int64, device="cuda")
    for k in range(len(tab)):
        o, m = tab[k].offset, tab[k].nx * tab[k].ny
        gk = S.Grid(tab[k].nx, tab[k].ny, tab[k].dx, tab[k].dy)
        qk = [x[o:o + m] for x in init]
        S.swe_init(gk, p, B[o:o + m], eta[o:o + m], qk)
        S.swe_max_speed(gk, p, B[o:o + m], qk, 0, spd)
    dt0 = p.cfl_desired / float(spd.view(torch.float64).item())
    work = [[torch.empty(ncell, **F64) for _ in range(3)] for _ in range(3)]
    return ps, p, B, init, work, ncell, dt0


def test_tuner_times_every_candidate_and_picks_the_fastest(S):
    """swe_level_tune runs every schedule in both launch modes from the same
    state (row chunks in the persistent mode too), finds every result equal
    to the first candidate's, and names the fastest."""
    ps, p, B, init, (wa, wb, ref), ncell, dt0 = _tuner_setup(S)
    tab, _ = S.patch_table(ps.nx, ps.ny, ps.dx)
    cands = [S.Level(tab, S.SCHED_STRIP), S.Level(tab, S.SCHED_PACKED)] + \
        [S.Level(tab, S.SCHED_PACKED, chunk_rows=r) for r in (1, 8, 16)]
    mism = torch.zeros(1, dtype=torch.int32, device="cuda")
    entries, best = S.level_tune(cands, p, B, init, wa, wb, ref, S.new_ctl(), mism, dt0, 5, ncell)
    assert sorted((l, pm) for l, pm, _ in entries) == [(l, pm) for l in range(len(cands)) for pm in (0, 1)]
    assert all(u > 0.0 for _, _, u in entries)
    assert entries[best][2] == min(u for _, _, u in entries)
    assert int(mism.item()) == 0
    print("tuner:", {f"{l}/{pm}": round(u, 1) for l, pm, u in entries}, "best", entries[best][:2])


def test_tuner_rejects_candidates_that_disagree(S):
    """Two 'schedules' of different levels (walls against extrapolating
    sides) give different states: the tuner reports it (SWE_E_HIP) instead of
    timing them."""
    ps, p, B, init, (wa, wb, ref), ncell, dt0 = _tuner_setup(S, n=40, seed=6)
    walls, _ = S.patch_table(ps.nx, ps.ny, ps.dx)
    open_, _ = S.patch_table(ps.nx, ps.ny, ps.dx, bc=(S.BC_EXTRAP,) * 4)
    cands = [S.Level(walls, S.SCHED_PACKED), S.Level(open_, S.SCHED_PACKED)]
    mism = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(S.SweError) as ei:
        S.level_tune(cands, p, B, init, wa, wb, ref, S.new_ctl(), mism, dt0, 5, ncell)
    assert ei.value.status == S.E_HIP
    assert int(mism.item()) > 0
