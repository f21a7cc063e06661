"""The regridding loop on the GPU: adjoint flags of a basin run are clustered
into boxes, the boxes refined 2x into patches filled by injection
(swe_prolong, bit for bit against the oracle's), and the patches advanced by
the batched level stepper against the oracle stepping each patch."""
import numpy as np
import pytest

from oracle import regrid as R
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


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def test_flags_to_patches_to_level(oracle, S):
    from test_gpu_level import oracle_level
    O = oracle
    n, ratio = 80, 2
    b = I.basin(n, 3)
    g = O.Grid(n, n, b.grid.dx, b.grid.dy)
    rc = O.run(g, O.Params(), O.NONLINEAR, b.B, b.eta0, (b.target[0], b.target[1], 60e3), 0.0, 1800.0, 3600.0,
               6, 1e-4, flag_every=3)
    flags = rc.flags_at[6]
    boxes = S.cluster(flags, 0.7, 2, 16)
    assert boxes == R.cluster(flags, 0.7, 2, 16) and len(boxes) >= 2
    print(f"regrid: {int(flags.sum())} flagged cells -> {len(boxes)} boxes", flush=True)
    # refined patches, filled by injection on the device
    nxp = [nx * ratio for (_, _, nx, _) in boxes]
    nyp = [ny * ratio for (_, _, _, ny) in boxes]
    dxp = [b.grid.dx / ratio] * len(boxes)
    tab, ncell = S.patch_table(nxp, nyp, dxp)
    lvl = S.Level(tab, S.SCHED_PACKED)
    box_t = dev(np.array(boxes, np.int32), torch.int32)
    gs = S.Grid(n, n, b.grid.dx, b.grid.dy)
    out_B = torch.full((ncell,), float("nan"), dtype=torch.float64, device="cuda")
    out_q = [torch.full((ncell,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
    S.prolong(gs, dev(b.B), [dev(x) for x in rc.q], box_t, lvl.patches_t, len(boxes), ratio, out_B, out_q)
    ref = R.prolong([rc.q[0], rc.q[1], rc.q[2], b.B], boxes, ratio)
    got = [x.cpu().numpy() for x in (out_q[0], out_q[1], out_q[2], out_B)]
    off = 0
    Bp, qp = [], []
    for k, parts in enumerate(ref):
        m = nxp[k] * nyp[k]
        for c in range(4):
            assert np.array_equal(got[c][off:off + m].reshape(nyp[k], nxp[k]), parts[c]), (k, c)
        qp.append([parts[0], parts[1], parts[2]])
        Bp.append(parts[3])
        off += m
    # advance the refined level and compare with the oracle patch by patch
    ps = I.PatchSet(nx=np.array(nxp), ny=np.array(nyp), dx=np.array(dxp), x_lo=None, y_lo=None, B=None, eta0=None)
    dts = [O.dt0(O.Grid(nxp[k], nyp[k], dxp[k], dxp[k]), O.Params(), O.NONLINEAR, Bp[k], *qp[k])
           for k in range(len(boxes))]
    dt0 = min(d for d in dts if d > 0)
    n_steps = 5
    qc, t, dt, acc, rej = oracle_level(O, ps, Bp, qp, dt0, n_steps)
    b2 = [torch.empty_like(x) for x in out_q]
    ctl = S.new_ctl()
    S.swe_ctl_set(ctl, 0.0, dt0, 1e30, 0)
    S.level_advance(lvl, S.Params(), out_B, out_q, b2, ctl, n_steps, 0)
    torch.cuda.synchronize()
    c = S.read_ctl(ctl)
    assert (c.n_accepted, c.n_rejected, c.t) == (acc, rej, t)
    cur = out_q if c.cur == 0 else b2
    res = [x.cpu().numpy() for x in cur]
    off = 0
    for k in range(len(boxes)):
        m = nxp[k] * nyp[k]
        for comp in range(3):
            gk = res[comp][off:off + m].reshape(nyp[k], nxp[k])
            rk = qc[k][comp]
            if comp == 0:
                gk, rk = gk + Bp[k], rk + Bp[k]
            scale = np.abs(rk).max() + (1.0 if comp == 0 else 0.0)
            assert np.abs(gk - rk).max() <= 1e-12 * max(scale, 1e-300), (k, comp)
        off += m


@pytest.mark.parametrize("ratio", [1, 3, 4, 6])
def test_prolong_ratios_match_oracle(S, ratio):
    """Injection at other refinement ratios (the paper's nested levels refine
    by 5 and 6, Sec. 6), for boxes of assorted shapes including ones on the
    grid's edges and corner, bit for bit against the oracle's repetition."""
    rng = np.random.default_rng(40 + ratio)
    nx, ny = 70, 45
    fields = [rng.normal(0.0, 1.0, (ny, nx)) for _ in range(4)]
    boxes = [(0, 0, 5, 7), (nx - 3, ny - 2, 3, 2), (11, 20, 17, 1), (30, 0, 1, ny), (20, 10, 13, 9)]
    nxp = [w * ratio for (_, _, w, _) in boxes]
    nyp = [h * ratio for (_, _, _, h) in boxes]
    tab, ncell = S.patch_table(nxp, nyp, [1.0] * len(boxes))
    # the device patch table alone (at ratio 1 some patches are one cell
    # wide, which injection allows and a level schedule does not)
    patches_t = dev(np.frombuffer(bytes(tab), dtype=np.uint8), torch.uint8)
    gs = S.Grid(nx, ny, 1.0, 1.0)
    out_B = torch.full((ncell,), float("nan"), dtype=torch.float64, device="cuda")
    out_q = [torch.full((ncell,), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
    box_t = dev(np.array(boxes, np.int32), torch.int32)
    S.prolong(gs, dev(fields[3]), [dev(x) for x in fields[:3]], box_t, patches_t, len(boxes), ratio,
              out_B, out_q)
    ref = R.prolong(fields, boxes, ratio)
    got = [x.cpu().numpy() for x in (out_q[0], out_q[1], out_q[2], out_B)]
    off = 0
    for k, parts in enumerate(ref):
        m = nxp[k] * nyp[k]
        for c in range(4):
            assert np.array_equal(got[c][off:off + m].reshape(nyp[k], nxp[k]), parts[c]), (k, c)
        off += m
    assert off == ncell
