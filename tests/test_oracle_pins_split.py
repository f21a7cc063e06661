"""Pins of the oracle's transverse splits over variable depth, its Gaussian
target data and its time-step rules (adjoint sub-stepping, first forward
step).

The linear models split a fluctuation that enters a cell on the
eigenvectors of a pair of cells that share the receiving cell (the 2D
equations of Sec. 5 linearized about the sea at rest, and their adjoint).
Which pair, and which cell's wave speed goes with which family, changes the
transverse terms by O(h) relative over smooth depth, so convergence rates
alone cannot tell the assignments apart (a scheme with the speeds swapped
still converges at second order).  The pins below use the principle of the
wave-propagation method that the 1D reflection/transmission pin fixes for
the normal solve: what moves into a cell travels in that cell's medium, so
it lies on that cell's own eigenvector of the family moving that way.  Over
four cells of four different depths a wrong pair or a swapped speed breaks
that relation by O(1).
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

from paper_1605_05320_amd import inputs as I

G = 9.81


# --------------------------------------------------------------------------
# transverse splits: what enters a diagonal neighbour lies on its own
# eigenvectors
# --------------------------------------------------------------------------
def _impulse_step(O, adjoint, order, seed):
    """One step from a single-cell impulse at (3, 3) of a 7 x 7 grid whose
    cells all have different depths (500..4000 m).  Returns (dq, c) with dq
    the change of every cell and c the cells' wave speeds sqrt(g hbar)."""
    rng = np.random.default_rng(seed)
    n = 7
    depth = rng.permutation(np.linspace(500.0, 4000.0, n * n)).reshape(n, n)
    B = -depth
    q0 = [np.zeros((n, n)) for _ in range(3)]
    for c in range(3):
        q0[c][3, 3] = rng.uniform(0.5, 1.5) * rng.choice([-1.0, 1.0])
    dx, dy = 1000.0, 1300.0
    g = O.Grid(n, n, dx, dy)
    p = O.Params(order=order, transverse=1)
    cmax = math.sqrt(G * depth.max())
    dt = 0.45 * min(dx, dy) / cmax
    step = O.adj_step if adjoint else O.lin_step2d
    q1 = step(g, p, B, q0[0], q0[1], q0[2], dt)[:3]
    dq = [q1[c] - q0[c] for c in range(3)]
    return dq, np.sqrt(G * depth)


@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_transverse_parts_lie_on_the_receiving_cells_eigenvectors(oracle, adjoint, order, seed):
    """A diagonal neighbour of the impulse has no edge with a wave of its own
    after one step: all it receives is the transverse part of one x-edge
    fluctuation split along y and of one y-edge fluctuation split along x,
    each moving into it.  Both must lie on that cell's eigenvectors (speed c of
    the cell itself) of the families moving away from the impulse:
      adjoint (eigenvectors (-c, 1) moving up/right, (c, 1) moving down/left,
               surface first, then the normal component):
          d_eta = -(sx c d_mu + sy c d_gamma)
      linear forward (eigenvectors (1, c) moving up/right, (1, -c) down/left):
          c d_eta = sx d_mu + sy d_gamma
    with sx = +1 for the neighbour on the right, -1 on the left, sy likewise
    above/below.  The speed of any other cell (the source cell, the other
    cell of a neighbouring pair) violates the relation by O(1), since every
    depth of the grid is different."""
    O = oracle
    dq, c = _impulse_step(O, adjoint, order, seed)
    for sx in (-1, 1):
        for sy in (-1, 1):
            j, i = 3 + sy, 3 + sx
            de, dm, dg = dq[0][j, i], dq[1][j, i], dq[2][j, i]
            cc = c[j, i]
            assert abs(dm) > 1e-8 and abs(dg) > 1e-8, "both transverse parts must reach the cell"
            scale = cc * (abs(dm) + abs(dg)) + abs(de) * cc
            if adjoint:
                res = de + (sx * cc * dm + sy * cc * dg)
            else:
                res = cc * de - (sx * dm + sy * dg)
            assert abs(res) <= 1e-12 * scale, (sx, sy, res, scale)


def test_transverse_pin_rejects_the_other_speeds(oracle):
    """The relation above is specific: with the speed of the diagonal cell's
    neighbours in its place it fails by far more than rounding (so the pin
    can tell a swapped or shifted assignment from the built one)."""
    O = oracle
    dq, c = _impulse_step(O, True, 2, 0)
    j, i = 4, 4
    de, dm, dg = dq[0][j, i], dq[1][j, i], dq[2][j, i]
    for cj, ci in ((3, 4), (4, 3), (3, 3), (5, 4), (4, 5)):
        cw = c[cj, ci]
        res = de + (cw * dm + cw * dg)
        assert abs(res) > 1e-6 * cw * (abs(dm) + abs(dg))


# --------------------------------------------------------------------------
# guided standing mode over depth varying across the basin
# --------------------------------------------------------------------------
LX, LY = 200.0e3, 100.0e3


def _depth(y):
    return 2500.0 + 1500.0 * np.cos(np.pi * y / LY)


def _mode(k):
    """Lowest standing mode of a closed basin [0, LX] x [0, LY] with depth
    h(y): eta = phi(y) cos(k x) cos(w t) solves both the linearized equations
    and the adjoint equations of Sec. 5 when (c^2 phi')' + (w^2 - c^2 k^2) phi = 0
    with phi' = 0 at the side walls (c^2 = g h).  Solved here by shooting
    (scipy ODE integrator to 1e-12, root of phi'(LY) in w) - independent of
    the oracle."""
    c2 = lambda y: G * _depth(y)

    def shoot(w):
        f = lambda y, s: [s[1] / c2(y), -(w * w - c2(y) * k * k) * s[0]]
        return solve_ivp(f, (0.0, LY), [1.0, 0.0], rtol=1e-12, atol=1e-14, dense_output=True)

    lo, hi = 0.5 * math.sqrt(G * 1000.0) * k, 0.999 * math.sqrt(G * 4000.0) * k
    w = brentq(lambda w: shoot(w).y[1, -1], lo, hi, xtol=1e-15, rtol=1e-15)
    return w, shoot(w)


def _mode_error(O, n, w, sol, k, adjoint, along_y):
    """L1 error of eta after one period (the exact state is the initial one)
    on an n x n/2 grid (or its transpose with the mode running along y)."""
    nl, nt = n, n // 2
    dl, dt_ = LX / nl, LY / nt
    xl = (np.arange(nl) + 0.5) * dl
    yt = (np.arange(nt) + 0.5) * dt_
    phi = sol.sol(yt)[0]
    eta = phi[:, None] * np.cos(k * xl)[None, :]
    B = -np.repeat(_depth(yt)[:, None], nl, axis=1)
    if along_y:
        eta, B = eta.T.copy(), B.T.copy()
        g = O.Grid(nt, nl, dt_, dl)
    else:
        g = O.Grid(nl, nt, dl, dt_)
    p = O.Params()
    T = 2.0 * math.pi / w
    steps = int(math.ceil(T / (0.9 * min(dl, dt_) / math.sqrt(G * 4000.0))))
    dt = T / steps
    q = [eta, np.zeros_like(eta), np.zeros_like(eta)]
    step = O.adj_step if adjoint else O.lin_step2d
    for _ in range(steps):
        q = list(step(g, p, B, q[0], q[1], q[2], dt)[:3])
    return float(np.abs(q[0] - eta).mean())


@pytest.mark.parametrize("along_y", [False, True])
def test_guided_mode_adjoint_second_order(oracle, along_y):
    """The adjoint (f-wave form with the transverse splits above) converges
    to the standing mode at second order, along x and along y."""
    O = oracle
    k = 2.0 * math.pi / LX
    w, sol = _mode(k)
    e = [_mode_error(O, n, w, sol, k, True, along_y) for n in (32, 64, 128)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert e[2] < 1.5e-3 and min(orders) > 1.8, (e, orders)


@pytest.mark.parametrize("along_y", [False, True])
def test_guided_mode_linear_forward_first_order(oracle, along_y):
    """The linear forward in wave form, the exact discrete transpose of the
    adjoint at first order, converges to the same mode over variable depth at
    first order only: its fluctuations sum to (d_mu, cL cR d_eta + (cR - cL) d_mu)
    at an edge, and the (cR - cL) d_mu term leaves an O(h) error where the
    depth varies (at constant depth it is second order, pinned by the
    axisymmetric wave)."""
    O = oracle
    k = 2.0 * math.pi / LX
    w, sol = _mode(k)
    e = [_mode_error(O, n, w, sol, k, False, along_y) for n in (32, 64, 128)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert e[2] < 1.5e-2 and min(orders) > 0.75, (e, orders)


# --------------------------------------------------------------------------
# Gaussian target (eq. phi_Alaska with a Gaussian in place of the indicator)
# --------------------------------------------------------------------------
def test_gaussian_target_closed_form(oracle):
    """phi = exp(-r^2/R^2): its integral is pi R^2 (2D) and sqrt(pi) R (1D);
    a uniform grid's midpoint sum reproduces a Gaussian's integral to far
    below rounding once R spans a few cells (Poisson summation); at r = R it
    is exactly exp(-1); it is 0 in cells dry for the adjoint."""
    O = oracle
    n, dx = 200, 1000.0
    R = 20.0e3
    xc = (100 + 0.5) * dx            # a cell centre
    yc = (90 + 0.5) * dx
    g = O.Grid(n, n, dx, dx)
    p = O.Params()
    B = np.full((n, n), -3000.0)
    phi = O.target(g, p, B, xc, yc, R, O.GAUSS)
    assert abs(phi.sum() * dx * dx - math.pi * R * R) <= 1e-9 * math.pi * R * R
    assert phi[90, 100] == 1.0
    # cells whose centre lies exactly R away along an axis
    for (j, i) in ((90, 120), (90, 80), (110, 100), (70, 100)):
        assert abs(phi[j, i] - math.exp(-1.0)) <= 2.0 ** -52
    # dry cells get 0; wet cells are unaffected by their dry neighbours
    B2 = B.copy()
    B2[:, :95] = 10.0
    phi2 = O.target(g, p, B2, xc, yc, R, O.GAUSS)
    assert not phi2[:, :95].any()
    assert np.array_equal(phi2[:, 95:], phi[:, 95:])
    # 1D
    g1 = O.Grid(4000, 1, 100.0, 1.0, -200.0e3)
    phi1 = O.target(g1, p, np.full(4000, -3000.0), -17.5e3, 0.0, 7.5e3, O.GAUSS)
    assert abs(phi1.sum() * 100.0 - math.sqrt(math.pi) * 7.5e3) <= 1e-9 * 7.5e3


# --------------------------------------------------------------------------
# time-step rules
# --------------------------------------------------------------------------
def test_adjoint_substeps_of_the_configured_runs(oracle):
    """n_sub = ceil(ds / dt_cfl), dt_cfl = 0.9 dx / c_max, dt = ds / n_sub.
    1D shelf (2000 cells over 400 km, deepest 4000 m, 3 h in 60 snapshot
    intervals): ds = 180 s, dt_cfl = 0.9 * 200 / sqrt(9.81 * 4000) = 0.90869 s,
    ds / dt_cfl = 198.09, so 199 sub-steps.  512^2 basin (2 km cells, deepest
    4000 m, 2 h in 64 intervals): ds = 112.5 s, dt_cfl = 9.0869 s, ratio
    12.38, so 13."""
    O = oracle
    s = I.shelf1d(2000, 0)
    n1, dt1 = O.adj_nsub(O.Grid(2000, 1, s.dx, 1.0, s.x_lo), O.Params(), s.B, 0.0, 10800.0, 60)
    assert n1 == 199 and dt1 == 180.0 / 199
    b = I.basin(512, 3)
    gb = O.Grid(512, 512, b.grid.dx, b.grid.dy)
    assert abs(b.B.min() + 4000.0) < 1e-6          # the abyssal plain is the deepest water
    n3, dt3 = O.adj_nsub(gb, O.Params(), b.B, 0.0, 7200.0, 64)
    assert n3 == 13 and dt3 == 112.5 / 13
    # a run whose ratio is an integer plus a little needs the next integer
    g = O.Grid(10, 1, 100.0)
    Bc = np.full(10, -1000.0)
    dtc = 0.9 * 100.0 / math.sqrt(G * 1000.0)
    n, _ = O.adj_nsub(g, O.Params(), Bc, 0.0, 10 * (7.0 * dtc * (1.0 + 1e-9)), 10)
    assert n == 8


def test_first_forward_step_closed_form(oracle):
    """dt0 = 0.9 / max over wet cells of max((|u| + sqrt(g h))/dx, (|v| + sqrt(g h))/dy).
    Stoker's dam break at rest (h = 2 | 1): 0.9 dx / sqrt(2 g).  A uniform
    current u = 3, v = -4 over h = 10 with dx = 2 dy: the y term wins."""
    O = oracle
    n = 16
    h = np.where(np.arange(n) < n // 2, 2.0, 1.0)[None, :].repeat(4, axis=0)
    B = -h
    g = O.Grid(n, 4, 50.0, 50.0)
    z = np.zeros_like(h)
    assert abs(O.dt0(g, O.Params(), O.NONLINEAR, B - 10.0, h, z, z) - 0.9 * 50.0 / math.sqrt(2 * G)) <= 1e-15
    h2 = np.full((4, n), 10.0)
    g2 = O.Grid(n, 4, 100.0, 50.0)
    want = 0.9 / ((4.0 + math.sqrt(G * 10.0)) / 50.0)
    got = O.dt0(g2, O.Params(), O.NONLINEAR, -h2, h2, 3.0 * h2, -4.0 * h2)
    assert abs(got - want) <= 1e-15 * want
    # a current against x sets the step through its magnitude
    g4 = O.Grid(n, 4, 50.0, 50.0)
    want4 = 0.9 / ((6.0 + math.sqrt(G * 10.0)) / 50.0)
    got4 = O.dt0(g4, O.Params(), O.NONLINEAR, -h2, h2, -6.0 * h2, 1.0 * h2)
    assert abs(got4 - want4) <= 1e-15 * want4
    # dry cells do not count
    h3 = h2.copy()
    h3[0, 0] = 1e-4
    hu3 = 3.0 * h2
    hu3[0, 0] = 1.0              # |u| = 1e4 in a dry cell
    got3 = O.dt0(g2, O.Params(), O.NONLINEAR, -h2, h3, hu3, -4.0 * h2)
    assert got3 == got
