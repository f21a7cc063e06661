"""ctypes front end of the CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py``.  The HIP library never imports it.

Arrays are numpy float64 (ny, nx) without ghost cells; 1D problems use
shape (nx,) or (1, nx).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SWE_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

BC_WALL, BC_EXTRAP = 0, 1
NONLINEAR, LINEAR = 0, 1
GAUSS, DISK = 0, 1


def build(openmp: bool = True) -> str:
    """Compile the oracle: plain C99, float64, no FMA contraction, no fast-math."""
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-o", LIB_PATH + ".tmp", os.path.join(HERE, "oracle.c"), "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("dx", C.c_double), ("dy", C.c_double),
                ("x_lo", C.c_double), ("y_lo", C.c_double), ("bc", C.c_int * 4)]


class _Params(C.Structure):
    _fields_ = [("g", C.c_double), ("sea_level", C.c_double), ("dry_tol", C.c_double),
                ("cfl_desired", C.c_double), ("cfl_max", C.c_double),
                ("order", C.c_int), ("transverse", C.c_int)]


_dp = C.POINTER(C.c_double)
_bp = C.POINTER(C.c_byte)


class _Problem(C.Structure):
    _fields_ = [("grid", _Grid), ("params", _Params), ("model", C.c_int),
                ("B", _dp), ("eta0", _dp),
                ("target_xc", C.c_double), ("target_yc", C.c_double), ("target_R", C.c_double),
                ("target_shape", C.c_int),
                ("t0", C.c_double), ("ts", C.c_double), ("tf", C.c_double), ("tol", C.c_double),
                ("K", C.c_int), ("flag_every", C.c_int),
                ("frames", _dp), ("q_out", _dp * 3),
                ("flags_at", _bp), ("flag_acc", _bp), ("maxip_acc", _dp),
                ("surface_tol", C.c_double), ("surface_flags_at", _bp),
                ("adj_grid", _Grid), ("adj_B", _dp), ("maxip_at", _dp)]


class _Result(C.Structure):
    _fields_ = [("n_adj_steps", C.c_int), ("n_sub", C.c_int), ("n_fwd_steps", C.c_int),
                ("n_rejected", C.c_int), ("n_flag_calls", C.c_int), ("n_clamped", C.c_int),
                ("status", C.c_int), ("dt_adj", C.c_double), ("t_end", C.c_double)]


@dataclass
class Grid:
    nx: int
    ny: int
    dx: float
    dy: float = 1.0
    x_lo: float = 0.0
    y_lo: float = 0.0
    bc: tuple = (BC_WALL, BC_WALL, BC_WALL, BC_WALL)

    def c(self) -> _Grid:
        g = _Grid(self.nx, self.ny, self.dx, self.dy, self.x_lo, self.y_lo)
        for k in range(4):
            g.bc[k] = self.bc[k]
        return g


@dataclass
class Params:
    g: float = 9.81
    sea_level: float = 0.0
    dry_tol: float = 1.0e-3
    cfl_desired: float = 0.9
    cfl_max: float = 1.0
    order: int = 2
    transverse: int = 1

    def c(self) -> _Params:
        return _Params(self.g, self.sea_level, self.dry_tol, self.cfl_desired, self.cfl_max,
                       self.order, self.transverse)


_lib = None


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(HERE, "oracle.c")
        stale = os.path.exists(LIB_PATH) and os.path.exists(src) and \
            os.path.getmtime(src) > os.path.getmtime(LIB_PATH) and "SWE_ORACLE_LIB" not in os.environ
        if not os.path.exists(LIB_PATH) or stale:
            build()
        _lib = C.CDLL(LIB_PATH)
        _lib.or_dt0.restype = C.c_double
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _p(a):
    return a.ctypes.data_as(_dp)


def _b(a):
    return a.ctypes.data_as(_bp) if a is not None else None


def swe_step(grid: Grid, prm: Params, B, h, hu, hv, dt):
    """One nonlinear 2D step.  Returns (h, hu, hv, cfl, n_clamped)."""
    shp = (grid.ny, grid.nx)
    B, h, hu, hv = (_f64(x, shp) for x in (B, h, hu, hv))
    o = [np.empty(shp) for _ in range(3)]
    cfl = C.c_double(0.0)
    ncl = C.c_int(0)
    rc = lib().or_swe_step(C.byref(grid.c()), C.byref(prm.c()), _p(B), _p(h), _p(hu), _p(hv),
                           _p(o[0]), _p(o[1]), _p(o[2]), C.c_double(dt), C.byref(cfl), C.byref(ncl))
    if rc != 0:
        raise ValueError("or_swe_step failed")
    return o[0], o[1], o[2], cfl.value, ncl.value


def lin_step(grid: Grid, prm: Params, B, eta, mu, dt):
    """One 1D linearized forward step.  Returns (eta, mu, cfl)."""
    shp = (grid.nx,)
    B, eta, mu = (_f64(x, shp) for x in (B, eta, mu))
    o = [np.empty(shp) for _ in range(2)]
    cfl = C.c_double(0.0)
    rc = lib().or_lin_step(C.byref(grid.c()), C.byref(prm.c()), _p(B), _p(eta), _p(mu),
                           _p(o[0]), _p(o[1]), C.c_double(dt), C.byref(cfl))
    if rc != 0:
        raise ValueError("or_lin_step failed")
    return o[0], o[1], cfl.value


def lin_step2d(grid: Grid, prm: Params, B, eta, mu, gamma, dt):
    """One 2D linearized forward step.  Returns (eta, mu, gamma, cfl)."""
    shp = (grid.ny, grid.nx)
    B, eta, mu, gamma = (_f64(x, shp) for x in (B, eta, mu, gamma))
    o = [np.empty(shp) for _ in range(3)]
    cfl = C.c_double(0.0)
    rc = lib().or_lin_step2d(C.byref(grid.c()), C.byref(prm.c()), _p(B), _p(eta), _p(mu), _p(gamma),
                             _p(o[0]), _p(o[1]), _p(o[2]), C.c_double(dt), C.byref(cfl))
    if rc != 0:
        raise ValueError("or_lin_step2d failed")
    return o[0], o[1], o[2], cfl.value


def adj_step(grid: Grid, prm: Params, B, q0, q1, q2, dt):
    """One time-reversed adjoint step (1D if ny == 1).  Returns (q0, q1, q2, cfl)."""
    shp = (grid.ny, grid.nx)
    B, q0, q1 = (_f64(x, shp) for x in (B, q0, q1))
    q2 = _f64(np.zeros(shp) if q2 is None else q2, shp)
    o = [np.empty(shp) for _ in range(3)]
    cfl = C.c_double(0.0)
    rc = lib().or_adj_step(C.byref(grid.c()), C.byref(prm.c()), _p(B), _p(q0), _p(q1), _p(q2),
                           _p(o[0]), _p(o[1]), _p(o[2]), C.c_double(dt), C.byref(cfl))
    if rc != 0:
        raise ValueError("or_adj_step failed")
    if grid.ny == 1:
        o[2][:] = 0.0
    return o[0], o[1], o[2], cfl.value


def target(grid: Grid, prm: Params, B, xc, yc, R, shape=GAUSS):
    shp = (grid.ny, grid.nx)
    B = _f64(B, shp)
    phi = np.empty(shp)
    lib().or_target(C.byref(grid.c()), C.byref(prm.c()), _p(B), C.c_double(xc), C.c_double(yc),
                    C.c_double(R), C.c_int(shape), _p(phi))
    return phi


def init_state(grid: Grid, prm: Params, model, B, eta0):
    shp = (grid.ny, grid.nx)
    B, eta0 = _f64(B, shp), _f64(eta0, shp)
    q = [np.empty(shp) for _ in range(3)]
    lib().or_init_state(C.byref(grid.c()), C.byref(prm.c()), C.c_int(model), _p(B), _p(eta0),
                        _p(q[0]), _p(q[1]), _p(q[2]))
    return q


def dt0(grid: Grid, prm: Params, model, B, q0, q1, q2):
    shp = (grid.ny, grid.nx)
    B, q0, q1, q2 = (_f64(x, shp) for x in (B, q0, q1, q2))
    return lib().or_dt0(C.byref(grid.c()), C.byref(prm.c()), C.c_int(model), _p(B), _p(q0),
                        _p(q1), _p(q2))


def adj_nsub(grid: Grid, prm: Params, B, t0, tf, K):
    shp = (grid.ny, grid.nx)
    B = _f64(B, shp)
    dt = C.c_double(0.0)
    ns = lib().or_adj_nsub(C.byref(grid.c()), C.byref(prm.c()), _p(B), C.c_double(t0),
                           C.c_double(tf), C.c_int(K), C.byref(dt))
    return ns, dt.value


def set_threads(n: int):
    """Threads of the oracle's row loops (results do not depend on it)."""
    lib().or_set_threads(C.c_int(int(n)))


def window(t, t0, ts, tf, K):
    """Returns (k_lo, k_hi) or None when t > tf."""
    lo, hi = C.c_int(0), C.c_int(0)
    ok = lib().or_window(C.c_double(t), C.c_double(t0), C.c_double(ts), C.c_double(tf),
                         C.c_int(K), C.byref(lo), C.byref(hi))
    return (lo.value, hi.value) if ok else None


def flag(grid: Grid, prm: Params, model, B, q0, q1, q2, frames, K, k_lo, k_hi, tol,
         flag_acc=None, maxip_acc=None):
    """Returns (flags int8, maxip); accumulators are updated in place if given."""
    shp = (grid.ny, grid.nx)
    B, q0, q1 = (_f64(x, shp) for x in (B, q0, q1))
    q2 = _f64(np.zeros(shp) if q2 is None else q2, shp)
    frames = np.ascontiguousarray(frames, dtype=np.float64)
    fl = np.empty(shp, np.int8)
    m = np.empty(shp)
    lib().or_flag(C.byref(grid.c()), C.byref(prm.c()), C.c_int(model), _p(B), _p(q0), _p(q1),
                  _p(q2), _p(frames), C.c_int(K), C.c_int(k_lo), C.c_int(k_hi), C.c_double(tol),
                  _b(fl), _p(m), _b(flag_acc), _p(maxip_acc) if maxip_acc is not None else None)
    return fl, m


@dataclass
class RunResult:
    frames: np.ndarray
    q: list
    flags_at: np.ndarray
    flag_acc: np.ndarray
    maxip_acc: np.ndarray
    n_adj_steps: int
    n_sub: int
    n_fwd_steps: int
    n_rejected: int
    n_flag_calls: int
    n_clamped: int
    status: int
    dt_adj: float
    t_end: float
    surface_flags_at: np.ndarray = None
    maxip_at: np.ndarray = None      # max inner product of the flag pass at t0 and each output time
    extra: dict = field(default_factory=dict)


def interp(grid: Grid, adj_grid: Grid, v):
    """Adjoint-grid plane v at the centres of grid (linear/bilinear, Sec. 4)."""
    v = _f64(v, (adj_grid.ny, adj_grid.nx))
    out = np.empty((grid.ny, grid.nx))
    lib().or_interp(C.byref(grid.c()), C.byref(adj_grid.c()), _p(v), _p(out))
    return out


def adj_split_parts(cL, cR, ydir, a):
    """(positive, negative) parts of the adjoint transverse split of the
    physical fluctuation a (3 components) on a wet-wet edge between cells of
    sound speeds cL and cR; ydir selects the y-edge frame."""
    a = _f64(a, (3,))
    pos, neg = np.empty(3), np.empty(3)
    lib().or_adj_split_parts(C.c_double(cL), C.c_double(cR), C.c_int(ydir), _p(a), _p(pos), _p(neg))
    return pos, neg


def flag_interp(grid: Grid, prm: Params, model, B, q0, q1, q2, adj_grid: Grid, adj_B, frames, K, k_lo, k_hi,
                tol, flag_acc=None, maxip_acc=None):
    """flag() with the snapshots on adj_grid.  Returns (flags, maxip)."""
    shp = (grid.ny, grid.nx)
    B, q0, q1 = (_f64(x, shp) for x in (B, q0, q1))
    q2 = _f64(q2, shp) if q2 is not None else np.zeros(shp)
    adj_B = _f64(adj_B, (adj_grid.ny, adj_grid.nx))
    frames = np.ascontiguousarray(frames, dtype=np.float64)
    fl = np.zeros(shp, np.int8)
    mx = np.zeros(shp)
    lib().or_flag_interp(C.byref(grid.c()), C.byref(prm.c()), C.c_int(model), _p(B), _p(q0), _p(q1), _p(q2),
                         C.byref(adj_grid.c()), _p(adj_B), _p(frames), C.c_int(K), C.c_int(k_lo),
                         C.c_int(k_hi), C.c_double(tol), _b(fl), _p(mx), _b(flag_acc),
                         _p(maxip_acc) if maxip_acc is not None else None)
    return fl, mx


def surface_flag(grid: Grid, prm: Params, model, B, q0, tol, flag_acc=None):
    """Surface flags |eta| > tol in wet cells (the criterion of Sec. 6)."""
    shp = (grid.ny, grid.nx)
    B, q0 = _f64(B, shp), _f64(q0, shp)
    fl = np.zeros(shp, np.int8)
    lib().or_surface_flag(C.byref(grid.c()), C.byref(prm.c()), C.c_int(model), _p(B), _p(q0),
                          C.c_double(tol), _b(fl), _b(flag_acc) if flag_acc is not None else None)
    return fl


def run(grid: Grid, prm: Params, model, B, eta0, target_xyR, t0, ts, tf, K, tol,
        flag_every=1, target_shape=GAUSS, surface_tol=None, adj_grid: Grid = None, adj_B=None) -> RunResult:
    """Adjoint snapshots then the forward run with flagging (Sec. 4); with
    surface_tol, also the surface flags at t0 and at the output times."""
    shp = (grid.ny, grid.nx)
    n = grid.nx * grid.ny
    ncomp = 3 if grid.ny > 1 else 2
    B, eta0 = _f64(B, shp), _f64(eta0, shp)
    ashp = shp if adj_grid is None else (adj_grid.ny, adj_grid.nx)
    frames = np.zeros((K + 1, ncomp) + ashp)
    q = [np.zeros(shp) for _ in range(3)]
    flags_at = np.zeros((K + 1,) + shp, np.int8)
    maxip_at = np.zeros((K + 1,) + shp)
    acc = np.zeros(shp, np.int8)
    macc = np.zeros(shp)
    pb = _Problem()
    pb.grid = grid.c()
    pb.params = prm.c()
    pb.model = model
    pb.B, pb.eta0 = _p(B), _p(eta0)
    pb.target_xc, pb.target_yc, pb.target_R = target_xyR
    pb.target_shape = target_shape
    pb.t0, pb.ts, pb.tf, pb.tol = t0, ts, tf, tol
    pb.K, pb.flag_every = K, flag_every
    pb.frames = _p(frames)
    for c in range(3):
        pb.q_out[c] = _p(q[c])
    pb.flags_at, pb.flag_acc, pb.maxip_acc = _b(flags_at), _b(acc), _p(macc)
    pb.maxip_at = _p(maxip_at)
    sflags = None
    if surface_tol is not None:
        sflags = np.zeros((K + 1,) + shp, np.int8)
        pb.surface_tol, pb.surface_flags_at = surface_tol, _b(sflags)
    if adj_grid is not None:
        adj_B = _f64(adj_B, ashp)
        pb.adj_grid, pb.adj_B = adj_grid.c(), _p(adj_B)
    res = _Result()
    lib().or_run(C.byref(pb), C.byref(res))
    del n
    return RunResult(frames=frames, q=q[:ncomp], flags_at=flags_at, flag_acc=acc, maxip_acc=macc,
                     n_adj_steps=res.n_adj_steps, n_sub=res.n_sub, n_fwd_steps=res.n_fwd_steps,
                     n_rejected=res.n_rejected, n_flag_calls=res.n_flag_calls,
                     n_clamped=res.n_clamped, status=res.status, dt_adj=res.dt_adj,
                     t_end=res.t_end, surface_flags_at=sflags, maxip_at=maxip_at)
