"""Thin ctypes binding of ``libswe.so`` (the C ABI of ``include/swe.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  Device memory and streams come from PyTorch
(float64 CUDA/HIP tensors; a 2D field is an (ny, nx) tensor whose row stride
is the grid pitch).  If the library is missing the import of a function
raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(HERE, "libswe.so")
LIB_PATH = os.environ.get("SWE_LIB") or DEFAULT_LIB

OK, E_INVAL, E_CFL, E_HIP, E_NOMEM, E_NONFINITE, E_NEGDEPTH = 0, -1, -2, -3, -4, -5, -6
BC_WALL, BC_EXTRAP = 0, 1
NONLINEAR, LINEAR = 0, 1
GAUSS, DISK = 0, 1


class SweError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"swe status {status}: {msg}")
        self.status = status


class swe_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("pitch", C.c_int32), ("bc", C.c_int32 * 4),
                ("dx", C.c_double), ("dy", C.c_double), ("x_lo", C.c_double), ("y_lo", C.c_double)]


class swe_params(C.Structure):
    _fields_ = [("model", C.c_int32), ("order", C.c_int32), ("transverse", C.c_int32),
                ("reserved", C.c_int32), ("g", C.c_double), ("sea_level", C.c_double),
                ("dry_tol", C.c_double), ("cfl_desired", C.c_double), ("cfl_max", C.c_double)]


class swe_fields(C.Structure):
    _fields_ = [("f0", C.c_void_p), ("f1", C.c_void_p), ("f2", C.c_void_p)]


class swe_problem(C.Structure):
    _fields_ = [("grid", swe_grid), ("params", swe_params), ("B", C.c_void_p), ("eta0", C.c_void_p),
                ("target_xc", C.c_double), ("target_yc", C.c_double), ("target_R", C.c_double),
                ("target_shape", C.c_int32), ("K", C.c_int32),
                ("t0", C.c_double), ("ts", C.c_double), ("tf", C.c_double), ("tol", C.c_double),
                ("flag_every", C.c_int32), ("full_frames", C.c_int32),
                ("frames", C.c_void_p), ("q_out", swe_fields), ("flags_at", C.c_void_p),
                ("flag_acc", C.c_void_p), ("maxip_acc", C.c_void_p),
                ("surface_tol", C.c_double), ("surface_flags_at", C.c_void_p),
                ("adj_grid", swe_grid), ("adj_B", C.c_void_p),
                ("launch_per_step", C.c_int32), ("reserved", C.c_int32)]


class swe_result(C.Structure):
    _fields_ = [("n_adj_steps", C.c_int32), ("n_sub", C.c_int32), ("n_fwd_steps", C.c_int32),
                ("n_rejected", C.c_int32), ("n_flag_calls", C.c_int32), ("n_clamped", C.c_int32),
                ("dt_adj", C.c_double), ("t_end", C.c_double)]


CTL_SPREAD = 8      # SWE_CTL_SPREAD
LEVEL_SYNC_WORDS = 4096   # SWE_LEVEL_SYNC_WORDS


class swe_ctl_state(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("t_out", C.c_double),
                ("cur", C.c_int32), ("final_step", C.c_int32), ("done", C.c_int32),
                ("last_accepted", C.c_int32), ("n_accepted", C.c_int32), ("n_rejected", C.c_int32)]


class swe_ctl(C.Structure):
    _fields_ = [("s", swe_ctl_state), ("cfl_bits", C.c_uint64), ("n_clamped", C.c_int32),
                ("n_nonfinite", C.c_int32), ("n_flag_calls", C.c_int32), ("reserved", C.c_int32),
                ("slot", swe_ctl_state * 2), ("pad_", C.c_uint8 * 88),
                ("ring", ((C.c_uint64 * 16) * CTL_SPREAD) * 3)]

    # flat access to the resolved state
    def __getattr__(self, name):
        if name in ("t", "dt", "t_out", "cur", "final_step", "done", "last_accepted", "n_accepted",
                    "n_rejected"):
            return getattr(self.s, name)
        raise AttributeError(name)


SCALARS_BYTES = 16  # swe_scalars: uint64 cfl_bits, int32 n_clamped, int32 n_nonfinite
CTL_BYTES = C.sizeof(swe_ctl)

_lib = None


def lib():
    """Load libswe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(python -m paper_1605_05320_amd.build)")
        if LIB_PATH == DEFAULT_LIB:
            # refuse a library built from other sources than those in the tree
            from . import build as _build
            try:
                with open(_build.STAMP) as f:
                    stamp = f.read().strip()
            except OSError:
                stamp = ""
            if stamp != _build.sources_hash():
                raise ImportError(f"{LIB_PATH} was not built from the current sources: rebuild it "
                                  "(python -m paper_1605_05320_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name in ("swe_step", "adj_step", "adj_target", "swe_init", "swe_max_speed", "adj_window",
                     "adj_flag", "swe_run", "swe_ctl_set", "swe_ctl_retarget", "swe_advance",
                     "swe_level_advance", "swe_level_schedule", "swe_level_tune", "swe_advance_flagged",
                     "swe_serve", "swe_surface_flag", "adj_flag_interp", "swe_cluster", "swe_prolong",
                     "swe_run_static", "adj_frame_bounds"):
            getattr(L, name).restype = C.c_int
        L.swe_run_workspace_bytes.restype = C.c_size_t
        L.swe_serve_footprint.restype = C.c_size_t
        L.swe_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(st: int):
    if st != OK:
        raise SweError(st, lib().swe_last_error().decode())


@dataclass
class Grid:
    nx: int
    ny: int
    dx: float
    dy: float = 1.0
    x_lo: float = 0.0
    y_lo: float = 0.0
    bc: tuple = (BC_WALL, BC_WALL, BC_WALL, BC_WALL)
    pitch: int | None = None

    def c(self) -> swe_grid:
        g = swe_grid(self.nx, self.ny, self.pitch or self.nx)
        for k in range(4):
            g.bc[k] = self.bc[k]
        g.dx, g.dy, g.x_lo, g.y_lo = self.dx, self.dy, self.x_lo, self.y_lo
        return g


@dataclass
class Params:
    model: int = NONLINEAR
    order: int = 2
    transverse: int = 1
    g: float = 9.81
    sea_level: float = 0.0
    dry_tol: float = 1.0e-3
    cfl_desired: float = 0.9
    cfl_max: float = 1.0

    def c(self) -> swe_params:
        return swe_params(self.model, self.order, self.transverse, 0, self.g, self.sea_level,
                          self.dry_tol, self.cfl_desired, self.cfl_max)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def fields(q) -> swe_fields:
    q = list(q) + [None] * (3 - len(q))
    return swe_fields(*(None if t is None else t.data_ptr() for t in q[:3]))


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def swe_step(grid: Grid, prm: Params, B, q_in, q_out, dt: float, scal=None, stream=None):
    _check(lib().swe_step(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), fields(q_in), fields(q_out),
                          C.c_double(dt), _ptr(scal), _stream(stream)))


def adj_step(grid: Grid, prm: Params, B, q_in, q_out, dt: float, scal=None, stream=None):
    _check(lib().adj_step(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), fields(q_in), fields(q_out),
                          C.c_double(dt), _ptr(scal), _stream(stream)))


def adj_target(grid: Grid, prm: Params, B, xc, yc, R, shape, phi, stream=None):
    _check(lib().adj_target(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), C.c_double(xc),
                            C.c_double(yc), C.c_double(R), C.c_int32(shape), fields(phi),
                            _stream(stream)))


def swe_init(grid: Grid, prm: Params, B, eta0, q, stream=None):
    _check(lib().swe_init(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), _ptr(eta0), fields(q),
                          _stream(stream)))


def swe_max_speed(grid: Grid, prm: Params, B, q, adjoint: int, out_bits, stream=None):
    _check(lib().swe_max_speed(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), fields(q or []),
                               C.c_int32(adjoint), _ptr(out_bits), _stream(stream)))


def adj_window(t, t0, ts, tf, K):
    lo, hi = C.c_int32(), C.c_int32()
    _check(lib().adj_window(C.c_double(t), C.c_double(t0), C.c_double(ts), C.c_double(tf),
                            C.c_int32(K), C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def adj_flag(grid: Grid, prm: Params, B, q, frames, K, k_lo, k_hi, tol, flags=None, maxip=None,
             flag_acc=None, maxip_acc=None, stream=None, bounds=None):
    _check(lib().adj_flag(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), fields(q), _ptr(frames),
                          C.c_int32(K), C.c_int32(k_lo), C.c_int32(k_hi), C.c_double(tol),
                          _ptr(flags), _ptr(maxip), _ptr(flag_acc), _ptr(maxip_acc), _ptr(bounds),
                          _stream(stream)))


def adj_frame_bounds(grid: Grid, frames, K, bounds, stream=None):
    """Non-zero boxes (i_lo, i_hi, j_lo, j_hi) of snapshots 0..K into the
    int32 device tensor `bounds` (4*(K+1) entries)."""
    _check(lib().adj_frame_bounds(C.byref(grid.c()), _ptr(frames), C.c_int32(K), _ptr(bounds), _stream(stream)))


def adj_flag_interp(grid: Grid, prm: Params, B, q, adj_grid: Grid, adj_B, frames, K, k_lo, k_hi, tol, flags=None,
                    maxip=None, flag_acc=None, maxip_acc=None, stream=None, bounds=None):
    _check(lib().adj_flag_interp(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), fields(q), C.byref(adj_grid.c()),
                                 _ptr(adj_B), _ptr(frames), C.c_int32(K), C.c_int32(k_lo), C.c_int32(k_hi),
                                 C.c_double(tol), _ptr(flags), _ptr(maxip), _ptr(flag_acc), _ptr(maxip_acc),
                                 _ptr(bounds), _stream(stream)))


def swe_surface_flag(grid: Grid, prm: Params, B, q, tol, flags=None, flag_acc=None, stream=None):
    _check(lib().swe_surface_flag(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), fields(q), C.c_double(tol),
                                  _ptr(flags), _ptr(flag_acc), _stream(stream)))


def make_problem(grid: Grid, prm: Params, B, eta0, target, t0, ts, tf, K, tol, frames, q_out,
                 flags_at=None, flag_acc=None, maxip_acc=None, flag_every=1, shape=GAUSS,
                 surface_tol=0.0, surface_flags_at=None, adj_grid: Grid = None, adj_B=None,
                 full_frames=0, launch_per_step=0) -> swe_problem:
    pb = swe_problem()
    pb.full_frames = full_frames
    pb.launch_per_step = launch_per_step
    pb.grid = grid.c()
    pb.params = prm.c()
    pb.B, pb.eta0 = B.data_ptr(), eta0.data_ptr()
    pb.target_xc, pb.target_yc, pb.target_R = target
    pb.target_shape = shape
    pb.K = K
    pb.t0, pb.ts, pb.tf, pb.tol = t0, ts, tf, tol
    pb.flag_every = flag_every
    pb.frames = frames.data_ptr()
    pb.q_out = fields(q_out)
    pb.flags_at = None if flags_at is None else flags_at.data_ptr()
    pb.flag_acc = None if flag_acc is None else flag_acc.data_ptr()
    pb.maxip_acc = None if maxip_acc is None else maxip_acc.data_ptr()
    pb.surface_tol = surface_tol
    pb.surface_flags_at = None if surface_flags_at is None else surface_flags_at.data_ptr()
    if adj_grid is not None:
        pb.adj_grid = adj_grid.c()
        pb.adj_B = adj_B.data_ptr()
    # the problem holds raw device pointers: keep the tensors alive with it
    pb._keep = (B, eta0, frames, tuple(q_out), flags_at, flag_acc, maxip_acc, surface_flags_at, adj_B)
    return pb


def swe_run_workspace_bytes(pb: swe_problem) -> int:
    return lib().swe_run_workspace_bytes(C.byref(pb))


def swe_run(pb: swe_problem, workspace, stream=None) -> swe_result:
    res = swe_result()
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().swe_run(C.byref(pb), _ptr(workspace), C.c_size_t(nbytes), C.byref(res),
                         _stream(stream)))
    return res


STATIC_WORKSPACE_BYTES = 64 << 20     # SWE_STATIC_WORKSPACE_BYTES


def swe_run_static(pb: swe_problem, stream=None) -> swe_result:
    """swe_run with the library's own fixed device workspace (no allocation)."""
    res = swe_result()
    _check(lib().swe_run_static(C.byref(pb), C.byref(res), _stream(stream)))
    return res


def new_ctl(device="cuda"):
    """A device buffer for one swe_ctl (uninitialised; use swe_ctl_set)."""
    import torch
    return torch.zeros(CTL_BYTES, dtype=torch.uint8, device=device)


def read_ctl(ctl_tensor) -> swe_ctl:
    raw = bytes(ctl_tensor.cpu().numpy().tobytes())
    return swe_ctl.from_buffer_copy(raw)


def swe_ctl_set(ctl, t, dt, t_out, cur=0, stream=None):
    _check(lib().swe_ctl_set(_ptr(ctl), C.c_double(t), C.c_double(dt), C.c_double(t_out),
                             C.c_int32(cur), _stream(stream)))


def swe_ctl_retarget(ctl, t_out, stream=None):
    _check(lib().swe_ctl_retarget(_ptr(ctl), C.c_double(t_out), _stream(stream)))


def swe_advance(grid: Grid, prm: Params, B, a, b, ctl, n_attempts: int, stream=None):
    _check(lib().swe_advance(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), fields(a), fields(b),
                             _ptr(ctl), C.c_int32(n_attempts), _stream(stream)))


class swe_flagging(C.Structure):
    _fields_ = [("frames", C.c_void_p), ("K", C.c_int32), ("flag_every", C.c_int32),
                ("t0", C.c_double), ("ts", C.c_double), ("tf", C.c_double), ("tol", C.c_double),
                ("flags_final", C.c_void_p), ("flag_acc", C.c_void_p), ("maxip_acc", C.c_void_p),
                ("adj_grid", C.POINTER(swe_grid)), ("adj_B", C.c_void_p), ("bounds", C.c_void_p)]


def swe_advance_flagged(grid: Grid, prm: Params, B, a, b, ctl, n_attempts: int, frames, K, flag_every,
                        t0, ts, tf, tol, flags_final=None, flag_acc=None, maxip_acc=None, adj_grid: Grid = None,
                        adj_B=None, stream=None, bounds=None):
    ag = None if adj_grid is None else C.pointer(adj_grid.c())
    fl = swe_flagging(frames.data_ptr(), K, flag_every, t0, ts, tf, tol,
                      None if flags_final is None else flags_final.data_ptr(),
                      None if flag_acc is None else flag_acc.data_ptr(),
                      None if maxip_acc is None else maxip_acc.data_ptr(),
                      ag, None if adj_B is None else adj_B.data_ptr(),
                      None if bounds is None else bounds.data_ptr())
    _check(lib().swe_advance_flagged(C.byref(grid.c()), C.byref(prm.c()), _ptr(B), fields(a), fields(b),
                                     _ptr(ctl), C.c_int32(n_attempts), C.byref(fl), _stream(stream)))


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------
class swe_request(C.Structure):
    _fields_ = [("arrival", C.c_double), ("grid", swe_grid), ("params", swe_params),
                ("B_host", C.c_void_p), ("eta0_host", C.c_void_p),
                ("target_xc", C.c_double), ("target_yc", C.c_double), ("target_R", C.c_double),
                ("target_shape", C.c_int32), ("K", C.c_int32),
                ("t0", C.c_double), ("ts", C.c_double), ("tf", C.c_double), ("tol", C.c_double),
                ("flag_every", C.c_int32), ("reserved", C.c_int32),
                ("flag_acc_host", C.c_void_p), ("maxip_acc_host", C.c_void_p), ("q_host", C.c_void_p * 3)]


class swe_request_stats(C.Structure):
    _fields_ = [("admitted", C.c_double), ("finished", C.c_double), ("latency", C.c_double),
                ("status", C.c_int32), ("slot", C.c_int32), ("n_adj_steps", C.c_int32),
                ("n_fwd_steps", C.c_int32), ("bytes", C.c_size_t)]


SERVE_DONE_FN = C.CFUNCTYPE(None, C.c_int32, C.POINTER(swe_request_stats), C.c_void_p)


class swe_serve_config(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("max_active", C.c_int32),
                ("realtime", C.c_int32), ("on_done", SERVE_DONE_FN), ("user", C.c_void_p)]


class Request:
    """One scenario for swe_serve, with host input and output arrays (numpy,
    C-contiguous float64 / int8 of shape (ny, nx)) kept alive here."""

    def __init__(self, grid: Grid, prm: Params, B, eta0, target, t0, ts, tf, K, tol, flag_every=1,
                 shape=GAUSS, arrival=0.0, want_q=True):
        import numpy as np
        self.B = np.ascontiguousarray(B, dtype=np.float64)
        self.eta0 = np.ascontiguousarray(eta0, dtype=np.float64)
        shp = self.B.shape
        ncomp = 3 if grid.ny > 1 else 2
        self.flag_acc = np.zeros(shp, np.int8)
        self.maxip_acc = np.zeros(shp, np.float64)
        self.q = [np.zeros(shp, np.float64) for _ in range(ncomp)] if want_q else []
        r = swe_request()
        r.arrival = arrival
        r.grid = grid.c()
        r.params = prm.c()
        r.B_host = self.B.ctypes.data
        r.eta0_host = self.eta0.ctypes.data
        r.target_xc, r.target_yc, r.target_R = target
        r.target_shape, r.K = shape, K
        r.t0, r.ts, r.tf, r.tol = t0, ts, tf, tol
        r.flag_every = flag_every
        r.flag_acc_host = self.flag_acc.ctypes.data
        r.maxip_acc_host = self.maxip_acc.ctypes.data
        for c in range(3):
            r.q_host[c] = self.q[c].ctypes.data if c < len(self.q) else None
        self.c = r


def serve_footprint(req: Request) -> int:
    return lib().swe_serve_footprint(C.byref(req.c))


def serve(reqs, arena, max_active: int, realtime: bool = False, check: bool = True, on_done=None):
    """Run swe_serve over a list of Request (ordered by arrival) with the
    device tensor ``arena`` as memory; on_done(index) is called (on a worker
    thread) as each request completes.  Returns (status, list of stats dicts)."""
    n = len(reqs)
    arr = (swe_request * n)(*[r.c for r in reqs])
    st = (swe_request_stats * n)()
    cb = SERVE_DONE_FN(lambda k, s, u: on_done(k)) if on_done else SERVE_DONE_FN()
    cfg = swe_serve_config(arena.data_ptr(), arena.numel() * arena.element_size(), max_active,
                           1 if realtime else 0, cb, None)
    rc = lib().swe_serve(arr, C.c_int32(n), C.byref(cfg), st)
    if check:
        _check(rc)
    out = [dict(admitted=s.admitted, finished=s.finished, latency=s.latency, status=s.status, slot=s.slot,
                n_adj_steps=s.n_adj_steps, n_fwd_steps=s.n_fwd_steps, bytes=s.bytes) for s in st]
    return rc, out


# --------------------------------------------------------------------------
# batched AMR level
# --------------------------------------------------------------------------
SCHED_STRIP, SCHED_PACKED = 0, 1


class swe_patch(C.Structure):
    _fields_ = [("offset", C.c_int64), ("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32 * 4),
                ("dx", C.c_double), ("dy", C.c_double)]


class swe_level(C.Structure):
    _fields_ = [("n_patches", C.c_int32), ("n_passes", C.c_int32), ("n_jobs", C.c_int32),
                ("chunk_rows", C.c_int32), ("patches", C.c_void_p), ("lanes", C.c_void_p),
                ("pass_rows", C.c_void_p), ("job_pass", C.c_void_p), ("sync", C.c_void_p),
                ("pass_row0", C.c_void_p)]


def patch_table(nx, ny, dx, dy=None, bc=(BC_WALL,) * 4):
    """Host array of swe_patch for patches stored back to back (offsets = running sums)."""
    n = len(nx)
    tab = (swe_patch * n)()
    off = 0
    for k in range(n):
        tab[k].offset = off
        tab[k].nx, tab[k].ny = int(nx[k]), int(ny[k])
        for c in range(4):
            tab[k].bc[c] = bc[c]
        tab[k].dx = float(dx[k])
        tab[k].dy = float(dx[k] if dy is None else dy[k])
        off += int(nx[k]) * int(ny[k])
    return tab, off


def level_schedule(tab, kind=SCHED_PACKED, chunk_rows=0):
    """Host schedule: returns (lanes int64[n_passes*64], pass_rows int32[n_passes],
    job_pass int32[n_jobs+1], pass_row0 int32[n_passes]) as numpy arrays."""
    import numpy as np
    n = len(tab)
    nj = C.c_int32(0)
    npass = lib().swe_level_schedule(tab, C.c_int32(n), C.c_int32(kind), C.c_int32(chunk_rows), None, None, None,
                                     None, C.byref(nj))
    if npass < 0:
        _check(npass)
    lanes = np.empty(npass * 64, np.int64)
    rows = np.empty(npass, np.int32)
    row0 = np.empty(npass, np.int32)
    jp = np.empty(nj.value + 1, np.int32)
    r = lib().swe_level_schedule(tab, C.c_int32(n), C.c_int32(kind), C.c_int32(chunk_rows),
                                 lanes.ctypes.data_as(C.c_void_p), rows.ctypes.data_as(C.c_void_p),
                                 row0.ctypes.data_as(C.c_void_p), jp.ctypes.data_as(C.c_void_p), C.byref(nj))
    if r < 0:
        _check(r)
    return lanes, rows, jp, row0


class Level:
    """A level's schedule and patch table on the device (tensors kept alive here)."""

    def __init__(self, tab, kind=SCHED_PACKED, device="cuda", chunk_rows=0):
        import numpy as np
        import torch
        lanes, rows, jp, row0 = level_schedule(tab, kind, chunk_rows)
        raw = np.frombuffer(bytes(tab), dtype=np.uint8)
        self.kind = kind
        self.chunk_rows = chunk_rows
        self.patches_t = torch.tensor(raw, dtype=torch.uint8, device=device)
        self.lanes_t = torch.tensor(lanes, device=device)
        self.rows_t = torch.tensor(rows, device=device)
        self.row0_t = torch.tensor(row0, device=device)
        self.jp_t = torch.tensor(jp, device=device)
        self.sync_t = torch.zeros(LEVEL_SYNC_WORDS, dtype=torch.int32, device=device)
        self.c = swe_level(len(tab), len(rows), len(jp) - 1, chunk_rows, self.patches_t.data_ptr(),
                           self.lanes_t.data_ptr(), self.rows_t.data_ptr(), self.jp_t.data_ptr(),
                           self.sync_t.data_ptr(), self.row0_t.data_ptr())
        self.lane_occupancy = float((lanes >= 0).mean())


def level_advance(level: Level, prm: Params, B, a, b, ctl, n_steps: int, persistent: int = 0,
                  stream=None):
    _check(lib().swe_level_advance(C.byref(level.c), C.byref(prm.c()), _ptr(B), fields(a), fields(b),
                                   _ptr(ctl), C.c_int32(n_steps), C.c_int32(persistent),
                                   _stream(stream)))


class swe_box(C.Structure):
    _fields_ = [("i_lo", C.c_int32), ("j_lo", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32)]


def cluster(flags, efficiency=0.7, min_side=4, max_side=32):
    """Host clustering of the non-zero cells of flags (numpy int8 (ny, nx)) into
    boxes [(i_lo, j_lo, nx, ny), ...] (see swe_cluster)."""
    import numpy as np
    f = np.ascontiguousarray(flags, dtype=np.int8)
    ny, nx = f.shape
    args = (f.ctypes.data_as(C.c_void_p), C.c_int32(nx), C.c_int32(ny), C.c_int32(nx), C.c_double(efficiency),
            C.c_int32(min_side), C.c_int32(max_side))
    cap = 1024
    out = (swe_box * cap)()
    n = lib().swe_cluster(*args, out, C.c_int32(cap))
    if n < 0:
        _check(n)
    if n > cap:                      # more boxes than the first buffer holds
        out = (swe_box * n)()
        n2 = lib().swe_cluster(*args, out, C.c_int32(n))
        if n2 < 0:
            _check(n2)
    return [(b.i_lo, b.j_lo, b.nx, b.ny) for b in out[:n]]


def prolong(grid: Grid, B, q, boxes_dev, patches_dev, n, ratio, out_B, out_q, stream=None):
    _check(lib().swe_prolong(C.byref(grid.c()), _ptr(B), fields(q), _ptr(boxes_dev), _ptr(patches_dev),
                             C.c_int32(n), C.c_int32(ratio), _ptr(out_B), fields(out_q), _stream(stream)))


class swe_tune_entry(C.Structure):
    _fields_ = [("level", C.c_int32), ("persistent", C.c_int32), ("us_per_attempt", C.c_double)]


def level_tune(levels, prm: Params, B, init, work_a, work_b, ref, ctl, mismatch, dt, n_trial, n_cells,
               stream=None):
    """Autotune the level schedule (see swe_level_tune).  Returns (entries, best)."""
    n = len(levels)
    arr = (C.POINTER(swe_level) * n)(*[C.pointer(l.c) for l in levels])
    out = (swe_tune_entry * (2 * n))()
    best = C.c_int32(-1)
    _check(lib().swe_level_tune(arr, C.c_int32(n), C.byref(prm.c()), _ptr(B), fields(init),
                                fields(work_a), fields(work_b), fields(ref), _ptr(ctl), _ptr(mismatch),
                                C.c_double(dt), C.c_int32(n_trial), C.c_int64(n_cells), out,
                                C.byref(best), _stream(stream)))
    return [(e.level, e.persistent, e.us_per_attempt) for e in out], best.value
