"""The C ABI without a GPU: the library loads and exports every function the
header declares, the ctypes mirrors of the header's structs have the C
layout (size and every field offset, compiled with gcc from the header), and
the host-only entry points (snapshot window, footprints, argument checks)
behave as documented."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1605_05320_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "swe.h")


@pytest.fixture(scope="module")
def S():
    from paper_1605_05320_amd import swe
    swe.lib()
    return swe


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = "\n".join(l for l in text.splitlines() if not l.lstrip().startswith("#"))
    names = re.findall(r"SWE_API\s+[\w\s\*]*?\b(\w+)\s*\(", text)
    assert len(names) >= 19
    return names


def test_every_declared_symbol_is_exported(S):
    names = declared_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(S.lib(), n)   # resolvable through the loader
    # nothing but the ABI leaks out of the library
    ours = {e for e in exported if e.startswith(("swe_", "adj_"))}
    assert ours == set(names)


def _struct_classes(S):
    return [S.swe_grid, S.swe_params, S.swe_fields, S.swe_problem, S.swe_result, S.swe_ctl_state,
            S.swe_ctl, S.swe_patch, S.swe_level, S.swe_tune_entry, S.swe_flagging, S.swe_request,
            S.swe_request_stats, S.swe_serve_config, S.swe_box]


def test_ctypes_mirrors_match_the_header(S, tmp_path):
    classes = _struct_classes(S)
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "swe.h"', "int main(void) {"]
    for cls in classes:
        name = cls.__name__
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for cls in classes:
        name = cls.__name__
        assert int(got[name]) == C.sizeof(cls), name
        for f in cls._fields_:
            assert int(got[f"{name}.{f[0]}"]) == getattr(cls, f[0]).offset, f"{name}.{f[0]}"


def test_binding_constants_match_the_header(S, tmp_path):
    consts = {"SWE_CTL_SPREAD": S.CTL_SPREAD, "SWE_LEVEL_SYNC_WORDS": S.LEVEL_SYNC_WORDS,
              "SWE_STATIC_WORKSPACE_BYTES": S.STATIC_WORKSPACE_BYTES}
    lines = ["#include <stdio.h>", '#include "swe.h"', "int main(void) {"]
    lines += [f'printf("{k} %llu\\n", (unsigned long long)({k}));' for k in consts]
    lines += ["return 0;", "}"]
    src = tmp_path / "consts.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "consts"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for k, v in consts.items():
        assert int(got[k]) == v, k


def test_window_matches_oracle(S, oracle):
    rng = np.random.default_rng(11)
    for K in (1, 3, 8, 32):
        t0, tf = 0.0, 7200.0
        for ts in (0.0, 1800.0, 3600.0, 7200.0):
            ts_grid = list(np.linspace(t0, tf, 4 * K + 1)) + list(rng.uniform(t0, tf, 50))
            for t in ts_grid:
                o = oracle.window(float(t), t0, ts, tf, K)
                lo, hi = S.adj_window(float(t), t0, ts, tf, K)
                assert o is not None and (lo, hi) == o, (K, ts, t)
    # past the final time the window is empty
    lo, hi = S.adj_window(7300.0, 0.0, 0.0, 7200.0, 4)
    assert lo > hi


def test_window_rejects_bad_arguments(S):
    with pytest.raises(S.SweError):
        S.adj_window(0.0, 0.0, 0.0, 10.0, 0)
    with pytest.raises(S.SweError):
        S.adj_window(0.0, 10.0, 10.0, 10.0, 4)


def _request(S, n, K=4, seed=1):
    b = I.basin(n, seed)
    g = S.Grid(b.grid.nx, b.grid.ny, b.grid.dx, b.grid.dy, b.grid.x_lo, b.grid.y_lo)
    return S.Request(g, S.Params(), b.B, b.eta0, b.target, 0.0, 1800.0, 3600.0, K, 1e-4)


def test_serve_footprint(S):
    r4 = _request(S, 64, K=4)
    r8 = _request(S, 64, K=8)
    f4, f8 = S.serve_footprint(r4), S.serve_footprint(r8)
    plane = 64 * 64 * 8
    # inputs, snapshots, final state, accumulators and the driver workspace
    assert f4 >= plane * (2 + 5 * 3 + 3 + 1) + 64 * 64
    assert f8 - f4 == 4 * 3 * plane
    assert f4 % 256 == 0
    bad = _request(S, 64)
    bad.c.K = 0
    assert S.serve_footprint(bad) == 0
    bad = _request(S, 64)
    bad.c.grid.pitch = 65
    assert S.serve_footprint(bad) == 0


def test_serve_rejects_bad_config_before_touching_the_device(S):
    r = _request(S, 32)
    arr = (S.swe_request * 1)(r.c)
    st = (S.swe_request_stats * 1)()
    cfg = S.swe_serve_config(None, 1 << 20, 1, 0)
    assert S.lib().swe_serve(arr, 1, C.byref(cfg), st) == S.E_INVAL
    cfg = S.swe_serve_config(256, 1 << 20, 0, 0)
    assert S.lib().swe_serve(arr, 1, C.byref(cfg), st) == S.E_INVAL
    cfg = S.swe_serve_config(257, 1 << 20, 1, 0)
    assert S.lib().swe_serve(arr, 1, C.byref(cfg), st) == S.E_INVAL
    # arrivals out of order
    r2 = _request(S, 32)
    r.c.arrival, r2.c.arrival = 1.0, 0.5
    arr = (S.swe_request * 2)(r.c, r2.c)
    st = (S.swe_request_stats * 2)()
    cfg = S.swe_serve_config(256, 1 << 30, 2, 1)
    assert S.lib().swe_serve(arr, 2, C.byref(cfg), st) == S.E_INVAL
    assert "arrival" in S.lib().swe_last_error().decode()


@pytest.mark.parametrize("field,value", [("g", 0.0), ("g", 1e101), ("dry_tol", 0.0), ("dry_tol", 1e-101),
                                         ("dry_tol", float("nan"))])
def test_step_rejects_parameters_out_of_range_before_touching_the_device(S, field, value):
    """g and dry_tol outside [1e-100, 1e100] are argument errors (the step
    kernels' square roots and divisions rely on that range); the check comes
    before any device call, so host buffers stand in for the planes."""
    import torch
    g = S.Grid(8, 8, 1.0, 1.0)
    prm = S.Params()
    setattr(prm, field, value)
    B = torch.zeros(64, dtype=torch.float64)
    qa = [torch.zeros(64, dtype=torch.float64) for _ in range(3)]
    qb = [torch.zeros(64, dtype=torch.float64) for _ in range(3)]
    null_stream = type("NullStream", (), {"cuda_stream": 0})()
    with pytest.raises(S.SweError) as e:
        S.swe_step(g, prm, B, qa, qb, 0.1, stream=null_stream)
    assert e.value.status == S.E_INVAL
    assert "1e-100" in S.lib().swe_last_error().decode()


def test_static_driver_refuses_a_problem_beyond_its_array(S):
    """swe_run_static refuses a grid whose workspace exceeds its fixed array
    before any device work (the pointers are never touched)."""
    n = 1200
    g = S.Grid(n, n, 1000.0, 1000.0)
    fake = C.c_void_p(0x1000)

    class T:            # a stand-in device pointer (never dereferenced)
        def data_ptr(self):
            return fake.value
    t = T()
    pb = S.make_problem(g, S.Params(), t, t, (0.0, 0.0, 1e4), 0.0, 0.0, 1.0, 1, 1e-4, t, [t, t, t])
    assert S.swe_run_workspace_bytes(pb) > S.STATIC_WORKSPACE_BYTES
    null_stream = type("Stream", (), {"cuda_stream": 0})()
    with pytest.raises(S.SweError) as ei:
        S.swe_run_static(pb, stream=null_stream)
    assert ei.value.status == S.E_NOMEM
    assert "static workspace" in str(ei.value)


@pytest.mark.parametrize("case,grid,msg", [
    ("empty x", dict(nx=0, ny=8), "nx = 0"),
    ("one column", dict(nx=1, ny=8), "nx = 1"),
    ("empty y", dict(nx=8, ny=0), "ny = 0"),
    ("pitch below nx", dict(nx=8, ny=8, pitch=7), "pitch"),
    ("row beyond the store range", dict(nx=(1 << 27) + 1, ny=2), "nx ="),
    ("zero dx", dict(nx=8, ny=8, dx=0.0), "dx"),
    ("NaN dx", dict(nx=8, ny=8, dx=float("nan")), "dx"),
    ("zero dy", dict(nx=8, ny=8, dy=0.0), "dy"),
    ("unknown boundary", dict(nx=8, ny=8, bc=(0, 0, 2, 0)), "bc[2]"),
])
def test_degenerate_grids_are_refused_before_touching_the_device(S, case, grid, msg):
    """Empty and one-column grids, a pitch below nx, a row too long for the
    kernels' 32-bit row offsets, non-positive or NaN cell sizes and unknown
    boundary codes are argument errors of every entry point that takes a grid;
    the check comes first, so host buffers stand in for the planes."""
    import torch
    kw = dict(dx=100.0, dy=100.0)
    kw.update(grid)
    g = S.Grid(**kw)
    B = torch.zeros(64, dtype=torch.float64)
    qa = [torch.zeros(64, dtype=torch.float64) for _ in range(3)]
    qb = [torch.zeros(64, dtype=torch.float64) for _ in range(3)]
    null_stream = type("NullStream", (), {"cuda_stream": 0})()
    for fn, prm in ((S.swe_step, S.Params()), (S.adj_step, S.Params())):
        with pytest.raises(S.SweError) as e:
            fn(g, prm, B, qa, qb, 0.1, stream=null_stream)
        assert e.value.status == S.E_INVAL, case
        assert msg in S.lib().swe_last_error().decode(), case


@pytest.mark.parametrize("case", ["zero dt", "negative dt", "NaN dt", "aliased planes", "nonlinear in 1D"])
def test_step_refuses_degenerate_calls(S, case):
    """A step of non-positive or NaN length, output planes that alias the
    inputs, and the (two-dimensional) nonlinear model on a single row are
    refused with SWE_E_INVAL before any device work."""
    import torch
    g = S.Grid(8, 1 if case == "nonlinear in 1D" else 8, 100.0, 100.0)
    B = torch.zeros(64, dtype=torch.float64)
    qa = [torch.zeros(64, dtype=torch.float64) for _ in range(3)]
    qb = qa if case == "aliased planes" else [torch.zeros(64, dtype=torch.float64) for _ in range(3)]
    dt = {"zero dt": 0.0, "negative dt": -1.0, "NaN dt": float("nan")}.get(case, 0.1)
    null_stream = type("NullStream", (), {"cuda_stream": 0})()
    with pytest.raises(S.SweError) as e:
        S.swe_step(g, S.Params(), B, qa, qb, dt, stream=null_stream)
    assert e.value.status == S.E_INVAL
