"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Two small drivers in tests/sanitize/ exercise, with random sizes, the code
that runs on the CPU: the oracle's entry points (built with gcc), and the
library's host paths that need no device (snapshot windows, level schedules,
flag clustering, footprints, workspace sizes, and the argument checks that
refuse a call before any device work).  The device code of the library is
compiled as usual; only its host side carries the sanitizers."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", *SAN, "-I" + os.path.join(ROOT, "oracle"),
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_main.c"), "-o", exe,
          "-lm", "-pthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    assert "oracle paths ok" in _run([exe], env=env, timeout=300)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="no hipcc")
def test_library_host_paths_under_sanitizers(tmp_path):
    from paper_1605_05320_amd import build as B
    flags = [f for f in B.HIPFLAGS if f != "-O3"] + ["-O1", "-g", "-fno-omit-frame-pointer"]
    host_san = [x for s in SAN for x in ("-Xarch_host", s)]

    def compile_one(src):
        obj = str(tmp_path / src.replace(".hip", ".o"))
        _run(["hipcc", *flags, *host_san, "-c", os.path.join(B.CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(5, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, B.SOURCES))
    exe = str(tmp_path / "host_san")
    _run(["hipcc", "--offload-arch=gfx950", "-g", *host_san, "-I" + os.path.join(ROOT, "include"), "-x", "hip",
          os.path.join(HERE, "host_main.cpp"), "-x", "none", *objs, "-o", exe, "-pthread"])
    # the HIP runtime's own allocations at start-up are not this library's
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    assert "host paths ok" in _run([exe], env=env, timeout=300)
