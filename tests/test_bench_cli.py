"""bench.py's host-side contract without a GPU: it measures one GPU only and
says so for --gpus above 1 (exit status 2, before touching a device), and the
counter post-processing (--traffic-from, --valu-from) rejects directories
without counter output."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_post_processing_needs_counter_output(tmp_path):
    r = run("--valu-from", str(tmp_path))
    assert r.returncode != 0
    assert "counter_collection.csv" in (r.stdout + r.stderr)
