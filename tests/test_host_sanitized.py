"""Host logic under address and undefined-behaviour sanitizers (CPU only):

  * the serving loop's admission bookkeeping (budget, active limit, pool of
    closed sessions' device memory) against a fake allocator, scripted and
    over seeded random open/close streams, with leak detection;
  * the C ABI's host paths (argument validation of the entry points, the
    interval / block-size / degree policies, server configuration) through
    a build of the library whose host code carries the sanitizers.

The binaries are (re)built by tests/host/build_checks.py when a source is
newer than them.
"""
import glob
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "host", "_build")
BINS = [os.path.join(OUT, "admission_check"), os.path.join(OUT, "capi_check")]


def _stale():
    srcs = (glob.glob(os.path.join(ROOT, "paper_1904_10585_amd", "csrc", "*")) +
            glob.glob(os.path.join(ROOT, "include", "*.h")) + glob.glob(os.path.join(HERE, "host", "*.cpp")))
    if not all(os.path.exists(b) for b in BINS):
        return True
    newest = max(os.path.getmtime(s) for s in srcs)
    return any(os.path.getmtime(b) < newest for b in BINS)


@pytest.fixture(scope="module")
def host_checks():
    if not os.path.exists(os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang++")):
        pytest.skip("no ROCm clang++")
    if _stale():
        sys.path.insert(0, os.path.join(HERE, "host"))
        import build_checks
        build_checks.build()
    return OUT


def _run(path, leaks):
    env = dict(os.environ, ASAN_OPTIONS=f"detect_leaks={1 if leaks else 0}:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([path], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    return out


def test_admission_bookkeeping_sanitized(host_checks):
    assert "admission checks passed" in _run(BINS[0], leaks=True)


def test_capi_host_paths_sanitized(host_checks):
    assert "C-ABI host checks passed" in _run(BINS[1], leaks=True)
