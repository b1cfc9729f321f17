"""The host half of the library (reordering, planning, block features, the learned rank
allocation, argument checks of the C-ABI) under AddressSanitizer and UndefinedBehaviorSanitizer:
the sanitizer build (build.py --sanitize) is loaded into a child Python with the shared
sanitizer runtime preloaded, and the host-library and rank tests must pass there with no report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2011_04235_amd")


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    csrc = os.path.join(PKG, "csrc")
    srcs = [os.path.join(csrc, f) for f in os.listdir(csrc)] + [os.path.join(ROOT, "include", "fastpi.h")]
    return any(os.path.getmtime(s) > t for s in srcs)


def test_host_code_clean_under_asan_and_ubsan():
    sys.path.insert(0, PKG)
    import build as b
    try:
        b.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    if _stale(b.SAN_OUT):
        b.build(sanitize=True)
    rt = b.sanitizer_runtime()
    assert os.path.exists(rt), rt
    env = dict(os.environ, FASTPI_LIBRARY=b.SAN_OUT, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_host_library.py"), os.path.join(ROOT, "tests", "test_rank_host.py")]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
