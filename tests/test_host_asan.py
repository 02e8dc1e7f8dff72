"""The host code of libdeskew.so under AddressSanitizer: the host-only ABI
checks (Eq. 1, the frame, the view and affine plans, argument validation
of every entry point) run in a child process against the ASan build of
the library, with the sanitizer runtime preloaded.  Any invalid host
memory access aborts the child with a report.  No kernel is launched."""
import os
import subprocess
import sys

import pytest

from paper_2211_00645_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    srcs = [os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC)] + \
        [os.path.join(B.INCLUDE, f) for f in os.listdir(B.INCLUDE)]
    return any(os.path.getmtime(p) > t for p in srcs)


def test_host_abi_checks_clean_under_asan():
    rt = B.asan_runtime()
    if not rt:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    if _stale(B.LIB_ASAN):
        B.build(asan=True)
    env = dict(os.environ, DSK_LIB=B.LIB_ASAN, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_abi_host.py")]
    out = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout[-3000:] + out.stderr[-3000:]
    assert "AddressSanitizer" not in out.stderr
    assert "passed" in out.stdout
