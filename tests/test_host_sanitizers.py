"""The host side of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer: the argument checks, workspace queries, contour
nodes, error strings and tuning-file parsing of test_abi.py run in a child
process against the sanitized build of the library (libfeastband_asan.so,
host code instrumented, device code never run from it) with the ASan
runtime preloaded; any sanitizer report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_code_clean_under_asan_and_ubsan():
    from paper_2012_00506_amd import build as b
    rt = b.asan_runtime()
    if not os.path.exists(b.OUT_SAN):
        pytest.skip("sanitized library not built (paper_2012_00506_amd.build --asan)")
    if rt is None:
        pytest.skip("no clang ASan runtime in this image")
    env = dict(os.environ, FEASTBAND_LIB=b.OUT_SAN, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    probe = ("import paper_2012_00506_amd._native as N; N.lib(); "
             "maps = open('/proc/self/maps').read(); "
             "print(N.LIB_PATH, 'libclang_rt.asan' in maps, 'libfeastband_asan' in maps)")
    r = subprocess.run([sys.executable, "-c", probe], env=env, capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-3000:]
    assert r.stdout.split()[1:] == ["True", "True"], r.stdout
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       env=env, capture_output=True, text=True, timeout=600, cwd=ROOT)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
