"""The host layer under AddressSanitizer and UndefinedBehaviorSanitizer: the
C-ABI tests of test_abi_cpu.py (argument checks, size queries, error paths; no
GPU needed) run again against a build of the same sources whose host code is
instrumented, in a child process with the sanitizer runtime preloaded.  Any
sanitizer report (out-of-bounds access, use after free, undefined behaviour
such as an out-of-range enum value) fails the test.

The instrumented library is built under paper_1401_2039_amd/_build/asan and
reused while the sources and flags are unchanged (a build takes a few
minutes)."""
import hashlib
import os
import shutil
import subprocess
import sys

import pytest

from paper_1401_2039_amd import build

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(build.BUILD_DIR, "asan")

pytestmark = pytest.mark.skipif(not os.path.exists(build.HIPCC) and shutil.which("hipcc") is None,
                                reason="hipcc not available")


def source_stamp():
    h = hashlib.sha256()
    for path in build.sources() + sorted(os.path.join(build.CSRC, f) for f in os.listdir(build.CSRC)
                                         if f.endswith(".h")) + [os.path.join(ROOT, "include", "qiral.h")]:
        h.update(path.encode())
        with open(path, "rb") as f:
            h.update(f.read())
    h.update(" ".join(build.CFLAGS + build.SAN_FLAGS).encode())
    return h.hexdigest()


@pytest.fixture(scope="module")
def sanitized_lib():
    rt = build.asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime next to the compiler")
    stamp_path = os.path.join(OUT, "stamp")
    lib = os.path.join(OUT, "libqiral_hip.so")
    stamp = source_stamp()
    fresh = os.path.exists(lib) and os.path.exists(stamp_path) and open(stamp_path).read() == stamp
    if not fresh:
        build.build_sanitized(OUT)
        with open(stamp_path, "w") as f:
            f.write(stamp)
    return lib, rt


def test_abi_under_asan_and_ubsan(sanitized_lib):
    lib, rt = sanitized_lib
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, QIRAL_LIB_PATH=lib,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(HERE, "test_abi_cpu.py"), "-q", "-p", "no:cacheprovider",
           "-m", "not gpu"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out and "failed" not in out, out[-2000:]
