"""The host side of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer: the ABI's validation tests and the RCM ordering
tests run in a child process against the instrumented build of the library
(the sanitizer runtime preloaded), and any report ends that process with an
error.  CPU only: no test in the child touches a device."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_abi_and_rcm_clean_under_asan_ubsan(tmp_path):
    from paper_2512_01257_amd import build_sanitize as bs

    lib = bs.build(outdir=str(tmp_path))
    env = dict(os.environ)
    env.update(
        LD_PRELOAD=bs.asan_runtime(),
        RAFEAST_LIB=lib,
        # the interpreter itself is not instrumented and keeps memory to the
        # end, so leak reports would be about Python, not the library
        ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
        UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
        # the child sees no device even where one is installed
        HIP_VISIBLE_DEVICES="",
    )
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_capi.py"), os.path.join(ROOT, "tests", "test_rcm.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in out and "failed" not in out
