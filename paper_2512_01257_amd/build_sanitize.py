"""Builds a variant of librafeast.so whose host code is instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (device code is compiled as
usual), by default under _build/sanitize/.  The CPU tests of the ABI's validation paths
and of the RCM ordering run against it (RAFEAST_LIB selects it, the
sanitizer runtime is preloaded); no GPU run uses it.
"""

from __future__ import annotations

import glob
import os

from paper_2512_01257_amd import build as _b

# every sanitizer option is scoped to the host pass
_HOST = ["address", "undefined"]
COMPILE = [f for s in _HOST for f in ("-Xarch_host", "-fsanitize=" + s)] + [
    "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
LINK = [f for s in _HOST for f in ("-Xarch_host", "-fsanitize=" + s)] + ["-shared-libsan"]
OUTDIR = os.path.join(_b.BUILD, "sanitize")
LIB = os.path.join(OUTDIR, "librafeast.so")


def asan_runtime() -> str:
    """The AddressSanitizer runtime of the HIP compiler's LLVM (to preload)."""
    for cand in sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")):
        return cand
    raise RuntimeError("libclang_rt.asan-x86_64.so not found")


def build(jobs: int = 8, outdir: str = OUTDIR) -> str:
    """Objects and librafeast.so in outdir; returns the library's path."""
    return _b.build(jobs, outdir, os.path.join(outdir, "librafeast.so"), COMPILE, LINK)


if __name__ == "__main__":
    print(build())
