"""Control-flow shape of the resident COCG kernel, read from the gfx950
assembly of this source tree (CPU only: hipcc emits it without a device).

Each workgroup of the resident kernel takes work items in a loop: thread 0
fetches the next item with an atomic, a workgroup barrier publishes it, and
the item runs to completion.  The compiler is free to restructure code
around the thread-0 blocks; one such restructuring merged the block that
ends an item with the next item's fetch, so that every other thread looped
straight back to the fetch's barrier and re-read the old item while thread
0 waited to run (the launch never ended).  The loop must stay uniform: its
header fetches and then waits at the barrier, and no loop latch is an
exec-mask latch (a divergent loop around workgroup barriers)."""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_resident_work_loop_is_uniform(tmp_path):
    from paper_2512_01257_amd import build

    src = os.path.join(build.CSRC, "k_cocg.hip")
    out = os.path.join(str(tmp_path), "k_cocg.s")
    flags = [f for f in build.FLAGS if f not in ("-fPIC",)]
    cmd = [_hipcc(), *flags, "--cuda-device-only", "-S", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    asm = open(out).read()
    parts = re.split(r"\n(_ZN7rafeast15k_cocg_resident\S+):", asm)
    kernels = [(parts[i], parts[i + 1][: parts[i + 1].find(".Lfunc_end")])
               for i in range(1, len(parts), 2)]
    # FP32 with 1, 2, 4 or 8 slots and FP64 with 1, 2 or 4, single and batched
    assert len(kernels) == 14
    for name, body in kernels:
        lines = body.split("\n")
        top = next(k for k, ln in enumerate(lines) if "=>This Loop Header: Depth=1" in ln)
        seq = []
        for ln in lines[top + 1:]:
            if "This Loop Header: Depth=2" in ln:
                break
            if "global_atomic_add" in ln:
                seq.append("fetch")
            elif "s_barrier" in ln:
                seq.append("barrier")
        assert seq[:2] == ["fetch", "barrier"], (name, seq)
        latches = [ln for ln in lines if re.search(r"s_andn2_b64\s+exec,\s*exec", ln)]
        assert not latches, (name, latches[:3])
