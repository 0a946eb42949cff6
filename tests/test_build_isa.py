"""Build-time check of the direct-to-LDS BF16x3 kernel's code (CPU only:
hipcc cross-compiles for gfx950): in the multiply phase of every variant
(between the wave's priority raise and its drop) there is no wait on vector
memory counters.  Such a wait makes the multiply of one K step wait for the
next step's loads, which the kernel issues just before it, and serializes the
pipeline (it cost a quarter of the kernel's rate when a refactoring let the
compiler insert one)."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2412_07631_amd", "csrc", "gemm_lds.hip")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_direct_load_kernels_have_no_memory_wait_in_their_multiply_phase():
    with tempfile.TemporaryDirectory() as d:
        cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-Wno-unused-result", "-c", SRC, "-o", os.path.join(d, "g.o"),
               "--save-temps"]
        subprocess.run(cmd, cwd=d, check=True, capture_output=True)
        asm = open(os.path.join(d, "gemm_lds-hip-amdgcn-amd-amdhsa-gfx950.s")).read()
    kernels = list(re.finditer(r"^(_ZN4ctqr17gemm_x3_dl_kernel[^\s:]*):", asm, re.M))
    assert len(kernels) >= 6
    for m in kernels:
        body = asm[m.end():asm.index(".Lfunc_end", m.end())]
        inside, phases, waits = False, 0, 0
        for line in body.splitlines():
            t = line.strip()
            if t.startswith("s_setprio 1"):
                inside, phases = True, phases + 1
            elif t.startswith("s_setprio 0"):
                inside = False
            elif inside and t.startswith("s_waitcnt") and "vmcnt" in t:
                waits += 1
        assert phases >= 1, m.group(1)
        assert waits == 0, "%s: %d vector-memory waits in the multiply phase" % (m.group(1), waits)
