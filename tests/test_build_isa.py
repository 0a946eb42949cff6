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


def _scratch_sizes(srcs):
    """ScratchSize of every ctqr kernel in the gfx950 code of the given
    sources, compiled in parallel."""
    sizes = {}
    with tempfile.TemporaryDirectory() as d:
        procs = []
        for s in srcs:
            out = os.path.join(d, s.replace(".hip", ".s"))
            cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
                   "-Xclang", "-packed-fp32-ops", "-Wno-unused-result", "--cuda-device-only", "-S",
                   os.path.join(ROOT, "paper_2412_07631_amd", "csrc", s), "-o", out]
            procs.append((out, subprocess.Popen(cmd, cwd=d, stdout=subprocess.PIPE, stderr=subprocess.PIPE)))
        for out, p in procs:
            assert p.wait() == 0, p.stderr.read().decode()[-2000:]
            asm = open(out).read()
            for m in re.finditer(r"^(_ZN4ctqr[^\s:]*):", asm, re.M):
                end = asm.index(".Lfunc_end", m.end())
                meta = re.search(r"; ScratchSize: (\d+)", asm[end:end + 4000])
                if meta:
                    sizes[m.group(1)] = int(meta.group(1))
    return sizes


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_solve_and_panel_kernels_keep_their_arrays_in_registers():
    """No private-memory (scratch) use where it was removed or measured to
    cost: the fused solve's FP32 kernel (variants that spilled were slower or
    were not run), the FP32 diagonal step of the triangular solves, and the
    two-reduction panel (a dynamic index into a private row once put 280 bytes
    there; 8 bytes remain, the call frame of its Cholesky and LU helpers)."""
    sizes = _scratch_sizes(["fused.hip", "solve.hip", "panel.hip"])
    fused = [k for k in sizes if "fused_solve_kernelIf" in k]
    diag = [k for k in sizes if "diag_f32_kernel" in k]
    cqr = [k for k in sizes if "panel_cqr_kernel" in k]
    assert fused and diag and len(cqr) == 2
    for k in fused + diag:
        assert sizes[k] == 0, "%s: %d bytes of scratch" % (k, sizes[k])
    for k in cqr:
        assert sizes[k] <= 8, "%s: %d bytes of scratch" % (k, sizes[k])
