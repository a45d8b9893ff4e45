"""The step kernels compile without register spills.

The fused step keeps two planes of 27 (f, g) pairs in flight per thread, so
its register budget is tight: a spill to scratch memory costs far more than
the arithmetic it saves.  Every compiled instantiation must use no scratch
(the 512-thread 64 x 8 shape exists for FP32 storage only: with FP64
populations it would spill, so it is not compiled).  Compiles the kernel
source for gfx950 on the host (device code only, about half a minute)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_09512_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _resources(tmp_path):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "--cuda-device-only",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Rpass-analysis=kernel-resource-usage",
           "-c", os.path.join(CSRC, "lbm_kernels.hip"), "-o", str(tmp_path / "k.o")]
    out = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stderr[-2000:]
    kernels, name = {}, None
    for line in out.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            kernels[name] = {}
            continue
        m = re.search(r"remark:\s+(.+?): (\d+)", line)
        if m and name:
            kernels[name][m.group(1).strip()] = int(m.group(2))
    return kernels


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_step_kernels_do_not_spill(tmp_path):
    kernels = _resources(tmp_path)
    # Itanium mangling: step_kernel<D, DEV, S, BX, BY, ...> -> ...ILi3ELb1EfLi64ELi8E...
    pat = re.compile(r"(?:step_kernel|batch_step_kernel|batch_persistent_kernel|pattern_kernel)"
                     r"ILi(\d)ELb(\d)E([fd])Li(\d+)ELi(\d+)E")
    seen = 0
    for name, res in kernels.items():
        m = pat.search(name)
        if not m:
            continue
        D, _, S, bx, by = m.groups()
        seen += 1
        assert not (D == "3" and S == "d" and (bx, by) == ("64", "8")), name
        assert res.get("ScratchSize [bytes/lane]", -1) == 0, (name, res)
        if (D, S, bx, by) == ("3", "f", "64", "8"):
            assert res.get("Occupancy [waves/SIMD]", 0) >= 2, (name, res)
    assert seen >= 36, f"only {seen} step kernels found"
