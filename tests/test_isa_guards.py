"""Guards on the gfx950 assembly of our own kernels, as built by the
package's build step: no packed-FP32 instructions (the build disables them),
and no mixed-precision FMA writing FP16 (it would round a sum once instead of
the documented FP32 rounding followed by FP16 rounding).  The device code
objects are taken out of the built objects and disassembled with the LLVM
tools of the ROCm install."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2309_08864_amd import build as B

LLVM = "/opt/rocm/llvm/bin/llvm-objdump"
# every kernel object the build compiles: kernels.hip once per storage type
KERNEL_OBJECTS = [e[2] for e in B.SOURCES if e[0] == "kernels.hip"]


def _asm(objname, tmp_path):
    obj = os.path.join(B.OBJ, objname)
    if not os.path.exists(obj) or not os.path.exists(LLVM):
        pytest.skip("library not built here, or no llvm-objdump")
    local = tmp_path / objname
    shutil.copy(obj, local)
    subprocess.run([LLVM, "--offloading", str(local)], cwd=tmp_path, check=True,
                   capture_output=True)
    dev = [f for f in os.listdir(tmp_path) if f.startswith(objname + ".") and "gfx950" in f]
    assert len(dev) == 1, f"no gfx950 code object in {objname}: {os.listdir(tmp_path)}"
    r = subprocess.run([LLVM, "-d", str(tmp_path / dev[0])], capture_output=True, text=True,
                       check=True)
    return r.stdout


@pytest.mark.parametrize("objname", KERNEL_OBJECTS)
def test_no_packed_fp32_and_no_fp16_fma_mix(objname, tmp_path):
    asm = _asm(objname, tmp_path)
    assert re.search(r"\bv_pk_(fma|mul|add)_f32\b", asm) is None
    assert re.search(r"\bv_fma_mix(lo|hi)_f16\b", asm) is None
    # the kernels are there
    assert "tb_kernel" in asm and "march3d_kernel" in asm
