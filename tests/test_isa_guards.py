"""Guards on the gfx950 assembly of our own kernels (compiled here with the
build's flags): no packed-FP32 instructions (the build disables them), and
no mixed-precision FMA writing FP16 (it would round a sum once instead of
the documented FP32 rounding followed by FP16 rounding)."""
import os
import re
import subprocess

import pytest

from paper_2309_08864_amd import build as B

KERNEL_SOURCES = ["kernels_f32.hip", "kernels_f64.hip", "kernels_bf16.hip", "kernels_f16.hip"]


def _asm(src, tmp_path):
    out = tmp_path / (src + ".s")
    cmd = [B.HIPCC, "-x", "hip"] + B.COMMON + ["-S", "--cuda-device-only",
                                              os.path.join(B.CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"hipcc unavailable or failed: {r.stderr[-300:]}")
    return out.read_text()


@pytest.mark.parametrize("src", KERNEL_SOURCES)
def test_no_packed_fp32_and_no_fp16_fma_mix(src, tmp_path):
    asm = _asm(src, tmp_path)
    assert re.search(r"\bv_pk_(fma|mul|add)_f32\b", asm) is None
    assert re.search(r"\bv_fma_mix(lo|hi)_f16\b", asm) is None
    # the kernels are there
    assert "tb_kernel" in asm
