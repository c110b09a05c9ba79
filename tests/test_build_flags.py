"""The library's build flags switch packed FP32 arithmetic off in device code.

hipcc's host pass warns that it does not know the `-packed-fp32-ops` target feature; the
gfx950 device pass takes it.  This checks the device assembly of a small kernel whose
float2 arithmetic the compiler packs by default: with the library's flags it holds no packed
FP32 instruction, without them it does (so the check can fail)."""
from __future__ import annotations

import os
import re
import shutil
import subprocess

import pytest

from paper_1807_03749_amd import build

KERNEL = r"""
#include <hip/hip_runtime.h>
__global__ void axpb(float2 *a, float2 b)
{
    const int i = threadIdx.x;
    float2 x = a[i];
    x.x = x.x * b.x + b.y;
    x.y = x.y * b.x + b.y;
    a[i] = x;
}
"""
PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")


def device_asm(tmp_path, flags):
    src = tmp_path / "k.hip"
    src.write_text(KERNEL)
    out = tmp_path / "k.s"
    keep = [f for f in flags if f not in ("-shared", "-fPIC")]
    subprocess.run([build.HIPCC, *keep, "--cuda-device-only", "-S", "-o", str(out), str(src)], check=True,
                   capture_output=True)
    return out.read_text()


@pytest.mark.skipif(not os.path.exists(build.HIPCC) and shutil.which("hipcc") is None, reason="no hipcc")
def test_packed_fp32_is_off_in_device_code(tmp_path):
    assert "-packed-fp32-ops" in build.FLAGS
    with_flags = device_asm(tmp_path, build.FLAGS)
    assert not PACKED.search(with_flags)
    i = build.FLAGS.index("-packed-fp32-ops")
    plain = build.FLAGS[: i - 3] + build.FLAGS[i + 1:]  # drop "-Xclang -target-feature -Xclang -packed-fp32-ops"
    assert "-packed-fp32-ops" not in plain
    assert PACKED.search(device_asm(tmp_path, plain)), "the probe kernel no longer packs by default"
