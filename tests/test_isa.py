"""The gfx950 code built from the HIP sources never writes through the scalar data cache (no
scalar stores, scalar atomics, or scalar-cache write-back/discard) and contains no packed FP32
arithmetic; both are checked on the AMD assembly of this repository's own kernels."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_08769_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

FORBIDDEN = re.compile(r"^\s*(s_store|s_atomic|s_buffer_store|s_scratch_store|s_dcache_wb|"
                       r"s_dcache_discard|v_pk_add_f32|v_pk_mul_f32|v_pk_fma_f32)\b", re.M)


def hip_sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", hip_sources())
def test_no_scalar_stores_or_packed_fp32(src, tmp_path):
    out = tmp_path / (src + ".s")
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-x", "hip",
           "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    text = out.read_text()
    assert "gfx950" in text
    bad = FORBIDDEN.findall(text)
    assert not bad, bad
