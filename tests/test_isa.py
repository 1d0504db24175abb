"""The gfx950 code built from the HIP sources never writes through the scalar data cache (no
scalar stores, scalar atomics, or scalar-cache write-back/discard) and contains no packed FP32
arithmetic, and the stage kernels the library runs by default do not spill registers to scratch;
all are checked on the AMD assembly of this repository's own kernels."""
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


@pytest.fixture(scope="module")
def assembly(tmp_path_factory):
    """The gfx950 assembly of a HIP source, compiled once per test module."""
    cache = {}

    def get(src):
        if src not in cache:
            out = tmp_path_factory.mktemp("isa") / (src + ".s")
            cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-I",
                   os.path.join(ROOT, "include"), "-I", CSRC, "-Xclang", "-target-feature",
                   "-Xclang", "-packed-fp32-ops", "-x", "hip", "--cuda-device-only", "-S",
                   os.path.join(CSRC, src), "-o", str(out)]
            subprocess.run(cmd, check=True, capture_output=True)
            cache[src] = out.read_text()
        return cache[src]
    return get


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", hip_sources())
def test_no_scalar_stores_or_packed_fp32(src, assembly):
    text = assembly(src)
    assert "gfx950" in text
    bad = FORBIDDEN.findall(text)
    assert not bad, bad


KERNEL_META = re.compile(r"\.name:\s*(\S+).*?\.private_segment_fixed_size:\s*(\d+)", re.S)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("src", ["stage_march.hip", "stage_march_gen.hip", "stage_tile.hip"])
def test_stage_kernels_do_not_spill(src, assembly):
    """Every stage kernel instance that the library picks by default holds its state in
    registers: the row-marching kernel under its 2-waves-per-SIMD budget (the 3-waves instances
    spill by construction and are only autotuner candidates) and every LDS tile."""
    text = assembly(src)
    names = subprocess.run(["c++filt"], input="\n".join(m.group(1) for m in KERNEL_META.finditer(text)),
                           capture_output=True, text=True, check=True).stdout.splitlines()
    checked, spills = 0, []
    for name, m in zip(names, KERNEL_META.finditer(text)):
        if "stage_march<" in name:
            # template arguments: precision, norm, BDF order, last stage, waves per SIMD, ...
            args = name[name.index("<") + 1:name.index(">(")].split(", ")
            if args[4] != "2":
                continue
        elif "stage_tile<" not in name:
            continue
        checked += 1
        if int(m.group(2)) != 0:
            spills.append((name, int(m.group(2))))
    assert checked > 0
    assert not spills, spills
