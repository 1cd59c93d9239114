"""Register and LDS budgets of the Voigt kernels (host only: device code is
compiled to gfx950 assembly and its kernel metadata read).

The FP32 kernel's speed rests on six waves per SIMD: at most 80 VGPRs, no
spills, and at most 26 KB of LDS per 256-thread workgroup (six workgroups in
the 160 KB of a CU).  The FP64 kernel runs four waves per SIMD (at most 128
VGPRs).  A change that breaks these budgets compiles and computes the same
numbers, so only this test notices it.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2105_13611_amd import build as B


def _kernel_metadata(asm_text):
    """Map kernel name -> dict of the integer fields of its metadata block."""
    meta = asm_text[asm_text.index(".amdgpu_metadata"):]
    out = {}
    for block in re.split(r"\n\s+- \.agpr_count:", meta)[1:]:
        name = re.search(r"\.name:\s+(\S+)", block)
        if not name:
            continue
        fields = {k: int(v) for k, v in re.findall(r"\.([a-z_]+):\s+(\d+)\s*$", block, re.M)}
        out[name.group(1)] = fields
    return out


@pytest.fixture(scope="module")
def voigt_metadata(tmp_path_factory):
    cc = B.hipcc()
    if not shutil.which(cc) and not os.path.exists(cc):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm") / "k_voigt.s"
    cmd = [cc] + B.flags() + ["-x", "hip", "--cuda-device-only", "-S",
                              os.path.join(B.CSRC, "k_voigt.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return _kernel_metadata(out.read_text())


def _find(meta, short):
    hits = [v for k, v in meta.items() if short in k]
    assert len(hits) == 1, (short, list(meta))
    return hits[0]


def test_voigt32_six_waves_per_simd(voigt_metadata):
    m = _find(voigt_metadata, "k_voigt32")
    assert m["vgpr_count"] <= 80, m
    assert m["vgpr_spill_count"] == 0, m
    assert m["sgpr_spill_count"] == 0, m
    assert m["private_segment_fixed_size"] == 0, m
    assert m["group_segment_fixed_size"] <= 26 * 1024, m
    assert 6 * m["group_segment_fixed_size"] <= 160 * 1024, m
    assert m["max_flat_workgroup_size"] == 256, m


def test_voigt64_four_waves_per_simd(voigt_metadata):
    m = _find(voigt_metadata, "k_voigt64")
    assert m["vgpr_count"] <= 128, m
    assert m["group_segment_fixed_size"] <= 40 * 1024, m
    assert m["max_flat_workgroup_size"] == 256, m
