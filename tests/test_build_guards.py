"""Guards on how the gfx950 library is compiled (CPU only: hipcc
cross-compiles).  Packed FP32 instructions are disabled for the device code,
and no device code may contain one."""
import os
import re
import shutil
import subprocess

import pytest

from paper_0908_3889_amd import build

PACKED = re.compile(r"\bv_pk_(fma|mul|add)_f32\b")


def test_build_disables_packed_fp32():
    src = open(build.__file__).read()
    assert '"-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"' in src
    assert "--offload-arch=gfx950" in src


@pytest.mark.parametrize("source", [os.path.basename(s) for s in build.SOURCES])
def test_device_code_has_no_packed_fp32(source, tmp_path):
    try:
        hipcc = build.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    if shutil.which(hipcc) is None and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = tmp_path / (source + ".s")
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(build.ROOT, "include"), "-I", build.CSRC, "--cuda-device-only",
           "-S", os.path.join(build.CSRC, source), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    asm = out.read_text()
    assert ".amdgcn_target" in asm or "amdgcn" in asm
    hits = PACKED.findall(asm)
    assert not hits, f"{len(hits)} packed FP32 instructions in {source}"
