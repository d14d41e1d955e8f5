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


def _resources(pattern):
    res = build.resource_usage()
    if not res:
        pytest.skip("library not built (no resource report)")
    hits = {k: v for k, v in res.items() if pattern in k}
    assert hits, pattern
    return hits


def test_hot_kernels_keep_their_register_budget():
    """The FP64 integration kernel runs at 2 waves per SIMD with at most the
    12 B of scratch its refill-pass constant takes; the backward kernel of
    the adjoint fits its registers without scratch (a regression here is the
    compiler deferring the row-adjoint updates again)."""
    for name, r in _resources("integrate_persistent_f64ILi256ELb0E").items():
        assert int(r["Occupancy [waves/SIMD]"]) == 2, name
        assert int(r["ScratchSize [bytes/lane]"]) <= 12, name
    for name, r in _resources("adjoint_kernelILi128").items():
        assert int(r["ScratchSize [bytes/lane]"]) == 0, name
        assert int(r["VGPRs Spill"]) == 0, name
        assert int(r["LDS Size [bytes/block]"]) <= 80 * 1024, name
    for name, r in _resources("integrate_persistent_f32sILi256E").items():
        assert int(r["Occupancy [waves/SIMD]"]) == 3 and int(r["ScratchSize [bytes/lane]"]) == 0, name
