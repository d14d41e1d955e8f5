"""Build the gfx950 shared library libpn.so in-tree.

    python -m paper_0908_3889_amd.build        (or python paper_0908_3889_amd/build.py)

One hipcc invocation for gfx950 only.  Packed FP32 instructions are disabled
for the device code (-packed-fp32-ops), and the resource usage of every
kernel (VGPRs, AGPRs, spills, LDS, occupancy) is written to
build_resource_usage.txt beside the library.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpn.so")
RESOURCE_REPORT = os.path.join(HERE, "build_resource_usage.txt")

SOURCES = [os.path.join(CSRC, "pn_lib.hip"), os.path.join(CSRC, "pn_stats.hip"),
           os.path.join(CSRC, "pn_generate.hip"), os.path.join(CSRC, "pn_probe.hip"),
           os.path.join(CSRC, "pn_order.hip"), os.path.join(CSRC, "pn_check.cpp")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the gfx950 library cannot be built")


def build(verbose: bool = False) -> str:
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Rpass-analysis=kernel-resource-usage",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *SOURCES, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    with open(RESOURCE_REPORT, "w") as f:
        f.write(proc.stderr)
    if proc.returncode != 0:
        sys.stderr.write(proc.stderr)
        raise RuntimeError("hipcc failed building libpn.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


# the sources the integration and adjoint kernels are compiled from
KERNEL_SOURCES = ["pn_lib.hip", "pn_device.hpp", "pn_adjoint.hpp"]


def source_digest() -> str:
    """sha256 over the sources of the integration kernels and the C header
    (file names and bytes), identifying the kernels that a stored counter
    reading was taken on."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES + ["../../include/pn.h"]:
        path = os.path.normpath(os.path.join(CSRC, f))
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def resource_usage() -> dict:
    """Parse build_resource_usage.txt into {kernel: {field: value}}."""
    out: dict = {}
    if not os.path.exists(RESOURCE_REPORT):
        return out
    cur = None
    for line in open(RESOURCE_REPORT):
        if "remark:" not in line:
            continue
        msg = line.split("remark:", 1)[1].strip()
        if msg.startswith("Function Name:"):
            cur = msg.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur is not None and ":" in msg:
            k, v = msg.split(":", 1)
            out[cur][k.strip()] = v.strip().split(" ")[0]
    return out


if __name__ == "__main__":
    build(verbose=True)
    for k, v in resource_usage().items():
        print(k, v)
