"""Builds the HIP library ``librx.so`` in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "librx.so")
SOURCES = ["rx_compile.cpp", "rx_api.cpp", "rx_kernels.hip"]
EXTRA_SOURCES_FILE = os.path.join(CSRC, "SOURCES")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def sources():
    srcs = list(SOURCES)
    if os.path.exists(EXTRA_SOURCES_FILE):
        for line in open(EXTRA_SOURCES_FILE):
            line = line.strip()
            if line and not line.startswith("#") and line not in srcs:
                srcs.append(line)
    return [os.path.join(CSRC, s) for s in srcs]


def build(verbose: bool = False) -> str:
    """Compile every source into paper_1108_3126_amd/librx.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", *sources(),
           "-o", tmp, "-lhiprtc", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build librx.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
