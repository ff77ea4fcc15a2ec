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


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source into paper_1108_3126_amd/librx.so (always rebuilds): one object per source,
    compiled in parallel, then one link."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    inc = [f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda so: _run([HIPCC, *FLAGS, *inc, "-c", so[0], "-o", so[1]], verbose),
                              zip(srcs, objs)))
    for src, res in zip(srcs, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)}")
    tmp = LIB + ".tmp"
    res = _run([HIPCC, *FLAGS, "-shared", *objs, "-o", tmp, "-lhiprtc", "-lpthread"], verbose)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to link librx.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
