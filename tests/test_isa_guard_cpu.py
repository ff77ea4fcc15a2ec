"""The static check behind the register-staged sliced kernels (CPU only: the
device compiler and the disassembler run without a GPU).  A kernel that leaves
its accumulation registers to its own 16-byte loads and LDS writes passes; a
kernel whose loaded register the compiler copies before the data has landed
is caught; the generated circuit kernels of the benchmark expression pass."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1108_3126_amd import rx
from paper_1108_3126_amd import workloads as W

CLANG = "/opt/rocm/llvm/bin/clang++"

SRC = r'''
#include <hip/hip_runtime.h>
typedef unsigned int v4 __attribute__((ext_vector_type(4)));
extern "C" __global__ void own_only(const unsigned char* p, unsigned* out) {
    __shared__ unsigned t[256];
    v4 x;
    asm volatile("global_load_dwordx4 %0, %1, off" : "=a"(x) : "v"(p + threadIdx.x * 16) : "memory");
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const unsigned a = (unsigned)(unsigned long long)(__attribute__((address_space(3))) unsigned*)(t + 4 * threadIdx.x);
    asm volatile("ds_write_b128 %0, %1" ::"v"(a), "a"(x) : "memory");
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    out[threadIdx.x] = t[threadIdx.x ^ 1];
}
extern "C" __global__ void copied(const unsigned char* p, unsigned* out) {
    v4 x;
    asm volatile("global_load_dwordx4 %0, %1, off" : "=a"(x) : "v"(p + threadIdx.x * 16) : "memory");
    out[threadIdx.x] = x.x + x.y;   // read by ordinary code with no wait: the compiler copies the AGPRs
}
'''


def _check(code, kernel):
    v = ctypes.c_int32(-1)
    rc = rx.lib().rx_isa_check_staging(code, len(code), b"gfx950", kernel, ctypes.byref(v))
    return rc, v.value, rx.lib().rx_last_error().decode()


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no device compiler")
def test_guard_passes_own_staging_and_catches_a_copy(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text(SRC)
    obj = tmp_path / "k.co"
    subprocess.check_call([CLANG, "-x", "hip", "--offload-arch=gfx950", "--offload-device-only",
                           "--no-gpu-bundle-output", "-O3", "-c", str(src), "-o", str(obj)])
    code = obj.read_bytes()
    rc, v, _ = _check(code, b"own_only")
    assert rc == rx.RX_OK and v == 0
    rc, v, msg = _check(code, b"copied")
    assert rc == rx.RX_OK and v > 0 and "accvgpr" in msg
    rc, _, _ = _check(code, b"no_such_kernel")
    assert rc == rx.RX_EINVAL
    rc, _, _ = _check(b"not an ELF file", b"own_only")
    assert rc == rx.RX_EINVAL


def test_generated_circuit_kernels_pass_the_guard():
    # compiled for gfx950 without a device: the check runs on the code object alone
    for prog, search in ((W.single_program(1), True), (W.small_program(0), False)):
        p = rx.compile(prog.ast, prog.root, prog.classes, search)
        p.jit("gfx950")
        g = p.jit_guard()
        assert g["ran"] == 1 and g["violations"] == [0] * 7 and g["dropped"] == 0, g
