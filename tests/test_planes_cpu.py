"""The plane form of the bit-sliced circuit on the CPU: the gather-and-transpose
code (rx_planes.h) compiled with g++ against a bit-by-bit construction of the
planes, and the generated plane-form circuit (the same source text hiprtc
compiles) driven by those planes over strings of uneven length, against the
oracle.  No GPU: the device build maps the three primitives to single
instructions; here they are plain C."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1108_3126_amd import rx
from paper_1108_3126_amd import workloads as W

CSRC = os.path.join(os.path.dirname(rx.__file__), "csrc")

HOST_PRIMS = r"""
#include <cstdint>
#include <cstddef>
static inline uint32_t pl_perm(uint32_t hi, uint32_t lo, uint32_t sel) {
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    uint32_t r = 0;
    for (int i = 0; i < 4; ++i) r |= (uint32_t)((v >> (8 * ((sel >> (8 * i)) & 7))) & 0xff) << (8 * i);
    return r;
}
static inline uint32_t pl_align(uint32_t hi, uint32_t lo, uint32_t r) {
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * (r & 3)));
}
#define RX_PL_DEV static inline
#define RX_PL_PERM(hi, lo, sel) pl_perm((hi), (lo), (sel))
#define RX_PL_SEL(a, b, m) ((((uint32_t)(a)) & (m)) | (((uint32_t)(b)) & ~(m)))
#define RX_PL_ALIGN(hi, lo, r) pl_align((hi), (lo), (r))
"""

# One slab (up to 2048 strings given by pointers into one buffer): all ticks of
# every lane, laid out as on the device (((t * 9 + q) * 64 + lane) * 4 + r).
SLAB_DRIVER = r"""
#include "rx_planes.h"
extern "C" void slab_planes(const uint8_t* bytes, const int64_t* lo, const int64_t* len, int64_t count,
                            int64_t ticks, uint32_t* out) {
    int64_t minlen = count ? len[0] : 0;
    for (int64_t k = 0; k < count; ++k) if (len[k] < minlen) minlen = len[k];
    if (count < 2048) minlen = 0;   // missing strings have length 0
    for (int lane = 0; lane < 64; ++lane) {
        for (int64_t c = 0; 4 * c < ticks; ++c) {
            uint32_t win[32][4];
            int64_t L[32];
            for (int j = 0; j < 32; ++j) {
                const int64_t k = j * 64 + lane;
                const int64_t o = k < count ? lo[k] : 0, n = k < count ? len[k] : 0;
                L[j] = n;
                rx::planes_window16(bytes + o, n, 16 * c, win[j]);
            }
            for (int kk = 0; kk < 4 && 4 * c + kk < ticks; ++kk) {
                uint32_t w[36];
                const int64_t t = 4 * c + kk;
                rx::planes_tick(win, L, kk, 4 * t, minlen, w);
                for (int q = 0; q < 9; ++q)
                    for (int r = 0; r < 4; ++r) out[((t * 9 + q) * 64 + lane) * 4 + r] = w[4 * q + r];
            }
        }
    }
}
"""


def _build(code, name):
    d = tempfile.mkdtemp(prefix="rxpl")
    cpp, so = os.path.join(d, name + ".cpp"), os.path.join(d, name + ".so")
    open(cpp, "w").write(code)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-w", "-I", CSRC, "-o", so, cpp])
    return ctypes.CDLL(so)


@pytest.fixture(scope="module")
def slab_lib():
    lib = _build(HOST_PRIMS + SLAB_DRIVER, "slab")
    lib.slab_planes.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    return lib


def slab_planes(lib, buf, lo, ln, ticks):
    lo = np.ascontiguousarray(lo, np.int64)
    ln = np.ascontiguousarray(ln, np.int64)
    out = np.zeros(ticks * 9 * 64 * 4, np.uint32)
    lib.slab_planes(buf.ctypes.data, lo.ctypes.data, ln.ctypes.data, len(lo), ticks, out.ctypes.data)
    return out.reshape(ticks, 9, 64, 4)


def naive_planes(buf, lo, ln, ticks):
    """Bit by bit: plane b of position p, lane l, bit j = bit b of string (64 j + l)'s byte p."""
    out = np.zeros((ticks, 9, 64, 4), np.uint64)
    for k in range(len(lo)):
        j, lane = divmod(k, 64)
        for p in range(min(int(ln[k]), 4 * ticks)):
            byte = int(buf[lo[k] + p])
            t, i = divmod(p, 4)
            for b in range(8):
                if (byte >> b) & 1:
                    w = 8 * i + b
                    out[t, w // 4, lane, w % 4] |= 1 << j
            out[t, 8, lane, i] |= 1 << j   # the string has byte p
    return out.astype(np.uint32)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planes_match_bit_by_bit_construction(slab_lib, seed):
    rng = np.random.default_rng(seed)
    count = [2048, 2048, 700][seed]
    ln = np.sort(rng.integers(0, 70, size=count)) if seed != 1 else rng.integers(0, 70, size=count)
    # every string at an odd, unaligned place in one buffer, with foreign bytes in between
    gaps = rng.integers(0, 19, size=count)
    lo = np.zeros(count, np.int64)
    pos = 3
    for k in range(count):
        pos += int(gaps[k])
        lo[k] = pos
        pos += int(ln[k])
    buf = rng.integers(0, 256, size=pos + 64, dtype=np.uint8)
    ticks = (int(ln.max()) + 3) // 4
    got = slab_planes(slab_lib, buf, lo, ln, ticks)
    want = naive_planes(buf, lo, ln, ticks)
    # bytes past a string's end are unspecified in the planes; the valid words must be exact
    valid = want[:, 8]
    assert np.array_equal(got[:, 8], valid)
    for t in range(ticks):
        for w in range(32):
            i = w // 8
            vmask = valid[t, :, i]
            assert np.array_equal(got[t, w // 4, :, w % 4] & vmask, want[t, w // 4, :, w % 4]), (t, w)


CIRCUIT_DRIVER = r"""
#include "rx_planes.h"
// Every slab of the given strings (in order, 2048 per slab) through the
// plane-form circuit: tick by tick, as the device kernel runs it.
extern "C" void run_planes(const uint8_t* bytes, const int64_t* lo, const int64_t* len, int64_t n,
                           unsigned char* out) {
    for (int64_t s0 = 0; s0 < n; s0 += 2048) {
        const int64_t count = n - s0 < 2048 ? n - s0 : 2048;
        int64_t mx = 0;
        for (int64_t k = 0; k < count; ++k) if (len[s0 + k] > mx) mx = len[s0 + k];
        const int64_t ticks = (mx + 3) / 4;
        for (int lane = 0; lane < 64; ++lane) {
            u32 st[RxProg0::NS];
            u32 acc;
            RxProg0::init(st, acc);
            u32 accf = acc;
            for (int64_t c = 0; 4 * c < ticks; ++c) {
                uint32_t win[32][4];
                int64_t L[32];
                for (int j = 0; j < 32; ++j) {
                    const int64_t k = j * 64 + lane;
                    const int64_t o = k < count ? lo[s0 + k] : 0, m = k < count ? len[s0 + k] : 0;
                    L[j] = m;
                    rx::planes_window16(bytes + o, m, 16 * c, win[j]);
                }
                for (int kk = 0; kk < 4 && 4 * c + kk < ticks; ++kk) {
                    u32 w[36];
                    rx::planes_tick(win, L, kk, 4 * (4 * c + kk), 0, w);
                    rx_planes_tick<RxProg0>(st, acc, accf, w);
                }
            }
            for (int j = 0; j < 32; ++j) {
                const int64_t k = j * 64 + lane;
                if (k < count) out[s0 + k] = (unsigned char)((accf >> j) & 1u);
            }
        }
    }
}
"""

PERM_CPU = r"""
static inline unsigned rx_perm_cpu(unsigned hi, unsigned lo, unsigned sel) {
    const unsigned long long v = ((unsigned long long)hi << 32) | lo;
    unsigned r = 0;
    for (int i = 0; i < 4; ++i) r |= (unsigned)((v >> (8 * ((sel >> (8 * i)) & 7))) & 0xff) << (8 * i);
    return r;
}
"""


def planes_circuit(p):
    src = p.jit_planes_source()
    host_part = src.split("// ---- device kernel ----")[0]
    code = ("#define __device__\n#define __forceinline__ inline\n" + PERM_CPU + host_part + HOST_PRIMS +
            CIRCUIT_DRIVER)
    lib = _build(code, "circ")
    lib.run_planes.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_void_p]

    def run(s):
        lo = np.ascontiguousarray(s.offsets[:-1], np.int64)
        ln = np.ascontiguousarray(np.diff(s.offsets), np.int64)
        data = s.data if s.data.size else np.zeros(16, np.uint8)
        out = np.zeros(max(s.n, 1), np.uint8)
        lib.run_planes(data.ctypes.data, lo.ctypes.data, ln.ctypes.data, s.n, out.ctypes.data)
        return out[:s.n]

    return run


def test_plane_circuit_uneven_lengths_against_oracle():
    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, True)
    rng = np.random.default_rng(4)
    member, _ = W.single_strings(prog, seed=44, n=64, length=256, plant_frac=1.0)
    strs = []
    for k in range(3000):
        n = int(rng.integers(0, 300))
        w = bytes(rng.integers(97, 123, size=n, dtype=np.uint8))
        if k % 5 == 0 and n > 0:   # a member of the language inside
            m = member.get(k % 64)
            at = int(rng.integers(0, n + 1))
            w = (w[:at] + m + w[at:])
        strs.append(w)
    s = W.pack(strs)
    got = planes_circuit(p)(s)
    want = oracle.match(prog.ast, prog.root, prog.classes, True, s.data, s.offsets, threads=4)
    assert got.sum() > 300 and np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(6))
def test_plane_circuit_small_anchored_programs(seed):
    prog = W.small_program(seed)
    p = rx.compile(prog.ast, prog.root, prog.classes, False)
    s = W.small_strings(seed, n=2500)
    got = planes_circuit(p)(s)
    want = oracle.match(prog.ast, prog.root, prog.classes, False, s.data, s.offsets, threads=4)
    assert np.array_equal(got, want)


SPEC_DRIVER = r"""
#include "rx_planes.h"
#include <vector>
// The split run of a long slab (the device kernel's wavefronts), all 64 lanes
// in lockstep: the slab's T ticks cut into ws segments of at least 64 ticks;
// segment i run from the start state (the first from the start), keeping its
// state after 4, 8, 16, 32 ticks; each run goes on past its segment and stops
// at the first kept state of the next run that equals its own for every
// string of every lane (the device's ballot) that has bytes left and is not
// in the search suffix's loop.  A string takes the accept bit of the run that
// holds the true state at its last byte, or accepts if a run stopped with it
// in the suffix loop.
extern "C" int run_planes_spec(const uint8_t* bytes, const int64_t* lo, const int64_t* len, int64_t n,
                               unsigned char* out, int64_t* stopped) {
    const int NS = RxProg0::NS, NCP = RxProg0::NCP;
    *stopped = 0;
    for (int64_t s0 = 0; s0 < n; s0 += 2048) {
        const int64_t count = n - s0 < 2048 ? n - s0 : 2048;
        int64_t mx = 0;
        for (int64_t k = 0; k < count; ++k) if (len[s0 + k] > mx) mx = len[s0 + k];
        const int64_t T = (mx + 3) / 4;
        // every tick of every lane
        std::vector<u32> W((size_t)(T > 0 ? T : 1) * 64 * 36);
        for (int lane = 0; lane < 64; ++lane)
            for (int64_t c = 0; 4 * c < T; ++c) {
                uint32_t win[32][4];
                int64_t L[32];
                for (int j = 0; j < 32; ++j) {
                    const int64_t k = j * 64 + lane;
                    const int64_t o = k < count ? lo[s0 + k] : 0, m = k < count ? len[s0 + k] : 0;
                    L[j] = m;
                    rx::planes_window16(bytes + o, m, 16 * c, win[j]);
                }
                for (int kk = 0; kk < 4 && 4 * c + kk < T; ++kk) {
                    uint32_t w[36];
                    rx::planes_tick(win, L, kk, 4 * (4 * c + kk), 0, w);
                    for (int i = 0; i < 36; ++i) W[((size_t)(4 * c + kk) * 64 + lane) * 36 + i] = w[i];
                }
            }
        auto valid = [&](int lane, int64_t t) { return t < T ? W[((size_t)t * 64 + lane) * 36 + 32] : 0u; };
        int ws = RxProg0::SPEC && NCP > 0 ? RxProg0::NW : 1;
        while (ws > 1 && T < 64 * ws) ws >>= 1;
        const int64_t seg = T / ws;
        // one run: every lane's state, from tick `from`
        struct Run {
            std::vector<u32> S, acc, accf;
        };
        auto start_run = [&](bool first) {
            Run R;
            R.S.assign((size_t)64 * NS, 0u);
            R.acc.assign(64, 0u);
            R.accf.assign(64, 0u);
            for (int lane = 0; lane < 64; ++lane) {
                u32 st[RxProg0::NS];
                RxProg0::init(st, R.acc[lane]);
                for (int k = 0; k < NS; ++k) R.S[(size_t)lane * NS + k] = st[k];
                R.accf[lane] = first ? R.acc[lane] : 0u;
            }
            return R;
        };
        auto step_run = [&](Run& R, int64_t t) {
            for (int lane = 0; lane < 64; ++lane) {
                u32 st[RxProg0::NS];
                for (int k = 0; k < NS; ++k) st[k] = R.S[(size_t)lane * NS + k];
                u32 ww[36];
                for (int i = 0; i < 36; ++i) ww[i] = W[((size_t)t * 64 + lane) * 36 + i];
                rx_planes_tick<RxProg0>(st, R.acc[lane], R.accf[lane], ww);
                for (int k = 0; k < NS; ++k) R.S[(size_t)lane * NS + k] = st[k];
            }
        };
        // kept states of runs 1 .. ws - 1
        std::vector<std::vector<u32>> kept((size_t)ws * (NCP > 0 ? NCP : 1));
        for (int i = 1; i < ws; ++i) {
            Run R = start_run(false);
            for (int64_t t = i * seg, c = 0; c < NCP; ++t) {
                step_run(R, t);
                if (t + 1 - i * seg == (4ll << c)) kept[(size_t)i * NCP + c++] = R.S;
            }
        }
        std::vector<u32> res(64, 0u), live(64, 0xffffffffu);
        for (int i = 0; i < ws; ++i) {
            Run R = start_run(i == 0);
            const int64_t next = i + 1 < ws ? (i + 1) * seg : T;
            bool same = false;
            int64_t t = i * seg;
            for (; t < next; ++t) step_run(R, t);
            std::vector<u32> vn(64, 0u), su(64, 0u);
            if (i + 1 < ws) {
                for (int c = 0; c < NCP && !same; ++c) {
                    for (; t < next + (4ll << c) && t < T; ++t) step_run(R, t);
                    if (t >= T) break;
                    bool all = true;
                    for (int lane = 0; lane < 64; ++lane) {
                        const u32 v = valid(lane, t);
                        const u32 sure = RxProg0::SUF >= 0 ? R.S[(size_t)lane * NS + (RxProg0::SUF >= 0 ? RxProg0::SUF : 0)] : 0u;
                        for (int k = 0; k < NS; ++k)
                            if ((R.S[(size_t)lane * NS + k] ^ kept[(size_t)(i + 1) * NCP + c][(size_t)lane * NS + k]) & v & ~sure)
                                all = false;
                        vn[lane] = v;
                        su[lane] = sure;
                    }
                    if (all) {
                        same = true;
                        *stopped += 1 + 100 * (c + 1);
                    }
                }
                if (!same)
                    for (; t < T; ++t) step_run(R, t);
            }
            if (!same) {
                for (int lane = 0; lane < 64; ++lane) res[lane] |= R.accf[lane] & live[lane];
                break;
            }
            for (int lane = 0; lane < 64; ++lane) {
                res[lane] |= (R.accf[lane] & live[lane] & ~vn[lane]) | (su[lane] & vn[lane] & live[lane]);
                live[lane] &= vn[lane] & ~su[lane];
            }
        }
        for (int lane = 0; lane < 64; ++lane)
            for (int j = 0; j < 32; ++j) {
                const int64_t k = j * 64 + lane;
                if (k < count) out[s0 + k] = (unsigned char)((res[lane] >> j) & 1u);
            }
    }
    return 1;
}
"""


def spec_circuit(p):
    src = p.jit_planes_source()
    host_part = src.split("// ---- device kernel ----")[0]
    code = ("#define __device__\n#define __forceinline__ inline\n" + PERM_CPU + host_part + HOST_PRIMS + SPEC_DRIVER)
    lib = _build(code, "spec")
    lib.run_planes_spec.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]

    def run(s):
        lo = np.ascontiguousarray(s.offsets[:-1], np.int64)
        ln = np.ascontiguousarray(np.diff(s.offsets), np.int64)
        data = s.data if s.data.size else np.zeros(16, np.uint8)
        out = np.zeros(max(s.n, 1), np.uint8)
        stopped = ctypes.c_int64()
        lib.run_planes_spec(data.ctypes.data, lo.ctypes.data, ln.ctypes.data, s.n, out.ctypes.data,
                            ctypes.byref(stopped))
        return out[:s.n], stopped.value

    return run, src


@pytest.mark.parametrize("k", [3, 5, 7, 12, 13, 15])
def test_split_long_slab_against_oracle(k):
    """A long slab of a searched program cut into segments run side by side (each run stopping where its
    state equals a kept state of the next) gives the oracle's bits; lines of 300-2,000 bytes of the
    batched workload's kind, and a slab too short to split."""
    prog = W.multi_programs(seed=2)[k]
    p = rx.compile(prog.ast, prog.root, prog.classes, True)
    run, src = spec_circuit(p)
    assert "SPEC = true" in src
    s = W.multi_lines(seed=30 + k, n=2048 * 40, hi=2000)
    lens = np.diff(s.offsets)
    keep = np.nonzero(lens >= 300)[0][:4096]
    short = np.nonzero((lens > 20) & (lens < 200))[0][:2048]
    s = W.pack([bytes(s.data[s.offsets[i]:s.offsets[i + 1]]) for i in np.concatenate([keep, short])])
    got, stopped = run(s)
    want = oracle.match(prog.ast, prog.root, prog.classes, True, s.data, s.offsets, threads=8)
    print(f"program {k}: meetings {stopped % 100}, kept-state index sum {stopped // 100}; accepted {int(want.sum())}",
          flush=True)
    assert stopped % 100 > 0
    assert np.array_equal(got, want)
