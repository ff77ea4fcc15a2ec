"""The generated bit-sliced circuit, compiled for the host CPU with g++ and run
on fixed-length strings, against the CPU oracle.  This checks the circuit
derivation, the label decoder and the 32x32 bit transpose without a GPU; the
same source text is what hiprtc compiles for gfx950."""
import ctypes
import os
import subprocess
import tempfile
import time

import numpy as np
import pytest

import oracle
from paper_1108_3126_amd import rx
from paper_1108_3126_amd import workloads as W

# v_perm_b32 on the host: byte i of the result is byte sel[i] of the 64-bit value {hi, lo}
PERM_CPU = r"""
static inline unsigned rx_perm_cpu(unsigned hi, unsigned lo, unsigned sel) {
    const unsigned long long v = ((unsigned long long)hi << 32) | lo;
    unsigned r = 0;
    for (int i = 0; i < 4; ++i) r |= (unsigned)((v >> (8 * ((sel >> (8 * i)) & 7))) & 0xff) << (8 * i);
    return r;
}
#define RX_PERM(hi, lo, sel) rx_perm_cpu((hi), (lo), (sel))
#define RX_SEL(a, b, m) ((((unsigned)(a)) & (m)) | (((unsigned)(b)) & ~(m)))
"""

DRIVER = r"""
extern "C" int rx_cpu_run(const unsigned char* bytes, long long length, long long n, unsigned char* out) {
    for (long long g = 0; g < n; g += 32) {
        u32 s[RX_NS];
        u32 acc;
        rx_init(s, acc);
        for (long long p = 0; p < length; p += 4) {
            u32 w[32];
            for (int j = 0; j < 32; ++j) {
                const long long sid = g + j < n ? g + j : n - 1;
                u32 v = 0;
                for (int k = 0; k < 4; ++k)
                    if (p + k < length) v |= (u32)bytes[sid * length + p + k] << (8 * k);
                w[j] = v;
            }
            rx_transpose32(w);
            for (int k = 0; k < 4 && p + k < length; ++k)
                rx_step(s, acc, w[8 * k + 0], w[8 * k + 1], w[8 * k + 2], w[8 * k + 3], w[8 * k + 4],
                        w[8 * k + 5], w[8 * k + 6], w[8 * k + 7]);
        }
        for (int j = 0; j < 32 && g + j < n; ++j) out[g + j] = (unsigned char)((acc >> j) & 1u);
    }
    return 0;
}
"""


def cpu_circuit(p: rx.Program):
    src = p.jit_source()
    host_part = src.split("// ---- device kernel ----")[0]
    code = "#define __device__\n#define __forceinline__ inline\n" + PERM_CPU + host_part + DRIVER
    d = tempfile.mkdtemp(prefix="rxjit")
    cpp, so = os.path.join(d, "c.cpp"), os.path.join(d, "c.so")
    open(cpp, "w").write(code)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-w", "-o", so, cpp])
    lib = ctypes.CDLL(so)
    lib.rx_cpu_run.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_longlong, ctypes.c_void_p]

    def run(data, length, n):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        out = np.zeros(max(n, 1), np.uint8)
        lib.rx_cpu_run(data.ctypes.data, length, n, out.ctypes.data)
        return out[:n]

    return run


def fixed_strings(rng, n, length, alphabet):
    alpha = np.frombuffer(alphabet, np.uint8)
    data = alpha[rng.integers(0, len(alpha), size=n * length)].astype(np.uint8)
    return W.Strings(data, np.arange(n + 1, dtype=np.int64) * length)


def test_circuit_single_program():
    prog = W.single_program(1)
    s, planted = W.single_strings(prog, seed=7, n=3000, length=64)
    p = rx.compile(prog.ast, prog.root, prog.classes, True)
    run = cpu_circuit(p)
    got = run(s.data, 64, s.n)
    want = oracle.match(prog.ast, prog.root, prog.classes, True, s.data, s.offsets)
    assert np.array_equal(got, want)
    assert want[planted].all()


@pytest.mark.parametrize("seed", range(8))
def test_circuit_small_programs(seed):
    rng = np.random.default_rng(50 + seed)
    for k in range(6):
        prog = W.small_program(seed * 10 + k)
        for length in (0, 1, 3, 8, 13):
            s = fixed_strings(rng, 100, length, b"ab")
            for search in (False, True):
                p = rx.compile(prog.ast, prog.root, prog.classes, search)
                got = cpu_circuit(p)(s.data, length, s.n) if k < 2 or length == 8 else None
                if got is None:
                    continue
                want = oracle.match(prog.ast, prog.root, prog.classes, search, s.data, s.offsets)
                assert np.array_equal(got, want), (seed, k, length, search)


@pytest.mark.parametrize("seed", range(4))
def test_circuit_random_kinds_and_classes(seed):
    rng = np.random.default_rng(900 + seed)
    classes = W.random_classes(rng, 4, universe=np.arange(0, 256), must=np.arange(97, 100))
    for _ in range(3):
        b, root, _ = W.random_tree(rng, int(rng.integers(3, 60)), lambda r: int(r.integers(97, 100)), 4, 0.3)
        ast = b.nodes
        if rng.random() < 0.3:
            leaves = [i for i, x in enumerate(ast) if x[0] == rx.BYTE]
            ast[leaves[0]] = (rx.EPS, 0, 0, -1, -1)
        for search in (False, True):
            p = rx.compile(ast, root, classes, search)
            run = cpu_circuit(p)
            for length in (5, 16):
                s = fixed_strings(rng, 96, length, bytes([97, 98, 99, 0, 255, 200]))
                want = oracle.match(ast, root, classes, search, s.data, s.offsets)
                assert np.array_equal(run(s.data, length, s.n), want), (seed, search, length)


def test_circuit_pathological():
    for family in ("nested", "altstar"):
        prog = W.pathological_program(family, 40)
        s = W.pathological_strings(family, 50, count=64)
        p = rx.compile(prog.ast, prog.root)
        got = cpu_circuit(p)(s.data, 50, s.n)
        want = oracle.match(prog.ast, prog.root, prog.classes, False, s.data, s.offsets)
        assert np.array_equal(got, want)
        assert want[:32].sum() == 0 and want[32:].all()


def test_hiprtc_compiles_for_gfx950():
    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, True)
    p.jit("gfx950")  # no device needed to compile
    st = p.jit_stats()
    assert st["ready"] == 0 and st["state_words"] > 0 and st["ops"] > 0
    # nothing is loaded without a device: no staging mode is available yet
    assert p.jit_staging() == [0] * 7
    # the same circuit text again reuses the code object compiled above
    t0 = time.perf_counter()
    rx.compile(prog.ast, prog.root, prog.classes, True).jit("gfx950")
    assert time.perf_counter() - t0 < 0.5


def _state_words(p):
    return int(p.jit_source().split("#define RX_NS ", 1)[1].split()[0])


@pytest.mark.parametrize("pattern,search,words,member", [
    (b"abc", False, 3, b"abc"),              # anchored literal: one word per byte, none shared
    (b"(x|y|z)*w", False, 1, b"xyzzyxw"),    # every leaf live at the start and with the same update
    (b"a*b", True, 1, b"zzaaabzz"),          # searched: a and b always live (constants), the suffix loop is the word
    (b"(ab)*c", True, 1, b"xabababcx"),      # searched: b only feeds updates that are always live, so it is dropped
    (b"(ab)*c", False, 2, b"ababc"),         # anchored: a and c share a word (same start, same update), b has its own
])
def test_state_words_closed_forms(pattern, search, words, member):
    """State words of the bit-sliced circuit, counted by hand from the position automaton (Def. 5.1):
    leaves with equal start values and updates share a word, constant leaves and leaves the accept
    bit never reads have none; the circuit still gives the oracle's bits (random strings over the
    pattern's letters, every seventh one a member)."""
    p = rx.compile_regex(pattern, search=search)
    assert _state_words(p) == words
    ast, root, classes = rx.parse(pattern)
    rng = np.random.default_rng(len(pattern) + search)
    n, length = 3000, len(member)
    s = fixed_strings(rng, n, length, b"abcxyzw")
    s.data.reshape(n, length)[::7] = np.frombuffer(member, np.uint8)
    want = oracle.match(ast, root, classes, search, s.data, s.offsets)
    assert want[::7].all() and not want.all()
    assert np.array_equal(cpu_circuit(p)(s.data, length, s.n), want)


def test_state_words_pathological_and_limit():
    """The 4,096-node pathological programs need at most two words (all their 'a' leaves agree); a
    200-byte anchored literal needs 200, more than the circuit keeps, and is refused."""
    for family, k in (("nested", 819), ("altstar", 585)):
        prog = W.pathological_program(family, k)
        p = rx.compile(prog.ast, prog.root)
        assert _state_words(p) <= 2
        s = W.pathological_strings(family, 48, count=64)
        want = oracle.match(prog.ast, prog.root, prog.classes, False, s.data, s.offsets)
        assert np.array_equal(cpu_circuit(p)(s.data, 48, s.n), want)
    p = rx.compile_regex(b"ab" * 100, search=False)
    assert _state_words(p) == 200
    with pytest.raises(rx.RxError) as ei:
        p.jit("gfx950")
    assert ei.value.code == rx.RX_ETOOBIG


CHUNK_DRIVER = r"""
// The chunk-parallel kernel on the host: per string, the 64 lanes' maps (the
// same rx_chunk_lane as on the device), composed in lane order.
extern "C" int rx_cpu_chunks(const unsigned char* bytes, long long length, long long n, unsigned char* out) {
    const long long Lc = ((length + 2047) / 2048 + 15) / 16 * 16;
    for (long long i = 0; i < n; ++i) {
        u32 f = 0u;
        for (int lane = 0; lane < 64; ++lane) f = rx_fn_compose(f, rx_chunk_lane(bytes + i * length, length, Lc, lane));
        out[i] = rx_chunk_result(f);
    }
    return 0;
}
"""


def cpu_chunks(p: rx.Program):
    src = p.jit_source()
    host_part = src.split("// ---- device kernel ----")[0]
    code = "#define __device__\n#define __forceinline__ inline\n" + PERM_CPU + host_part + CHUNK_DRIVER
    d = tempfile.mkdtemp(prefix="rxchunk")
    cpp, so = os.path.join(d, "c.cpp"), os.path.join(d, "c.so")
    open(cpp, "w").write(code)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-w", "-o", so, cpp])
    lib = ctypes.CDLL(so)
    lib.rx_cpu_chunks.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_longlong, ctypes.c_void_p]

    def run(data, length, n):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        out = np.zeros(max(n, 1), np.uint8)
        lib.rx_cpu_chunks(data.ctypes.data, length, n, out.ctypes.data)
        return out[:n]

    return run


@pytest.mark.parametrize("family,k,length", [("nested", 819, 100_000), ("altstar", 585, 40_000), ("nested", 3, 1),
                                             ("altstar", 7, 33), ("nested", 40, 4097)])
def test_chunk_parallel_pathological(family, k, length):
    """The chunk-parallel form (a chunk is a map of the circuit's 2^words states, Def. 5.1; maps compose in
    order) on the 4,096-node programs and small ones, lengths from one byte (one chunk) to 10^5 (2,048
    chunks of 49 -> 64 bytes): the closed form a^(n-1) t accepted, a^n not, and the oracle's bits."""
    prog = W.pathological_program(family, k)
    p = rx.compile(prog.ast, prog.root)
    s = W.pathological_strings(family, length, count=8)
    got = cpu_chunks(p)(s.data, length, s.n)
    assert got[:4].sum() == 0 and got[4:].all()
    want = oracle.match(prog.ast, prog.root, prog.classes, False, s.data, s.offsets)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("pattern,search", [(b"(x|y|z)*w", False), (b"a*b", True), (b"(ab)*c", True), (b"a(b|c)", False),
                                            (b"(a|b)*abb", False), (b"x*", False)])
def test_chunk_parallel_small_patterns(pattern, search):
    """Circuits of one or two words (counted by the generator), random strings over the pattern's letters
    with members planted, lengths that leave the last chunks empty or short: the oracle's bits."""
    p = rx.compile_regex(pattern, search=search)
    words = int(p.jit_source().split("#define RX_NS ", 1)[1].split()[0])
    if words > 2:
        pytest.skip(f"{words} state words")
    ast, root, classes = rx.parse(pattern)
    run = cpu_chunks(p)
    rng = np.random.default_rng(len(pattern))
    for length in (5, 47, 1000, 70_001):
        n = 24 if length > 10_000 else 200
        s = fixed_strings(rng, n, length, b"abcxyzw")
        want = oracle.match(ast, root, classes, search, s.data, s.offsets)
        assert np.array_equal(run(s.data, length, n), want), length


LONG_DRIVER = r"""
// rx_match_long's circuit form on the host: every segment of 2,048 chunks,
// every lane's NS + 1 runs (the same rx_aff_lane_maps as on the device), the maps
// composed in chunk order, then applied to the start state.
extern "C" int rx_cpu_long(const unsigned char* bytes, long long length, long long Lc, unsigned char* out) {
    u32 f[RX_M];
    bool any = false;
    for (long long base = 0; base < length; base += 2048 * Lc) {
        const long long seglen = length - base < 2048 * Lc ? length - base : 2048 * Lc;
        for (int lane = 0; lane < 64; ++lane) {
            u32 flat[RX_M * 32], maps[32][RX_M];
            rx_aff_lane_maps(bytes + base, seglen, Lc, lane, flat, 1);
            for (int r = 0; r < RX_M; ++r)
                for (int j = 0; j < 32; ++j) maps[j][r] = flat[r * 32 + j];
            for (int j = 0; j < 32; ++j) {
                if ((32ll * lane + j) * Lc >= seglen) break;
                if (any) rx_aff_compose(f, maps[j]);
                else {
                    for (int i = 0; i < RX_M; ++i) f[i] = maps[j][i];
                    any = true;
                }
            }
        }
    }
    out[0] = rx_aff_result(f, any);
    return 0;
}
"""


def cpu_long(p: rx.Program):
    src = p.jit_source()
    host_part = src.split("// ---- device kernel ----")[0]
    code = "#define __device__\n#define __forceinline__ inline\n" + PERM_CPU + host_part + LONG_DRIVER
    d = tempfile.mkdtemp(prefix="rxlong")
    cpp, so = os.path.join(d, "c.cpp"), os.path.join(d, "c.so")
    open(cpp, "w").write(code)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-w", "-o", so, cpp])
    lib = ctypes.CDLL(so)
    lib.rx_cpu_long.argtypes = [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_longlong, ctypes.c_void_p]

    def run(data, lc=16):
        data = np.ascontiguousarray(data, dtype=np.uint8)
        out = np.zeros(1, np.uint8)
        lib.rx_cpu_long(data.ctypes.data if data.size else None, data.size, lc, out.ctypes.data)
        return int(out[0])

    return run


def test_long_circuit_chunks_single_program():
    """One long string as circuit chunks, each an affine map of the state words (the step's updates are ORs
    of terms reading at most one word, Def. 5.1): the ~200-node searched expression (17 words) on text with
    and without a planted member, at lengths that leave partial segments and chunks, chunks of 16 and 48
    bytes; the oracle's bit every time."""
    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, True)
    words = int(p.jit_source().split("#define RX_NS ", 1)[1].split()[0])
    assert words <= 31
    run = cpu_long(p)
    pieces, planted = W.single_strings(prog, seed=31, n=600, length=256, plant_frac=0.05)
    bits = oracle.match(prog.ast, prog.root, prog.classes, True, pieces.data, pieces.offsets)
    clean = np.concatenate([pieces.data[i * 256:(i + 1) * 256] for i in np.nonzero(bits == 0)[0][:200]])
    member = pieces.data[planted[0] * 256:(planted[0] + 1) * 256]
    rng = np.random.default_rng(5)
    for length in (0, 1, 255, 4096, 40_000, 70_001):
        text = np.resize(clean, length)
        for plant in (False, True):
            t = text.copy()
            if plant and length >= 256:
                at = int(rng.integers(0, length - 255))
                t[at:at + 256] = member
            want = int(oracle.match(prog.ast, prog.root, prog.classes, True, t, np.array([0, length], np.int64))[0])
            for lc in (16, 48):
                assert run(t, lc) == want, (length, plant, lc)


@pytest.mark.parametrize("pattern,search", [(b"(ab)*c", False), (b"a(b|c)*d", False), (b"(x|y|z)*w", False),
                                            (b"abc", True)])
def test_long_circuit_chunks_small_patterns(pattern, search):
    """Anchored and searched patterns whose result depends on the whole string (a member, a member with
    one byte changed at a chunk boundary or inside a chunk), lengths across segment boundaries."""
    p = rx.compile_regex(pattern, search=search)
    ast, root, classes = rx.parse(pattern)
    run = cpu_long(p)
    rng = np.random.default_rng(len(pattern))
    for length in (3, 17, 2048 * 16 + 5, 2 * 2048 * 16 + 33):
        if pattern == b"(ab)*c":
            base = np.frombuffer((b"ab" * length)[:length - 1] + b"c", np.uint8) if length % 2 else None
        elif pattern == b"a(b|c)*d":
            base = np.frombuffer(b"a" + bytes(rng.choice(list(b"bc"), size=length - 2)) + b"d", np.uint8)
        elif pattern == b"(x|y|z)*w":
            base = np.frombuffer(bytes(rng.choice(list(b"xyz"), size=length - 1)) + b"w", np.uint8)
        else:
            base = np.frombuffer(bytes(rng.choice(list(b"abcx"), size=length)), np.uint8)
        if base is None:
            continue
        for flip in (None, 0, length // 2, 16 * 2048, length - 1):
            t = base.copy()
            if flip is not None and flip < length:
                t[flip] = ord("q")
            want = int(oracle.match(ast, root, classes, search, t, np.array([0, length], np.int64))[0])
            assert run(t, 16) == want, (length, flip)
