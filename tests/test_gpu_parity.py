"""GPU parity: the HIP kernels (through the C interface) against the CPU
oracle, bit for bit, on seeded inputs.  Also determinacy across kernel
variants and launch shapes (Thm. 7.2: the parallel schedule does not change
the result) and edge cases."""
import numpy as np
import pytest

import oracle
from paper_1108_3126_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VARIANTS = None


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1108_3126_amd import rx

    global VARIANTS
    VARIANTS = [rx.VARIANT_LANE, rx.VARIANT_WAVE]
    return torch.device("cuda:0")


def gpu_match(prog, s, dev, variant=0, block=0, grid=0, unroll=0, p=None):
    from paper_1108_3126_amd import rx

    if p is None:
        p = rx.compile(prog.ast, prog.root, prog.classes, prog.search).upload(dev)
    d = torch.from_numpy(s.data if s.data.size else np.zeros(1, np.uint8)).to(dev)
    o = torch.from_numpy(s.offsets).to(dev)
    out = rx.match(p, d, o, launch=(variant, block, grid, unroll) if variant or block or grid else None)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_match(prog, s, index=None):
    return oracle.match(prog.ast, prog.root, prog.classes, prog.search, s.data, s.offsets, index=index)


def test_small_seed0_all_variants(dev):
    prog = W.small_program(0)
    s = W.small_strings(0)
    want = oracle_match(prog, s)
    print("small seed 0: n", s.n, "accepted", int(want.sum()), flush=True)
    for v in VARIANTS:
        assert np.array_equal(gpu_match(prog, s, dev, variant=v), want), v


@pytest.mark.parametrize("block", range(0, 1000, 50))
def test_small_fuzz(dev, block):
    from paper_1108_3126_amd import rx

    for seed in range(block, block + 50):
        prog = W.small_program(seed)
        s = W.small_strings(seed)
        for search in (False, True):
            prog.search = search
            want = oracle_match(prog, s)
            p = rx.compile(prog.ast, prog.root, prog.classes, search).upload(dev)
            got = gpu_match(prog, s, dev, p=p)
            assert np.array_equal(got, want), (seed, search, np.nonzero(got != want)[0][:5])


def test_single_program_reduced(dev):
    prog = W.single_program(1)
    s, planted = W.single_strings(prog, seed=1, n=4096)
    want = oracle_match(prog, s)
    assert want[planted].all()
    print("single reduced: accepted", int(want.sum()), "planted", len(planted), flush=True)
    for v in VARIANTS:
        assert np.array_equal(gpu_match(prog, s, dev, variant=v), want), v


@pytest.mark.parametrize("seed", [3, 4])
def test_single_program_other_seeds(dev, seed):
    prog = W.single_program(seed)
    s, planted = W.single_strings(prog, seed=seed, n=2048)
    want = oracle_match(prog, s)
    assert want[planted].all()
    assert np.array_equal(gpu_match(prog, s, dev), want)


def test_launch_shapes_are_determinate(dev):
    prog = W.single_program(1)
    s, _ = W.single_strings(prog, seed=5, n=3000)
    from paper_1108_3126_amd import rx

    base = gpu_match(prog, s, dev)
    for v, block, grid in [(rx.VARIANT_LANE, 64, 1), (rx.VARIANT_LANE, 128, 7), (rx.VARIANT_LANE, 256, 0),
                           (rx.VARIANT_WAVE, 64, 3), (rx.VARIANT_WAVE, 512, 0), (rx.VARIANT_WAVE, 1024, 2)]:
        assert np.array_equal(gpu_match(prog, s, dev, variant=v, block=block, grid=grid), base), (v, block, grid)


def test_edge_cases(dev):
    from paper_1108_3126_amd import rx

    # (a|b)* c? with classes, empty strings, unaligned offsets, bytes 0 and 255
    ast = [(rx.BYTE, 97, 0, -1, -1), (rx.CLASS, 0, 0, -1, -1), (rx.ALT, 0, 0, 0, 1), (rx.STAR, 0, 0, 2, -1),
           (rx.BYTE, 0, 0, -1, -1), (rx.OPT, 0, 0, 4, -1), (rx.CAT, 0, 0, 3, 5)]
    classes = W.random_classes(np.random.default_rng(9), 1)
    classes[0] = W.class_words({98, 255})
    prog = W.Program(np.array(ast, dtype=W.AST_DTYPE), 6, classes, False)
    strs = [b"", b"a", b"\x00", b"ab\xff\x00", b"ab\xffa\x00\x00", b"x", b"\xff" * 37, b"a" * 17 + b"\x00",
            b"b" * 15, b"b" * 16, b"b" * 33 + b"\x01"]
    s = W.pack(strs)
    for search in (False, True):
        prog.search = search
        want = oracle_match(prog, s)
        for v in VARIANTS:
            assert np.array_equal(gpu_match(prog, s, dev, variant=v), want), (search, v)
    # every string empty
    s0 = W.pack([b""] * 70)
    prog.search = False
    want = oracle_match(prog, s0)
    assert want.all()
    for v in VARIANTS:
        assert np.array_equal(gpu_match(prog, s0, dev, variant=v), want)
    # strings starting at every alignment inside one buffer
    rng = np.random.default_rng(11)
    data = rng.choice(np.frombuffer(b"ab\x00\xff", np.uint8), size=4000)
    cuts = np.sort(rng.integers(0, 4000, size=300))
    offs = np.concatenate([[0], cuts, [4000]]).astype(np.int64)
    s1 = W.Strings(data.astype(np.uint8), offs)
    for search in (False, True):
        prog.search = search
        want = oracle_match(prog, s1)
        for v in VARIANTS:
            assert np.array_equal(gpu_match(prog, s1, dev, variant=v), want), (search, v)


def test_zero_strings_is_noop(dev):
    from paper_1108_3126_amd import rx

    p = rx.compile([(rx.BYTE, 97, 0, -1, -1)], 0).upload(dev)
    out = rx.match(p, torch.zeros(1, dtype=torch.uint8, device=dev), torch.zeros(1, dtype=torch.int64, device=dev))
    assert out.numel() == 0


@pytest.mark.parametrize("family,k", [("nested", 1), ("nested", 8), ("nested", 64), ("altstar", 1), ("altstar", 8),
                                      ("altstar", 64)])
def test_pathological_small_k(dev, family, k):
    prog = W.pathological_program(family, k)
    for n in (1, 2, 100, 1000):
        s = W.pathological_strings(family, n, count=64)
        want = oracle_match(prog, s)
        assert want[:32].sum() == 0 and want[32:].all()  # closed form: a* t
        assert np.array_equal(gpu_match(prog, s, dev), want), (family, k, n)


@pytest.mark.parametrize("family,k", [("nested", 819), ("altstar", 585)])
def test_pathological_4096_nodes(dev, family, k):
    prog = W.pathological_program(family, k)
    s = W.pathological_strings(family, 1000, count=16)
    print(f"pathological {family} k={k} n=1000", flush=True)
    want = oracle_match(prog, s)
    assert want[:8].sum() == 0 and want[8:].all()
    assert np.array_equal(gpu_match(prog, s, dev), want)


@pytest.mark.parametrize("family,k", [("nested", 819), ("altstar", 585), ("nested", 40)])
def test_wavefronts_per_string(dev, family, k):
    """One, two, four, eight or sixteen wavefronts per string (partial next sets meeting in LDS) give the same bits, with
    tables in LDS (nested, 40), through the caches (altstar) and with chunk-union rows (both 4,096-node
    programs); offsets and fixed layouts."""
    from paper_1108_3126_amd import rx

    prog = W.pathological_program(family, k)
    s = W.pathological_strings(family, 700, count=40)
    want = oracle_match(prog, s)
    assert want[:20].sum() == 0 and want[20:].all()
    p = rx.compile(prog.ast, prog.root).upload(dev)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    for ws in (0, 1, 2, 4, 8, 16):
        got = rx.match(p, d, o, launch=(rx.VARIANT_WAVE, 0, 0, ws)).cpu().numpy()
        assert np.array_equal(got, want), ws
        got = rx.match_fixed(p, d, 700, s.n, launch=(rx.VARIANT_WAVE, 0, 0, ws)).cpu().numpy()
        assert np.array_equal(got, want), ws
    with pytest.raises(rx.RxError):
        rx.match(p, d, o, launch=(rx.VARIANT_WAVE, 0, 0, 3))


def test_wavefronts_per_string_searched(dev):
    """A searched program with classes on sets above 16 words (the wavefront kernels), uneven lengths."""
    from paper_1108_3126_amd import rx

    progs = W.multi_programs(seed=11, count=2, lo=1400, hi=1600)
    prog = max(progs, key=lambda q: len(q.ast))
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev)
    assert p.info.words > 16
    s = W.multi_lines(seed=12, n=300, hi=600)
    want = oracle.match(prog.ast, prog.root, prog.classes, True, s.data, s.offsets)
    d, o = torch.from_numpy(s.data).to(dev), torch.from_numpy(s.offsets).to(dev)
    for ws in (1, 2, 4, 8, 16):
        assert np.array_equal(rx.match(p, d, o, launch=(rx.VARIANT_WAVE, 0, 0, ws)).cpu().numpy(), want), ws


# ---------------------------------------------------------------------------
# bit-sliced circuit kernel (fixed-length strings)
# ---------------------------------------------------------------------------
def fixed_match(p, s, length, dev, variant=0, burst=0):
    from paper_1108_3126_amd import rx

    d = torch.from_numpy(s.data if s.data.size else np.zeros(16, np.uint8)).to(dev)
    out = rx.match_fixed(p, d, length, s.n, launch=(variant, 0, 0, burst) if variant else None)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_sliced_single_program(dev):
    from paper_1108_3126_amd import rx

    prog = W.single_program(1)
    s, planted = W.single_strings(prog, seed=21, n=5000, length=256)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev).jit()
    assert p.jit_stats()["ready"] == 1
    staging = p.jit_staging()
    print("sliced single: staging", staging, flush=True)
    assert staging[0] == 5 and staging[5] == 1   # the skewed kernel is kept and is the default
    # the static check of the register-staged kernels ran on the device's code object, and every
    # kernel the staging report keeps passed it
    guard = p.jit_guard()
    print("sliced single: guard", guard, flush=True)
    assert guard["ran"] == 1
    for k, mode in enumerate((1, 3, 4)):
        if staging[mode] == 1:
            assert guard["violations"][k] == 0 and not guard["dropped"] >> k & 1
        if guard["dropped"] >> k & 1:
            assert staging[mode] == 0
    assert guard["violations"][3] == 0 and not guard["dropped"] & 8   # the default kernel passed
    # the run-time check ran every kept kernel against the table step on a seeded batch; a kernel
    # it dropped no longer shows in the staging report
    check = p.jit_selfcheck()
    print("sliced single: run-time check", check, flush=True)
    assert check["ran"] == 1
    for k, mode in enumerate((1, 3, 4)):
        if check["dropped"] >> k & 1:
            assert staging[mode] == 0
    assert not check["dropped"] & 8   # the default kernel agreed
    want = oracle_match(prog, s)
    print("sliced single: accepted", int(want.sum()), flush=True)
    for v in (rx.VARIANT_SLICED, rx.VARIANT_LANE, rx.VARIANT_WAVE, 0):
        assert np.array_equal(fixed_match(p, s, 256, dev, v), want), v
    assert np.array_equal(fixed_match(p, s, 256, dev, rx.VARIANT_SLICED, 2), want)
    assert np.array_equal(fixed_match(p, s, 256, dev, rx.VARIANT_SLICED, 3), want)
    assert np.array_equal(fixed_match(p, s, 256, dev, rx.VARIANT_SLICED, 4), want)
    assert np.array_equal(fixed_match(p, s, 256, dev, rx.VARIANT_SLICED, 5), want)


@pytest.mark.parametrize("burst", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("length", [16, 32, 48, 64, 80, 112, 272])
def test_sliced_lengths_and_counts(dev, length, burst):
    from paper_1108_3126_amd import rx

    rng = np.random.default_rng(length)
    prog = W.single_program(3)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev).jit()
    for n in (1, 31, 33, 2047, 2049, 4100):
        s, _ = W.single_strings(prog, seed=length + n, n=n, length=length, plant_frac=0.3)
        want = oracle_match(prog, s)
        assert np.array_equal(fixed_match(p, s, length, dev, rx.VARIANT_SLICED, burst), want), (length, n)


@pytest.mark.parametrize("seed", range(6))
def test_sliced_small_programs(dev, seed):
    from paper_1108_3126_amd import rx

    rng = np.random.default_rng(seed)
    for k in range(5):
        prog = W.small_program(100 + seed * 5 + k)
        for search in (False, True):
            p = rx.compile(prog.ast, prog.root, prog.classes, search).upload(dev).jit()
            data = np.frombuffer(b"ab", np.uint8)[rng.integers(0, 2, size=3000 * 32)].astype(np.uint8)
            s = W.Strings(data, np.arange(3001, dtype=np.int64) * 32)
            prog.search = search
            want = oracle_match(prog, s)
            for burst in (3, 4, 5):
                assert np.array_equal(fixed_match(p, s, 32, dev, rx.VARIANT_SLICED, burst), want), (seed, k, search)


def test_sliced_pathological(dev):
    from paper_1108_3126_amd import rx

    for family, k in (("nested", 40), ("altstar", 30)):
        prog = W.pathological_program(family, k)
        s = W.pathological_strings(family, 1008, count=64)
        p = rx.compile(prog.ast, prog.root).upload(dev).jit()
        want = oracle_match(prog, s)
        assert want[:32].sum() == 0 and want[32:].all()
        for burst in (3, 4, 5):
            assert np.array_equal(fixed_match(p, s, 1008, dev, rx.VARIANT_SLICED, burst), want), family
    # the 4,096-node programs: every 'a' leaf of one family holds the same word, so the circuit is tiny
    for family, k in (("nested", 819), ("altstar", 585)):
        prog = W.pathological_program(family, k)
        s = W.pathological_strings(family, 1008, count=64)
        p = rx.compile(prog.ast, prog.root).upload(dev).jit()
        assert p.jit_stats()["state_words"] <= 2
        assert np.array_equal(fixed_match(p, s, 1008, dev, rx.VARIANT_SLICED, 4), oracle_match(prog, s)), family
    # a 200-byte anchored literal: 200 distinct words, more than the circuit keeps
    with pytest.raises(rx.RxError) as ei:
        rx.compile_regex(b"ab" * 100, search=False).jit()
    assert ei.value.code == rx.RX_ETOOBIG


def test_chunk_parallel_pathological(dev):
    """Circuits of at most two words run chunk-parallel (one wavefront per string, 2,048 chunks, each a
    map of the circuit's states): the 4,096-node programs at lengths 1 .. 10^5 against the closed form
    and the oracle, unaligned bytes, and the automatic choice; a circuit of more words is refused."""
    from paper_1108_3126_amd import rx

    for family, k in (("nested", 819), ("altstar", 585)):
        prog = W.pathological_program(family, k)
        p = rx.compile(prog.ast, prog.root).upload(dev).jit()
        assert p.jit_stats()["state_words"] <= 2
        for length in (1, 33, 1008, 4097, 100_000):
            s = W.pathological_strings(family, length, count=64 if length < 10_000 else 8)
            # the closed form a^(n-1) t everywhere; the oracle as well up to 4,097 bytes
            half = s.n // 2
            want = np.concatenate([np.zeros(half, np.uint8), np.ones(s.n - half, np.uint8)])
            if length < 10_000:
                assert np.array_equal(oracle_match(prog, s), want)
            got = fixed_match(p, s, length, dev, rx.VARIANT_CHUNKS)
            assert np.array_equal(got, want), (family, length)
            # one byte into the buffer: every string unaligned
            buf = torch.from_numpy(np.concatenate([np.zeros(1, np.uint8), s.data])).to(dev)
            out = rx.match_fixed(p, buf[1:], length, s.n, launch=(rx.VARIANT_CHUNKS, 0, 0, 0)).cpu().numpy()
            assert np.array_equal(out, want), (family, length, "unaligned")
            d = torch.from_numpy(s.data).to(dev)
            assert np.array_equal(rx.match_fixed(p, d, length, s.n).cpu().numpy(), want)
    big = W.single_program(1)
    q = rx.compile(big.ast, big.root, big.classes, True).upload(dev).jit()
    with pytest.raises(rx.RxError) as ei:
        fixed_match(q, W.pathological_strings("nested", 64, count=4), 64, dev, rx.VARIANT_CHUNKS)
    assert ei.value.code == rx.RX_EINVAL


def test_fixed_layout_fallbacks(dev):
    """rx_match_fixed where the sliced kernel does not apply (length not a multiple of 16, a byte
    buffer not 16-byte aligned, length 0) runs the table-form kernel; explicit sliced requests there
    are refused with RX_EINVAL."""
    from paper_1108_3126_amd import rx

    prog = W.single_program(4)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev).jit()
    for length in (17, 40, 255):
        s, _ = W.single_strings(prog, seed=length, n=3000, length=length, plant_frac=0.3)
        want = oracle_match(prog, s)
        d = torch.from_numpy(s.data).to(dev)
        assert np.array_equal(fixed_match(p, s, length, dev), want), length
        with pytest.raises(rx.RxError) as ei:
            rx.match_fixed(p, d, length, s.n, launch=(rx.VARIANT_SLICED, 0, 0, 0))
        assert ei.value.code == rx.RX_EINVAL
    # a 16-byte length, but the strings start one byte into the buffer
    s, _ = W.single_strings(prog, seed=9, n=3000, length=64, plant_frac=0.3)
    want = oracle_match(prog, s)
    buf = torch.zeros(s.data.size + 16, dtype=torch.uint8, device=dev)
    buf[1:1 + s.data.size] = torch.from_numpy(s.data).to(dev)
    out = rx.match_fixed(p, buf[1:1 + s.data.size], 64, s.n)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)
    # length 0: every string is empty; a searched non-nullable expression rejects them all
    out = rx.match_fixed(p, torch.zeros(16, dtype=torch.uint8, device=dev), 0, 100)
    torch.cuda.synchronize()
    assert out.cpu().numpy().sum() == 0


def test_parsed_patterns_on_gpu(dev):
    """Regular-expression text through rx_parse, matched on the GPU (table form and the sliced circuit),
    against Python's re on bytes with DOTALL."""
    import re

    from paper_1108_3126_amd import rx

    pats = [b"a(b|c)*d", b"(a|aa)*b", b"x{2,3}y{,2}z{2}", b"[^a-c]+\\d?", b"\\w+@\\w+\\.com", b"(|a)(b|)",
            b"(ab){0,4}c+", b"[a-c]*1[\\x30-\\x39]{2}", b".\\..", b"((a*)*)*b"]
    rng = np.random.default_rng(77)
    alphabet = np.frombuffer(b"abcdx1.@\n", np.uint8)
    strings = [bytes(alphabet[rng.integers(0, len(alphabet), size=rng.integers(0, 20))]) for _ in range(2000)]
    strings += [b"abcbd", b"aaab", b"xxyzz", b"u_1@host.com", b"abababc", b"ab112"]
    s = W.pack(strings)
    fixed = [bytes(alphabet[rng.integers(0, len(alphabet), size=32)]) for _ in range(2048)]
    fs = W.pack(fixed)
    for pat in pats:
        r = re.compile(pat, re.DOTALL)
        for search in (False, True):
            f = r.search if search else r.fullmatch
            want = np.array([1 if f(w) else 0 for w in strings], np.uint8)
            p = rx.compile_regex(pat, search=search).upload(dev)
            assert np.array_equal(gpu_match(None, s, dev, p=p), want), (pat, search)
            p.jit()
            want = np.array([1 if f(w) else 0 for w in fixed], np.uint8)
            assert np.array_equal(fixed_match(p, fs, 32, dev), want), (pat, search, "sliced")


def _first_by_prefixes(prog, strings, search):
    """Earliest accepting prefix by brute force: the oracle on every prefix of every string."""
    pre, owner, plen = [], [], []
    for i, w in enumerate(strings):
        for k in range(len(w) + 1):
            pre.append(w[:k])
            owner.append(i)
            plen.append(k)
    ps = W.pack(pre)
    acc = oracle.match(prog.ast, prog.root, prog.classes, search, ps.data, ps.offsets)
    first = np.full(len(strings), -1, np.int64)
    for a, i, k in zip(acc, owner, plen):
        if a and first[i] < 0:
            first[i] = k
    return first


def _gpu_first(p, strings, dev):
    from paper_1108_3126_amd import rx

    s = W.pack(strings)
    d = torch.from_numpy(s.data if s.data.size else np.zeros(1, np.uint8)).to(dev)
    out = rx.match_first(p, d, torch.from_numpy(s.offsets).to(dev))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_match_first_small_programs(dev):
    from paper_1108_3126_amd import rx

    for seed in range(60):
        prog = W.small_program(seed)
        s = W.small_strings(seed)
        strings = [bytes(s.data[s.offsets[i]:s.offsets[i + 1]]) for i in range(200)]
        for search in (False, True):
            prog.search = search
            p = rx.compile(prog.ast, prog.root, prog.classes, search).upload(dev)
            want = _first_by_prefixes(prog, strings, search)
            got = _gpu_first(p, strings, dev)
            assert np.array_equal(got, want), (seed, search, np.nonzero(got != want)[0][:5])


def test_match_first_single_program(dev):
    from paper_1108_3126_amd import rx

    prog = W.single_program(1)
    s, planted = W.single_strings(prog, seed=33, n=240, length=256, plant_frac=0.5)
    strings = [bytes(s.data[s.offsets[i]:s.offsets[i + 1]]) for i in range(s.n)]
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev)
    want = _first_by_prefixes(prog, strings, True)
    got = _gpu_first(p, strings, dev)
    assert (got[planted] >= 0).all()
    assert np.array_equal(got, want)
    # the result bit of a searched program is "some prefix is accepted"
    bits = gpu_match(prog, s, dev, p=p)
    assert np.array_equal(bits, (got >= 0).astype(np.uint8))


def test_match_first_wavefront_programs(dev):
    """Programs above 16 words run one wavefront per string: brute force on short strings, the
    closed form (a^n rejected, a^(n-1) t accepted exactly at its end) on long ones."""
    from paper_1108_3126_amd import rx

    for family, k in (("nested", 819), ("altstar", 585)):
        prog = W.pathological_program(family, k)
        p = rx.compile(prog.ast, prog.root).upload(dev)
        assert p.info.words > 16
        short = W.pathological_strings(family, 24, count=8)
        strings = [bytes(short.data[short.offsets[i]:short.offsets[i + 1]]) for i in range(short.n)]
        assert np.array_equal(_gpu_first(p, strings, dev), _first_by_prefixes(prog, strings, False)), family
        long = W.pathological_strings(family, 3000, count=64)
        strings = [bytes(long.data[long.offsets[i]:long.offsets[i + 1]]) for i in range(long.n)]
        got = _gpu_first(p, strings, dev)
        assert (got[:32] == -1).all() and (got[32:] == 3000).all(), family


def _gpu_first_fixed(p, s, length, dev, buf=None):
    from paper_1108_3126_amd import rx

    d = buf if buf is not None else torch.from_numpy(s.data if s.data.size else np.zeros(16, np.uint8)).to(dev)
    out = rx.match_first_fixed(p, d, length, s.n)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_match_first_fixed_sliced_small_programs(dev):
    """The skewed bit-sliced kernel's earliest-accept form: two-letter strings in three workgroups
    (the last one ragged), every string against the oracle on every prefix."""
    from paper_1108_3126_amd import rx

    sliced = 0
    for seed in range(12):
        rng = np.random.default_rng(seed)
        prog = W.small_program(300 + seed)
        length = (16, 32, 48)[seed % 3]
        n = 4096 + 37 * seed + 1
        data = np.frombuffer(b"ab", np.uint8)[rng.integers(0, 2, size=n * length)].astype(np.uint8)
        s = W.Strings(data, np.arange(n + 1, dtype=np.int64) * length)
        strings = [bytes(data[i * length:(i + 1) * length]) for i in range(n)]
        for search in (False, True):
            prog.search = search
            p = rx.compile(prog.ast, prog.root, prog.classes, search).upload(dev).jit()
            assert p.jit_staging()[6] in (1, 2)
            sliced += not p.info.nullable
            want = _first_by_prefixes(prog, strings, search)
            got = _gpu_first_fixed(p, s, length, dev)
            assert np.array_equal(got, want), (seed, search, np.nonzero(got != want)[0][:5])
    assert sliced >= 8


def test_match_first_fixed_single_program(dev):
    """~200-node searched expression, 256-byte strings: the sliced form against the table form on every
    string, a sample against the oracle on every prefix, and accepted iff rx_match_fixed says so."""
    from paper_1108_3126_amd import rx

    prog = W.single_program(1)
    s, planted = W.single_strings(prog, seed=34, n=6000, length=256, plant_frac=0.3)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev).jit()
    st = p.jit_staging()
    print("first fixed: staging", st, flush=True)
    assert st[6] == 1
    got = _gpu_first_fixed(p, s, 256, dev)
    table = _gpu_first(p, [bytes(s.data[i * 256:(i + 1) * 256]) for i in range(s.n)], dev)
    assert np.array_equal(got, table)
    assert (got[planted] > 0).all() and (got <= 256).all()
    assert np.array_equal((got >= 0).astype(np.uint8), fixed_match(p, s, 256, dev))
    idx = np.unique(np.concatenate([np.arange(0, s.n, 500), planted[:40], [2047, 2048, s.n - 1]]))
    strings = [bytes(s.data[i * 256:(i + 1) * 256]) for i in idx]
    assert np.array_equal(got[idx], _first_by_prefixes(prog, strings, True))


def test_match_first_fixed_fallbacks(dev):
    """Where the sliced kernel does not apply (length not a multiple of 16, unaligned bytes, no compiled
    circuit, length 0) the table form answers; a nullable expression answers 0 for every string."""
    from paper_1108_3126_amd import rx

    prog = W.small_program(305)
    rng = np.random.default_rng(3)
    for length in (0, 7, 40):
        n = 700
        data = np.frombuffer(b"ab", np.uint8)[rng.integers(0, 2, size=n * length)].astype(np.uint8)
        s = W.Strings(data, np.arange(n + 1, dtype=np.int64) * length)
        strings = [bytes(data[i * length:(i + 1) * length]) for i in range(n)]
        for search in (False, True):
            prog.search = search
            p = rx.compile(prog.ast, prog.root, prog.classes, search).upload(dev).jit()
            assert np.array_equal(_gpu_first_fixed(p, s, length, dev), _first_by_prefixes(prog, strings, search))
    # 64-byte strings one byte into the buffer, and the same strings with no compiled circuit
    big = W.single_program(4)
    s, _ = W.single_strings(big, seed=8, n=2100, length=64, plant_frac=0.4)
    strings = [bytes(s.data[i * 64:(i + 1) * 64]) for i in range(s.n)]
    want = _first_by_prefixes(big, strings, True)
    p = rx.compile(big.ast, big.root, big.classes, True).upload(dev).jit()
    buf = torch.zeros(s.data.size + 16, dtype=torch.uint8, device=dev)
    buf[1:1 + s.data.size] = torch.from_numpy(s.data).to(dev)
    assert np.array_equal(_gpu_first_fixed(p, s, 64, dev, buf=buf[1:1 + s.data.size]), want)
    assert np.array_equal(_gpu_first_fixed(p, s, 64, dev), want)
    q = rx.compile(big.ast, big.root, big.classes, True).upload(dev)
    assert np.array_equal(_gpu_first_fixed(q, s, 64, dev), want)
    # a nullable expression: the empty prefix is accepted
    star = rx.compile_regex(b"(ab)*", search=False).upload(dev).jit()
    assert star.info.nullable
    assert (_gpu_first_fixed(star, s, 64, dev) == 0).all()
    # long strings: nested stars, closed form a^n rejected, a^(n-1) t accepted at its end
    for family, k in (("nested", 40), ("altstar", 30)):
        pp = W.pathological_program(family, k)
        ls = W.pathological_strings(family, 1008, count=64)
        r = rx.compile(pp.ast, pp.root).upload(dev).jit()
        got = _gpu_first_fixed(r, ls, 1008, dev)
        assert (got[:32] == -1).all() and (got[32:] == 1008).all(), family


def test_match_first_parsed_patterns_against_re(dev):
    """Searched: the end of the match that ends first, against Python re on every prefix."""
    import re

    from paper_1108_3126_amd import rx

    rng = np.random.default_rng(5)
    alphabet = np.frombuffer(b"abcx1", np.uint8)
    strings = [bytes(alphabet[rng.integers(0, len(alphabet), size=rng.integers(0, 24))]) for _ in range(400)]
    for pat in (b"b(a|c)+x", b"(ab|ba){2}", b"c[ab]*1", b"x?1+", b"a(b|)c"):
        r = re.compile(pat, re.DOTALL)
        want = np.array([next((k for k in range(len(w) + 1) if r.search(w[:k])), -1) for w in strings], np.int64)
        p = rx.compile_regex(pat, search=True).upload(dev)
        assert np.array_equal(_gpu_first(p, strings, dev), want), pat
