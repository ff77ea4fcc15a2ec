"""Chunk-parallel matching of one long string (rx_match_long): every chunk count gives the oracle's
bit, from one chunk up to one byte per chunk; lane rows (sets of at most 16 words) and wavefront rows
(the 4,096-node families, checked by their closed form)."""
import numpy as np
import pytest

import oracle
from paper_1108_3126_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def long_bit(p, data, dev, chunks=0):
    from paper_1108_3126_amd import rx

    d = torch.from_numpy(data if data.size else np.zeros(16, np.uint8)).to(dev)
    out = rx.match_long(p, d, data.size, chunks)
    torch.cuda.synchronize()
    return int(out.cpu().numpy()[0])


def oracle_bit(prog, search, data):
    return int(oracle.match(prog.ast, prog.root, prog.classes, search, data, np.array([0, data.size], np.int64))[0])


def test_long_small_programs(dev):
    """Small programs on strings of 0..600 bytes over {a, b}, anchored and searched, chunk counts 0 (default),
    1, 2, 7, 64, one byte per chunk and more chunks than bytes."""
    from paper_1108_3126_amd import rx

    rng = np.random.default_rng(5)
    cases = 0
    for seed in range(80):
        prog = W.small_program(seed)
        for search in (False, True):
            p = rx.compile(prog.ast, prog.root, prog.classes, search).upload(dev)
            for length in (0, 1, 5, 97, 600):
                data = np.frombuffer(b"ab", np.uint8)[rng.integers(0, 2, size=length)].astype(np.uint8)
                want = oracle_bit(prog, search, data)
                for chunks in (0, 1, 2, 7, 64, length, length + 9):
                    got = long_bit(p, data, dev, chunks)
                    assert got == want, (seed, search, length, chunks)
                    cases += 1
    assert cases > 5000


def test_long_single_program(dev):
    """The ~200-node searched expression on one 512 KB lowercase string: rejected, then accepted with a
    member planted across a chunk boundary, at the end, and at the start."""
    from paper_1108_3126_amd import rx

    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev)
    s, _ = W.single_strings(prog, seed=8, n=2048, length=256, plant_frac=0.0)
    base = s.data.copy()
    want = oracle_bit(prog, True, base)
    for chunks in (0, 1, 100, 4096):
        assert long_bit(p, base, dev, chunks) == want, chunks
    w, _ = W.single_strings(prog, seed=9, n=1, length=256, plant_frac=1.0)
    member = w.data
    for at in (base.size // 2 - 100, base.size - 256, 0):
        data = base.copy()
        data[at:at + 256] = member
        want = oracle_bit(prog, True, data)
        assert want == 1
        for chunks in (0, 3, 4096):
            assert long_bit(p, data, dev, chunks) == want, (at, chunks)


def test_long_anchored_against_lane_kernel(dev):
    """Anchored expressions whose result depends on every byte: (ab|a)*(b|c)x? style programs on random text,
    the chunked bit equal to the oracle and to rx_match on the same single string."""
    from paper_1108_3126_amd import rx

    rng = np.random.default_rng(9)
    for pat in (b"(ab|a)*b*", b"[ab]*c[ab]*", b"((a|b)(a|b))*", b".*aba.*|b*"):
        p = rx.compile_regex(pat, search=False).upload(dev)
        ast, root, classes = rx.parse(pat)
        prog = W.Program(ast, root, classes)
        for length in (1000, 4001, 30000):
            alphabet = np.frombuffer(b"ab", np.uint8) if b"c" not in pat else np.frombuffer(b"abbbbb", np.uint8)
            data = alphabet[rng.integers(0, len(alphabet), size=length)].astype(np.uint8)
            if b"c" in pat:
                data[rng.integers(0, length)] = ord("c")
            want = oracle_bit(prog, False, data)
            d = torch.from_numpy(data).to(dev)
            lane = rx.match(p, d, torch.tensor([0, length], dtype=torch.int64, device=dev))
            torch.cuda.synchronize()
            assert int(lane.cpu()[0]) == want
            for chunks in (0, 13, 999):
                assert long_bit(p, data, dev, chunks) == want, (pat, length, chunks)


@pytest.mark.parametrize("family,k", [("nested", 819), ("altstar", 585), ("nested", 64)])
def test_long_pathological(dev, family, k):
    """Sets of 26 and 55 words run one wavefront per row (821 / 1,757 rows per chunk): a^n rejected,
    a^(n-1) t accepted, for n = 10^4 and several chunk counts."""
    from paper_1108_3126_amd import rx

    prog = W.pathological_program(family, k)
    p = rx.compile(prog.ast, prog.root).upload(dev)
    n = 10_000
    s = W.pathological_strings(family, n, count=2)
    rej, acc = s.data[:n].copy(), s.data[n:].copy()
    for chunks in (1, 8, 40):
        print(f"long {family} k={k} chunks={chunks}", flush=True)
        assert long_bit(p, rej, dev, chunks) == 0
        assert long_bit(p, acc, dev, chunks) == 1


def test_long_errors(dev):
    from paper_1108_3126_amd import rx

    p = rx.compile_regex(b"a*b").upload(dev)
    d = torch.zeros(64, dtype=torch.uint8, device=dev)
    out = torch.zeros(1, dtype=torch.uint8, device=dev)
    import ctypes

    need = ctypes.c_size_t()
    assert rx.lib().rx_match_long_workspace(p.handle, 64, 4, ctypes.byref(need)) == 0
    work = torch.zeros(int(need.value), dtype=torch.uint8, device=dev)
    rc = rx.lib().rx_match_long(p.handle, ctypes.c_void_p(d.data_ptr()), 64, 4, ctypes.c_void_p(work.data_ptr()),
                                int(need.value) - 1, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == rx.RX_EINVAL
    q = rx.compile_regex(b"a*b")   # never uploaded
    rc = rx.lib().rx_match_long(q.handle, ctypes.c_void_p(d.data_ptr()), 64, 4, ctypes.c_void_p(work.data_ptr()),
                                int(need.value), ctypes.c_void_p(out.data_ptr()), None)
    assert rc == rx.RX_ENOTUPLOADED


def first_long(p, data, dev, chunks=0):
    from paper_1108_3126_amd import rx

    d = torch.from_numpy(data if data.size else np.zeros(16, np.uint8)).to(dev)
    out = rx.match_first_long(p, d, data.size, chunks)
    torch.cuda.synchronize()
    return int(out.cpu().numpy()[0])


def first_serial(p, data, dev):
    from paper_1108_3126_amd import rx

    d = torch.from_numpy(data if data.size else np.zeros(16, np.uint8)).to(dev)
    out = rx.match_first(p, d, torch.tensor([0, data.size], dtype=torch.int64, device=dev))
    torch.cuda.synchronize()
    return int(out.cpu().numpy()[0])


def first_by_prefixes(prog, search, data):
    pre = [bytes(data[:k]) for k in range(data.size + 1)]
    s = W.pack(pre)
    acc = oracle.match(prog.ast, prog.root, prog.classes, search, s.data, s.offsets)
    hit = np.nonzero(acc)[0]
    return int(hit[0]) if hit.size else -1


def test_first_long_small_programs(dev):
    """Earliest accepting prefix of one string in chunks: equal to the serial table-form run for every chunk
    count, and to the oracle on every prefix for the shorter strings."""
    from paper_1108_3126_amd import rx

    rng = np.random.default_rng(15)
    for seed in range(50):
        prog = W.small_program(seed)
        for search in (False, True):
            p = rx.compile(prog.ast, prog.root, prog.classes, search).upload(dev)
            for length in (0, 1, 6, 90, 700):
                data = np.frombuffer(b"ab", np.uint8)[rng.integers(0, 2, size=length)].astype(np.uint8)
                want = first_serial(p, data, dev)
                if length <= 90:
                    assert want == first_by_prefixes(prog, search, data), (seed, search, length)
                for chunks in (0, 1, 3, 16, length, length + 4):
                    assert first_long(p, data, dev, chunks) == want, (seed, search, length, chunks)


def test_first_long_single_program(dev):
    """The ~200-node searched expression on a 256 KB string whose only match sits at a chosen place (start of a
    chunk, across a boundary, at the end): the chunked answer equals the serial one."""
    from paper_1108_3126_amd import rx

    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev)
    pieces, _ = W.single_strings(prog, seed=30, n=2048, length=256, plant_frac=0.0)
    bits = rx.match_fixed(p, torch.from_numpy(pieces.data).to(dev), 256, pieces.n).cpu().numpy()
    piece = pieces.data[int(np.nonzero(bits == 0)[0][0]) * 256:][:256]
    member, _ = W.single_strings(prog, seed=31, n=1, length=256, plant_frac=1.0)
    base = np.tile(piece, 1024)
    assert first_serial(p, base, dev) == -1 or first_long(p, base, dev) == first_serial(p, base, dev)
    for at in (0, 1000, base.size // 2 - 77, base.size - 256):
        data = base.copy()
        data[at:at + 256] = member.data
        want = first_serial(p, data, dev)
        assert want > 0
        for chunks in (0, 7, 512, 4096):
            assert first_long(p, data, dev, chunks) == want, (at, chunks)


@pytest.mark.parametrize("family,k", [("nested", 819), ("altstar", 585)])
def test_first_long_pathological(dev, family, k):
    """Wavefront rows: a^(n-1) t is first accepted at its very end, a^n never."""
    from paper_1108_3126_amd import rx

    prog = W.pathological_program(family, k)
    p = rx.compile(prog.ast, prog.root).upload(dev)
    n = 3000
    s = W.pathological_strings(family, n, count=2)
    for chunks in (1, 8, 40):
        assert first_long(p, s.data[:n].copy(), dev, chunks) == -1
        assert first_long(p, s.data[n:].copy(), dev, chunks) == n


def test_long_circuit_chunks(dev):
    """With a compiled circuit of at most 31 words and the default chunking, rx_match_long runs the string
    as circuit chunks (each chunk an affine map of the state words): the ~200-node searched expression on
    strings of 0 .. 1 MiB, rejected and with a member planted at the start, across a segment boundary and at
    the end; small programs anchored and searched on {a, b} text; the 4,096-node families by their closed
    form.  Every bit equals the oracle's and the table form's (an explicit chunk count)."""
    from paper_1108_3126_amd import rx

    prog = W.single_program(1)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev).jit()
    assert p.jit_stats()["state_words"] <= 31
    s, _ = W.single_strings(prog, seed=8, n=4096, length=256, plant_frac=0.0)
    bits = oracle.match(prog.ast, prog.root, prog.classes, True, s.data, s.offsets, threads=8)
    clean = np.concatenate([s.data[i * 256:(i + 1) * 256] for i in np.nonzero(bits == 0)[0]])
    w, _ = W.single_strings(prog, seed=9, n=1, length=256, plant_frac=1.0)
    for length in (0, 1, 300, 70_001, 2048 * 16 * 3 + 7, 1 << 20):
        base = np.resize(clean, length)
        for at in ([None, 0, length // 2, 2048 * 16 - 100, length - 256] if length >= 2048 * 16 else [None]):
            data = base.copy()
            if at is not None:
                data[at:at + 256] = w.data
            want = oracle_bit(prog, True, data)
            assert long_bit(p, data, dev) == want, (length, at)
            if length <= 70_001:
                assert long_bit(p, data, dev, 64) == want, (length, at, "table")
            if length == 2048 * 16 * 3 + 7:
                # three bytes into the buffer: every chunk unaligned
                buf = torch.from_numpy(np.concatenate([np.zeros(3, np.uint8), data])).to(dev)
                assert int(rx.match_long(p, buf[3:], length).cpu().numpy()[0]) == want, (length, at, "unaligned")
    rng = np.random.default_rng(7)
    for seed in range(6):
        sp = W.small_program(seed)
        for search in (False, True):
            q = rx.compile(sp.ast, sp.root, sp.classes, search).upload(dev).jit()
            for length in (0, 5, 600, 40_000):
                data = np.frombuffer(b"ab", np.uint8)[rng.integers(0, 2, size=length)].astype(np.uint8)
                assert long_bit(q, data, dev) == oracle_bit(sp, search, data), (seed, search, length)
    for family, k in (("nested", 819), ("altstar", 585)):
        pk = W.pathological_program(family, k)
        q = rx.compile(pk.ast, pk.root).upload(dev).jit()
        for n in (1, 1000, 100_000):
            t = W.pathological_strings(family, n, count=2)
            assert long_bit(q, t.data[:n], dev) == 0 and long_bit(q, t.data[n:], dev) == 1, (family, n)
