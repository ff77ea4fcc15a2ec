"""The node-per-thread machine (one thread per node of d[], stamp vectors c and n; the paper's
GPU prototype run as one persistent launch) against the oracle, the closed forms of the
nested-star families and Python's re; every result equal to the lockstep tables' (rx_match)."""
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


def run_nodes(p, s, dev):
    from paper_1108_3126_amd import rx

    d = torch.from_numpy(s.data if s.data.size else np.zeros(1, np.uint8)).to(dev)
    out = rx.match_nodes(p, d, torch.from_numpy(s.offsets).to(dev))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def run_tables(p, s, dev):
    from paper_1108_3126_amd import rx

    d = torch.from_numpy(s.data if s.data.size else np.zeros(1, np.uint8)).to(dev)
    out = rx.match(p, d, torch.from_numpy(s.offsets).to(dev))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_nodes_small_fuzz(dev):
    """Small programs (at most 16 AST nodes) on 1000 strings of length 0..32 over {a, b}, anchored and searched."""
    from paper_1108_3126_amd import rx

    for seed in range(200):
        prog = W.small_program(seed)
        s = W.small_strings(seed)
        for search in (False, True):
            p = rx.compile(prog.ast, prog.root, prog.classes, search)
            want = oracle.match(prog.ast, prog.root, prog.classes, search, s.data, s.offsets)
            got = run_nodes(p, s, dev)
            assert np.array_equal(got, want), (seed, search, np.nonzero(got != want)[0][:5])


def test_nodes_single_program(dev):
    """The ~200-node searched expression with classes on 3,000 strings of 256 bytes, 30% planted."""
    from paper_1108_3126_amd import rx

    prog = W.single_program(1)
    s, planted = W.single_strings(prog, seed=41, n=3000, length=256, plant_frac=0.3)
    p = rx.compile(prog.ast, prog.root, prog.classes, True).upload(dev)
    want = oracle.match(prog.ast, prog.root, prog.classes, True, s.data, s.offsets)
    got = run_nodes(p, s, dev)
    assert got[planted].all()
    assert np.array_equal(got, want)
    assert np.array_equal(got, run_tables(p, s, dev))


@pytest.mark.parametrize("family,k", [("nested", 819), ("altstar", 585), ("nested", 8), ("altstar", 64)])
def test_nodes_pathological(dev, family, k):
    """Nested-star families up to 4,096 nodes (1,024 threads, four nodes each): a^n rejected, a^(n-1) t accepted."""
    from paper_1108_3126_amd import rx

    prog = W.pathological_program(family, k)
    p = rx.compile(prog.ast, prog.root)
    s = W.pathological_strings(family, 120, count=16)
    got = run_nodes(p, s, dev)
    assert got[:8].sum() == 0 and got[8:].all()
    short = W.pathological_strings(family, 9, count=8)
    want = oracle.match(prog.ast, prog.root, prog.classes, False, short.data, short.offsets)
    assert np.array_equal(run_nodes(p, short, dev), want)


def test_nodes_parsed_patterns(dev):
    import re

    from paper_1108_3126_amd import rx

    rng = np.random.default_rng(12)
    alphabet = np.frombuffer(b"abcx1.", np.uint8)
    strings = [bytes(alphabet[rng.integers(0, len(alphabet), size=rng.integers(0, 18))]) for _ in range(1500)]
    s = W.pack(strings)
    for pat in (b"a(b|c)*x", b"(a|aa)*b?1", b"x{2,3}[ab]+", b"(|a)(b|)", b"((a*)*)*c", b"[^x.]+\\.?1{0,2}"):
        r = re.compile(pat, re.DOTALL)
        for search in (False, True):
            f = r.search if search else r.fullmatch
            want = np.array([1 if f(w) else 0 for w in strings], np.uint8)
            p = rx.compile_regex(pat, search=search)
            assert np.array_equal(run_nodes(p, s, dev), want), (pat, search)


def test_nodes_edges(dev):
    """No strings, only empty strings, one string across the whole grid, the node limit."""
    from paper_1108_3126_amd import rx

    p = rx.compile_regex(b"(ab)*", search=False)
    d = torch.zeros(16, dtype=torch.uint8, device=dev)
    out = rx.match_nodes(p, d, torch.zeros(1, dtype=torch.int64, device=dev))
    assert out.numel() == 0
    s = W.pack([b""] * 5000)
    assert run_nodes(p, s, dev).all()
    q = rx.compile_regex(b"a+b", search=True)
    assert run_nodes(q, s, dev).sum() == 0
    s = W.pack([b"ab" * 3000 + b"x"])
    assert run_nodes(p, s, dev).tolist() == [0]
    assert run_nodes(q, s, dev).tolist() == [1]
    big = W.pathological_program("altstar", 1200)   # 8,401 nodes
    pb = rx.compile(big.ast, big.root)
    with pytest.raises(rx.RxError) as ei:
        rx.match_nodes(pb, d, torch.tensor([0, 4], dtype=torch.int64, device=dev))
    assert ei.value.code == rx.RX_ETOOBIG
