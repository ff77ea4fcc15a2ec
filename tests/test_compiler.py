"""Host compiler checks (no GPU): node array and cont against Fig. 4.1, the
evolution tables against Example 7.1 and against the oracle's own evolution,
a plain table interpreter against the oracle, validation errors, and the
exported symbols of the C library."""
import os
import re

import numpy as np
import pytest

import oracle
from oracle import pwpi
from paper_1108_3126_amd import rx
from paper_1108_3126_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")
NAMES = {"CAT": rx.CAT, "STAR": rx.STAR, "ALT": rx.ALT}


def fig41_rows():
    rows = []
    for line in open(os.path.join(GOLD, "fig4_1_heap.txt")):
        if line.startswith("#") or not line.strip():
            continue
        p, op, c0, c1, cont = line.split()
        rows.append((op, int(c0), int(c1), int(cont)))
    return rows


def bits(words, n):
    return {i for i in range(n) if (int(words[i >> 5]) >> (i & 31)) & 1}


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "rx.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(rx_[a-z_0-9]+)\s*\(", hdr))
    assert {"rx_compile", "rx_match", "rx_program_upload"} <= declared
    L = rx.lib()
    missing = [name for name in sorted(declared) if not hasattr(L, name)]
    assert not missing
    assert declared <= set(rx.SIGNATURES)
    assert "gfx950" in rx.version()


def test_fig41_node_array_bfs_any_input_order():
    # the same tree given in a scrambled AST order packs to Fig. 4.1 exactly
    ast = [(rx.BYTE, 97, 0, -1, -1), (rx.STAR, 0, 0, 0, -1), (rx.BYTE, 98, 0, -1, -1),
           (rx.STAR, 0, 0, 1, -1), (rx.CAT, 0, 0, 3, 2)]
    p = rx.compile(ast, 4)
    got = p.nodes()
    want = fig41_rows()
    assert len(got) == len(want)
    for (kind, c0, c1, label, cont), (op, w0, w1, wc) in zip(got, want):
        if op in NAMES:
            assert (kind, c0, c1, cont) == (NAMES[op], w0, w1, wc)
        else:
            assert (kind, label, cont) == (rx.BYTE, ord(op), wc)


def test_ex71_first_and_follow():
    p = rx.compile([(rx.CAT, 0, 0, 1, 2), (rx.STAR, 0, 0, 3, -1), (rx.BYTE, 98, 0, -1, -1),
                    (rx.STAR, 0, 0, 4, -1), (rx.BYTE, 97, 0, -1, -1)], 0)
    first, follow, mask, leaf = p.sets()
    L = p.info.n_leaves
    to_ptr = lambda s: {int(leaf[r]) if r < L else -1 for r in s}
    assert to_ptr(bits(first, L + 1)) == {2, 4}  # evolve {p0}
    rank = {int(n): r for r, n in enumerate(leaf)}
    assert to_ptr(bits(follow[rank[4]], L + 1)) == {2, 4}  # a moves to p3, which evolves to {p2, p4}
    assert to_ptr(bits(follow[rank[2]], L + 1)) == {-1}  # b moves to null
    assert to_ptr(bits(mask[ord("a")], L + 1)) == {4}
    assert p.info.nullable == 0


def _bfs_map(ast, root):
    """AST index -> d[] index under breadth-first numbering (children c0 then c1)."""
    order = [root]
    for p in order:
        k, _, _, c0, c1 = ast[p]
        if k in (rx.CAT, rx.ALT):
            order += [c0, c1]
        elif k in (rx.STAR, rx.PLUS, rx.OPT):
            order.append(c0)
    return {a: i for i, a in enumerate(order)}


@pytest.mark.parametrize("seed", range(6))
def test_tables_equal_oracle_evolution(seed):
    rng = np.random.default_rng(300 + seed)
    classes = W.random_classes(rng, 3)
    for _ in range(20):
        b, root, _ = W.random_tree(rng, int(rng.integers(1, 60)), lambda r: int(r.integers(97, 100)), 3, 0.3)
        ast = b.nodes
        p = rx.compile(ast, root, classes)
        first, follow, mask, leaf = p.sets()
        L = p.info.n_leaves
        h = pwpi.Heap(ast, root, classes)
        bfs = _bfs_map(ast, root)
        # oracle pointer -> d[] index (PLUS companions are not leaves, so leaves suffice)
        to_d = lambda s: {bfs[q] if q != pwpi.NULL else -1 for q in s}
        from_ranks = lambda s: {int(leaf[r]) if r < L else -1 for r in s}
        assert from_ranks(bits(first, L + 1)) == to_d(pwpi.evolve(h, {h.root}))
        inv = {v: k for k, v in bfs.items()}
        for r in range(L):
            x = inv[int(leaf[r])]
            assert from_ranks(bits(follow[r], L + 1)) == to_d(pwpi.evolve(h, {h.cont[x]}))
            lab = h.label[x]
            for c in (0, 97, 98, 99, 255):
                assert ((int(mask[c][r >> 5]) >> (r & 31)) & 1) == (c in lab)


def table_interpreter(first, follow, mask, L, w):
    """The lockstep macro step (Def. 5.2) on the compiled tables, as plain Python sets."""
    S = bits(first, L + 1)
    for c in w:
        X = S & bits(mask[c], L + 1)
        S = set()
        for x in X:
            S |= bits(follow[x], L + 1)
    return int(L in S)


@pytest.mark.parametrize("seed", range(4))
def test_table_interpreter_matches_oracle(seed):
    prog = W.small_program(seed)
    s = W.small_strings(seed, n=200)
    for search in (False, True):
        p = rx.compile(prog.ast, prog.root, prog.classes, search)
        first, follow, mask, _ = p.sets()
        got = [table_interpreter(first, follow, mask, p.info.n_leaves, s.get(i)) for i in range(s.n)]
        want = oracle.match(prog.ast, prog.root, prog.classes, search, s.data, s.offsets).tolist()
        assert got == want


def test_table_interpreter_single_program_sample():
    prog = W.single_program(1)
    s, planted = W.single_strings(prog, seed=1, n=64)
    p = rx.compile(prog.ast, prog.root, prog.classes, True)
    assert p.info.suffix_any == 1 and p.info.search == 1
    first, follow, mask, _ = p.sets()
    got = [table_interpreter(first, follow, mask, p.info.n_leaves, s.get(i)) for i in range(s.n)]
    want = oracle.match(prog.ast, prog.root, prog.classes, True, s.data, s.offsets).tolist()
    assert got == want
    assert all(want[i] for i in planted)


def test_plus_and_opt_wiring():
    # a+ : PLUS(0) with a companion loop node appended after the tree
    p = rx.compile([(rx.BYTE, 97, 0, -1, -1), (rx.PLUS, 0, 0, 0, -1)], 1)
    nodes = p.nodes()
    assert [n[0] for n in nodes] == [rx.PLUS, rx.BYTE, rx.PLUSLOOP]
    assert nodes[1][4] == 2 and nodes[2][4] == -1 and nodes[2][1] == 1
    # a? : the child continues where the OPT continues
    p = rx.compile([(rx.BYTE, 97, 0, -1, -1), (rx.OPT, 0, 0, 0, -1)], 1)
    assert p.nodes()[1][4] == -1 and p.info.nullable == 1


def test_search_wrapper_shape():
    p = rx.compile([(rx.BYTE, 97, 0, -1, -1)], 0, search=True)
    nodes = p.nodes()
    assert nodes[0][0] == rx.CAT and p.info.suffix_any == 1 and p.info.m == 7 and p.info.n_leaves == 3


@pytest.mark.parametrize(
    "ast,root,ncls",
    [
        ([(rx.CAT, 0, 0, 1, 1), (rx.BYTE, 97, 0, -1, -1)], 0, 0),  # shared child
        ([(rx.STAR, 0, 0, 1, -1), (rx.STAR, 0, 0, 0, -1)], 0, 0),  # cycle through the root
        ([(rx.CAT, 0, 0, 1, 5), (rx.BYTE, 97, 0, -1, -1)], 0, 0),  # child out of range
        ([(9, 0, 0, -1, -1)], 0, 0),  # bad kind
        ([(rx.CLASS, 0, 3, -1, -1)], 0, 1),  # class out of range
        ([(rx.BYTE, 97, 0, -1, -1), (rx.BYTE, 98, 0, -1, -1)], 0, 0),  # unreachable node
        ([(rx.BYTE, 97, 0, -1, -1)], 3, 0),  # root out of range
        ([(rx.BYTE, 97, 0, -1, -1), (rx.STAR, 0, 0, 2, -1), (rx.STAR, 0, 0, 1, -1)], 0, 0),  # detached cycle
    ],
)
def test_validation_errors(ast, root, ncls):
    with pytest.raises(rx.RxError) as ei:
        rx.compile(ast, root, [set([97])] * ncls)
    assert ei.value.code == rx.RX_EINVAL


def test_large_left_deep_programs():
    for family, k, m, L in (("nested", 819, 4096, 820), ("altstar", 585, 4096, 1756)):
        prog = W.pathological_program(family, k)
        assert len(prog.ast) == m
        p = rx.compile(prog.ast, prog.root)
        assert p.info.m == m and p.info.n_leaves == L and p.info.depth >= k


def test_too_many_leaves():
    prog = W.pathological_program("altstar", 1400)  # 4201 leaves
    with pytest.raises(rx.RxError) as ei:
        rx.compile(prog.ast, prog.root)
    assert ei.value.code == rx.RX_ETOOBIG


def test_match_without_upload_is_an_error():
    p = rx.compile([(rx.BYTE, 97, 0, -1, -1)], 0)
    L = rx.lib()
    import ctypes

    rc = L.rx_match(p.handle, ctypes.c_void_p(16), ctypes.c_void_p(16), 1, ctypes.c_void_p(16), None)
    assert rc == rx.RX_ENOTUPLOADED
    assert L.rx_match(p.handle, None, None, 0, None, None) == rx.RX_ENOTUPLOADED
    assert L.rx_match(None, None, None, 0, None, None) == rx.RX_EINVAL


def test_missing_library_fails_loudly(monkeypatch):
    """No fallback: without the built library every entry point raises instead of computing elsewhere."""
    monkeypatch.setattr(rx, "_lib", None)
    monkeypatch.setattr(rx, "LIB_PATH", os.path.join(ROOT, "no-such-dir", "librx.so"))
    with pytest.raises(ImportError):
        rx.compile_regex(b"ab")
    with pytest.raises(ImportError):
        rx.parse(b"a*b")
