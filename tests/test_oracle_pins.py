"""Pins for the CPU oracle: the paper's worked examples, the big-step definition
by brute force, theorems as cross-engine invariants, language identities and a
library special case.  None of these call the HIP library."""
import itertools
import os

import numpy as np
import pytest

import oracle
from oracle import pwpi
from oracle.pwpi import ALT, BYTE, CAT, CLASS, EPS, NULL, OPT, PLUS, STAR

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KINDS = {"CAT": CAT, "STAR": STAR, "ALT": ALT}


def fig41_ast():
    rows = []
    for line in open(os.path.join(GOLD, "fig4_1_heap.txt")):
        if line.startswith("#") or not line.strip():
            continue
        p, op, c0, c1, cont = line.split()
        if op in KINDS:
            rows.append(((KINDS[op], 0, 0, int(c0), int(c1)), int(cont)))
        else:
            rows.append(((BYTE, ord(op), 0, -1, -1), int(cont)))
    return [r[0] for r in rows], [r[1] for r in rows]


def all_strings(alpha=b"ab", max_len=6):
    for n in range(max_len + 1):
        for t in itertools.product(alpha, repeat=n):
            yield bytes(t)


def enum_trees(max_nodes, leaves=((BYTE, 97), (BYTE, 98), (EPS, 0)), unary=(STAR,), binary=(CAT, ALT)):
    """All ASTs with at most max_nodes nodes, as node lists with the root last."""
    memo = {}

    def trees(n):
        if n in memo:
            return memo[n]
        out = []
        if n == 1:
            for k, b in leaves:
                out.append([(k, b, 0, -1, -1)])
        else:
            for u in unary:
                for t in trees(n - 1):
                    out.append(t + [(u, 0, 0, len(t) - 1, -1)])
            for k in binary:
                for left in range(1, n - 1):
                    for tl in trees(left):
                        for tr in trees(n - 1 - left):
                            shift = [(a, b, c, d + len(tl) if d >= 0 else d, e + len(tl) if e >= 0 else e)
                                     for (a, b, c, d, e) in tr]
                            out.append(tl + shift + [(k, 0, 0, len(tl) - 1, len(tl) + len(tr) - 1)])
        memo[n] = out
        return out

    for n in range(1, max_nodes + 1):
        yield from trees(n)


def c_oracle(ast, root, classes, search, strings):
    from paper_1108_3126_amd.workloads import pack

    s = pack(strings)
    return oracle.match(ast, root, classes, search, s.data, s.offsets, threads=2)


# ---------------------------------------------------------------------------
# worked examples
# ---------------------------------------------------------------------------
def test_fig41_cont_table_python_and_c():
    ast, cont = fig41_ast()
    h = pwpi.Heap(ast, 0, [])
    assert h.cont == cont
    assert oracle.heap_cont(ast, 0) == cont


def _traces():
    traces, cur = {}, None
    for line in open(os.path.join(GOLD, "ex4_6_traces.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            traces[cur] = []
            continue
        p, rest = line.split()
        traces[cur].append((int(p), b"" if rest == "-" else rest.encode()))
    return traces


def test_ex46_runs_are_pwpi_runs():
    ast, _ = fig41_ast()
    h = pwpi.Heap(ast, 0, [])
    w = b"aab"
    for name, run in _traces().items():
        cfgs = [(p, len(w) - len(rest)) for p, rest in run]
        for a, b in zip(cfgs, cfgs[1:]):
            assert pwpi.pwpi_step_ok(h, a, b, w), (name, a, b)
    # the accepting run ends in the accepting configuration <null; eps>
    assert _traces()["accepting"][-1] == (NULL, b"")
    assert pwpi.pwpi_accepts(h, w)
    assert oracle.match(ast, 0, [], False, w, [0, 3])[0] == 1


def test_ex71_pointer_sets():
    ast, _ = fig41_ast()
    h = pwpi.Heap(ast, 0, [])
    want = []
    for line in open(os.path.join(GOLD, "ex7_1_sets.txt")):
        if line.startswith("#") or not line.strip():
            continue
        want.append(frozenset(int(x) for x in line.split("=")[1].split(",")))
    # lockstep_trace alternates evolve / advance; Example 7.1 lists evolve, advance, evolve, ...
    trace = pwpi.lockstep_trace(h, b"aab")
    assert trace[: len(want)] == want
    assert NULL in trace[-1]


def test_ex33_nested_star_terminates_and_accepts():
    # (a*)* : EKW without a visited set loops on <(a*)*; []; a> (Example 3.3)
    ast = [(BYTE, 97, 0, -1, -1), (STAR, 0, 0, 0, -1), (STAR, 0, 0, 1, -1)]
    for n in range(0, 12):
        w = b"a" * n
        assert pwpi.ekw_accepts(ast, 2, [], w)
        assert pwpi.pwpi_accepts(pwpi.Heap(ast, 2, []), w)
    # backtracking with a visited set rejects a^1000 b quickly (Section 3 remark)
    w = b"a" * 1000 + b"b"
    assert oracle.match(ast, 2, [], False, w, [0, len(w)])[0] == 0
    assert oracle.match(ast, 2, [], False, w[:-1], [0, len(w) - 1])[0] == 1


# ---------------------------------------------------------------------------
# brute force against the big-step definition (Fig. 2.1); theorems 3.2, 4.7,
# 5.4 and 7.2 say every machine accepts the same strings
# ---------------------------------------------------------------------------
ENGINES = ["ekw", "pwpi", "lockstep", "seq"]


def _engine(name, ast, root, classes, w, search=False):
    if name == "ekw":
        return pwpi.ekw_accepts(ast, root, classes, w, search)
    h = pwpi.Heap(ast, root, classes, search)
    return {"pwpi": pwpi.pwpi_accepts, "lockstep": pwpi.lockstep_accepts, "seq": pwpi.seq_lockstep_accepts}[name](h, w)


def test_all_small_trees_against_bigstep():
    strings = list(all_strings(b"ab", 5))
    n_trees = 0
    for nodes in enum_trees(5):
        root = len(nodes) - 1
        want = [pwpi.bigstep_accepts(nodes, root, [], w) for w in strings]
        got_c = c_oracle(nodes, root, [], False, strings).astype(bool).tolist()
        assert got_c == want, nodes
        for name in ENGINES:
            assert [_engine(name, nodes, root, [], w) for w in strings] == want, (name, nodes)
        n_trees += 1
    assert n_trees == 411


def _random_ast(rng, n_nodes, n_classes=2):
    from paper_1108_3126_amd.workloads import random_tree

    b, root, _ = random_tree(rng, n_nodes, lambda r: int(r.choice([97, 98])), n_classes, 0.2)
    if rng.random() < 0.3:  # sprinkle an EPS leaf
        nodes = b.nodes
        leaves = [i for i, x in enumerate(nodes) if x[0] == BYTE]
        if leaves:
            i = leaves[int(rng.integers(0, len(leaves)))]
            nodes[i] = (EPS, 0, 0, -1, -1)
    return b.nodes, root


@pytest.mark.parametrize("seed", range(4))
def test_random_trees_all_kinds_against_bigstep(seed):
    rng = np.random.default_rng(1000 + seed)
    classes = [{97}, {97, 98}]
    strings = list(all_strings(b"abc", 4))
    for _ in range(40):
        nodes, root = _random_ast(rng, int(rng.integers(1, 13)))
        for search in (False, True):
            want = [pwpi.bigstep_accepts(nodes, root, classes, w, search) for w in strings]
            assert c_oracle(nodes, root, classes, search, strings).astype(bool).tolist() == want
            for name in ENGINES:
                assert [_engine(name, nodes, root, classes, w, search) for w in strings] == want, (name, nodes, search)
            assert [pwpi.re_accepts(nodes, root, classes, w, search) for w in strings] == want


# ---------------------------------------------------------------------------
# language identities
# ---------------------------------------------------------------------------
def _lang(nodes, root, strings, classes=()):
    return c_oracle(nodes, root, list(classes), False, strings).tolist()


def _shift(nodes, by):
    return [(k, b, c, d + by if d >= 0 else d, e + by if e >= 0 else e) for (k, b, c, d, e) in nodes]


@pytest.mark.parametrize("seed", range(3))
def test_language_identities(seed):
    rng = np.random.default_rng(2000 + seed)
    strings = list(all_strings(b"ab", 6))
    for _ in range(25):
        e, re_ = _random_ast(rng, int(rng.integers(1, 8)), 0)
        f, rf = _random_ast(rng, int(rng.integers(1, 6)), 0)
        g, rg = _random_ast(rng, int(rng.integers(1, 5)), 0)
        L = lambda nodes, root: _lang(nodes, root, strings)
        # (e*)* = e*
        star = e + [(STAR, 0, 0, re_, -1)]
        assert L(star + [(STAR, 0, 0, len(e), -1)], len(e) + 1) == L(star, len(e))
        # e+ = e e*
        plus = e + [(PLUS, 0, 0, re_, -1)]
        e2 = _shift(e, len(e))
        ee = e + e2 + [(STAR, 0, 0, re_ + len(e), -1)]
        ee += [(CAT, 0, 0, re_, len(ee) - 1)]
        assert L(plus, len(e)) == L(ee, len(ee) - 1)
        # e? = e | eps
        opt = e + [(OPT, 0, 0, re_, -1)]
        alt_eps = e + [(EPS, 0, 0, -1, -1), (ALT, 0, 0, re_, len(e))]
        assert L(opt, len(e)) == L(alt_eps, len(e) + 1)
        # e | e = e ; e eps = e
        assert L(e + e2 + [(ALT, 0, 0, re_, re_ + len(e))], 2 * len(e)) == L(e, re_)
        assert L(e + [(EPS, 0, 0, -1, -1), (CAT, 0, 0, re_, len(e))], len(e) + 1) == L(e, re_)
        # e | f = f | e ; (e f) g = e (f g)
        fs = _shift(f, len(e))
        ef = e + fs
        assert L(ef + [(ALT, 0, 0, re_, rf + len(e))], len(ef)) == L(ef + [(ALT, 0, 0, rf + len(e), re_)], len(ef))
        gs = _shift(g, len(ef))
        efg = ef + gs
        n0 = len(efg)
        left = efg + [(CAT, 0, 0, re_, rf + len(e)), (CAT, 0, 0, n0, rg + len(ef))]
        right = efg + [(CAT, 0, 0, rf + len(e), rg + len(ef)), (CAT, 0, 0, re_, n0)]
        assert L(left, n0 + 1) == L(right, n0 + 1)


def test_alternation_star_equals_single_star():
    # (a|aa)* = a*  and  ((a*)*)* = a*
    strings = list(all_strings(b"ab", 7))
    a_star = [(BYTE, 97, 0, -1, -1), (STAR, 0, 0, 0, -1)]
    alt = [(BYTE, 97, 0, -1, -1), (BYTE, 97, 0, -1, -1), (BYTE, 97, 0, -1, -1), (CAT, 0, 0, 1, 2),
           (ALT, 0, 0, 0, 3), (STAR, 0, 0, 4, -1)]
    nested = [(BYTE, 97, 0, -1, -1), (STAR, 0, 0, 0, -1), (STAR, 0, 0, 1, -1), (STAR, 0, 0, 2, -1)]
    want = _lang(a_star, 1, strings)
    assert _lang(alt, 5, strings) == want
    assert _lang(nested, 3, strings) == want
    assert sum(want) == 8


def test_search_is_substring_match():
    rng = np.random.default_rng(7)
    strings = list(all_strings(b"ab", 6))
    for _ in range(30):
        e, r = _random_ast(rng, int(rng.integers(1, 8)), 0)
        got = c_oracle(e, r, [], True, strings).tolist()
        subs = lambda w: {w[i:j] for i in range(len(w) + 1) for j in range(i, len(w) + 1)}
        anchored = dict(zip(list(all_strings(b"ab", 6)), _lang(e, r, strings)))
        want = [int(any(anchored[s] for s in subs(w))) for w in strings]
        assert got == want


def test_classes_and_full_byte_range():
    # a class leaf over all 256 bytes, and literals at byte 0 and 255
    full = (1 << 256) - 1
    nodes = [(CLASS, 0, 0, -1, -1), (STAR, 0, 0, 0, -1), (BYTE, 0, 0, -1, -1), (BYTE, 255, 0, -1, -1),
             (CAT, 0, 0, 2, 3), (CAT, 0, 0, 1, 4)]
    strings = [b"", b"\x00\xff", b"xyz\x00\xff", b"\x00", b"\xff\x00", bytes(range(0, 256, 11)) + b"\x00\xff"]
    got = c_oracle(nodes, 5, [full], False, strings).tolist()
    want = [int(pwpi.bigstep_accepts(nodes, 5, [full], w)) for w in strings]
    assert got == want == [0, 1, 1, 0, 0, 1]


def test_malformed_ast_rejected():
    with pytest.raises(ValueError):
        oracle.match([(CAT, 0, 0, 0, 0)], 0, [], False, b"", [0, 0])
    with pytest.raises(ValueError):  # shared child (not a tree)
        oracle.match([(BYTE, 97, 0, -1, -1), (CAT, 0, 0, 0, 0)], 1, [], False, b"", [0, 0])
    with pytest.raises(ValueError):
        pwpi.Heap([(BYTE, 97, 0, -1, -1), (CAT, 0, 0, 0, 0)], 1, [])


# ---------------------------------------------------------------------------
# planted mistakes: the pins above must catch a plausible bug in the oracle
# ---------------------------------------------------------------------------
class _StarContToParentCont(pwpi.Heap):
    def _wire_cont(self):
        super()._wire_cont()
        for p in range(self.m):
            if self.kind[p] == STAR:
                self.cont[self.c0[p]] = self.cont[p]  # wrong: the body must loop back to the star


class _CatSwapped(pwpi.Heap):
    def eps_succ(self, p):
        if p != NULL and self.kind[p] == CAT:
            return [self.c1[p]]  # wrong operand: concatenation enters its right child
        return super().eps_succ(p)


@pytest.mark.parametrize("bug", [_StarContToParentCont, _CatSwapped])
def test_planted_oracle_mistakes_are_caught(bug):
    ast, cont = fig41_ast()
    strings = list(all_strings(b"ab", 5))
    caught = bug(ast, 0, []).cont != cont
    for nodes in enum_trees(4):
        root = len(nodes) - 1
        want = [pwpi.bigstep_accepts(nodes, root, [], w) for w in strings]
        h = bug(nodes, root, [])
        if [pwpi.pwpi_accepts(h, w) for w in strings] != want:
            caught = True
            break
    assert caught


def test_class_encoding_is_explicit():
    # bytes 0x40-0x47 as four words: every word is <= 255, which a value-based guess reads as the byte
    # list {0, 255}; the encoding comes from the type, so both oracles see the same set.
    words = pwpi.Words([0, 0xFF, 0, 0])
    assert pwpi._class_set(words) == frozenset(range(0x40, 0x48))
    assert pwpi._class_set(np.array([0, 0xFF, 0, 0], np.uint64)) == frozenset(range(0x40, 0x48))
    low = pwpi.Words([0xFF, 0, 0, 0])                      # bytes 0..7
    assert pwpi._class_set(low) == frozenset(range(8))
    assert pwpi._class_set([0, 0xFF, 0, 0]) == frozenset({0, 255})   # a plain list holds member bytes
    assert pwpi._class_set(1 << 0x41) == frozenset({0x41})
    with pytest.raises(ValueError):
        pwpi._class_set([256])
    # one CLASS leaf starred then 'z': the C oracle, the Python PW-pi machine and Python re agree
    nodes = [(CLASS, 0, 0, -1, -1), (STAR, 0, 0, 0, -1), (BYTE, ord("z"), 0, -1, -1), (CAT, 0, 0, 1, 2)]
    strings = [b"z", b"@Az", b"GGGz", b"Hz", b"\x00z", b"\x07z", b"\xffz", b"A", b"@@"]
    for cls, members in ((words, range(0x40, 0x48)), (low, range(8)),
                         (np.array([[0, 0xFF, 0, 0]], np.uint64), range(0x40, 0x48))):
        classes = cls if isinstance(cls, np.ndarray) else [cls]
        want = [int(all(b in members for b in w[:-1]) and w[-1:] == b"z") for w in strings]
        assert c_oracle(nodes, 3, classes, False, strings).tolist() == want
        h = pwpi.Heap(nodes, 3, classes)
        assert [int(pwpi.pwpi_accepts(h, w)) for w in strings] == want
        assert [int(pwpi.re_accepts(nodes, 3, classes, w)) for w in strings] == want
