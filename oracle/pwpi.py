"""Plain CPU oracles for regular expression matching (test infrastructure only).

Nothing in the product path imports this module: only the tests, the smoke
check and the benchmark's CPU-baseline leg do.  It shares no code with the HIP
library; the only thing both sides see is the AST record layout
``(kind, byte, cls, c0, c1)`` that the C interface also uses.

Engines, each written from the paper (Rathnayake & Thielecke, "Regular
Expression Matching and Operational Semantics", SOS 2011):

* ``bigstep_accepts``  -- Fig. 2.1, the big-step definition of ``e matches w``,
  evaluated by memoised recursion over (node, i, j).
* ``ekw_accepts``      -- Def. 3.1 / Fig. 3.1, the EKW machine, searched with a
  visited set (Example 3.3 shows it loops otherwise).
* ``pwpi_accepts``     -- Def. 4.5 / Fig. 4.2, the PW-pi machine over the heap
  of Def. 4.1 with ``cont`` of Def. 4.4, explored by backtracking with a visited
  set of configurations (p, i).  This is THE oracle for GPU parity; its C twin
  is ``rx_oracle.c``.
* ``evolve`` / ``lockstep_accepts`` -- Def. 5.1 - 5.3, the generic lockstep
  machine, written directly from the set definitions.
* ``seq_lockstep_accepts`` -- Def. 6.1 / 6.2, the sequential lockstep machine.

Readings where the paper is silent (all engines follow them):

* Alphabet: bytes 0..255; strings are byte strings of any length.
* Extensions beyond the grammar of Section 2: CLASS leaves (a set of bytes;
  a CLASS leaf ``x`` makes the move ``x --a--> cont x`` for every ``a`` in its
  set), OPT ``e?`` (moves to its child and to its continuation; the child's
  continuation is the OPT's) and PLUS ``e+`` (moves to its child; the child's
  continuation is a companion loop node ``q`` that moves to the child and to
  the PLUS's continuation).  Their languages are those of ``e|eps`` and
  ``e e*``.
* ``null`` is kept as an element of evolved sets when it is reachable, so the
  acceptance test of Def. 5.3 (``null`` in S at the end of input) has
  something to test (Def. 5.1 read literally drops it).
* Fig. 6.1's star rule re-pushes ``p`` itself; the child ``p'`` is meant
  (Fig. 4.2 and the process translation of Section 7 both enter the child).
* Search mode wraps the expression as ``.*(e).*`` where ``.`` is any byte.
"""
from __future__ import annotations

import re
from functools import lru_cache

EPS, BYTE, CLASS, CAT, ALT, STAR, PLUS, OPT = range(8)
KIND_NAMES = ["EPS", "BYTE", "CLASS", "CAT", "ALT", "STAR", "PLUS", "OPT"]
NULL = -1
# heap-only node kind: the loop companion of a PLUS node (reading above)
_PLUSLOOP = 100
ALL_BYTES = frozenset(range(256))


class Words(tuple):
    """A byte set given as four 64-bit words: byte b is bit (b & 63) of word b >> 6."""

    def __new__(cls, words):
        words = tuple(int(w) for w in words)
        if len(words) != 4 or any(not 0 <= w < (1 << 64) for w in words):
            raise ValueError("a word-encoded class is exactly four 64-bit words")
        return super().__new__(cls, words)


def _class_set(mask) -> frozenset:
    """The byte set of a class.  The encoding is taken from the type, never from the values:

    * a Python ``int``: a 256-bit mask (byte b is bit b);
    * ``Words`` or a numpy ``uint64`` array of shape (4,): four 64-bit words
      (byte b is bit b & 63 of word b >> 6) -- the layout of the C interface;
    * any other iterable: the member bytes themselves (each 0..255).
    """
    if isinstance(mask, bool):
        raise TypeError("a class is not a bool")
    if isinstance(mask, int):
        if not 0 <= mask < (1 << 256):
            raise ValueError("a 256-bit class mask is out of range")
        return frozenset(b for b in range(256) if (mask >> b) & 1)
    dtype = getattr(mask, "dtype", None)
    if isinstance(mask, Words) or (dtype is not None and str(dtype) == "uint64"):
        w = Words(list(mask))
        return frozenset(b for b in range(256) if (w[b >> 6] >> (b & 63)) & 1)
    members = [int(v) for v in mask]
    if any(not 0 <= v <= 255 for v in members):
        raise ValueError("a class given by its members holds bytes 0..255 only")
    return frozenset(members)


def label_of(node, classes):
    """The byte set matched by a leaf node (BYTE or CLASS)."""
    kind, byte, cls = node[0], node[1], node[2]
    if kind == BYTE:
        return frozenset([byte])
    if kind == CLASS:
        return _class_set(classes[cls])
    raise ValueError("not a leaf")


def check_tree(ast, root):
    """Every node reachable from ``root`` once, no cycles (Def. 4.3 with disjoint union, Def. 4.2)."""
    n = len(ast)
    if not 0 <= root < n:
        raise ValueError("root out of range")
    seen = [False] * n
    stack = [root]
    while stack:
        p = stack.pop()
        if seen[p]:
            raise ValueError(f"node {p} has two parents or lies on a cycle")
        seen[p] = True
        kind, _, _, c0, c1 = ast[p]
        kids = []
        if kind in (CAT, ALT):
            kids = [c0, c1]
        elif kind in (STAR, PLUS, OPT):
            kids = [c0]
        elif kind not in (EPS, BYTE, CLASS):
            raise ValueError(f"bad kind {kind}")
        for c in kids:
            if not 0 <= c < n:
                raise ValueError(f"child {c} of node {p} out of range")
            stack.append(c)
    if not all(seen):
        raise ValueError("nodes unreachable from the root")


def search_wrap(ast, root, classes):
    """Return (ast', root', classes') for ``.*(e).*``, appending nodes after the originals."""
    ast = [tuple(x) for x in ast]
    classes = list(classes)
    any_cls = len(classes)
    classes.append(ALL_BYTES)
    base = len(ast)
    ast += [
        (CLASS, 0, any_cls, -1, -1),  # base+0: .
        (STAR, 0, 0, base + 0, -1),  # base+1: .*
        (CAT, 0, 0, base + 1, root),  # base+2: .* e
        (CLASS, 0, any_cls, -1, -1),  # base+3: .
        (STAR, 0, 0, base + 3, -1),  # base+4: .*
        (CAT, 0, 0, base + 2, base + 4),  # base+5: (.* e) .*
    ]
    return ast, base + 5, classes


class Heap:
    """The heap pi of Def. 4.1 with the continuation function of Def. 4.4.

    Pointers are AST indices; a PLUS node ``p`` gets a companion loop pointer
    appended after the AST nodes.  ``cont[p]`` is NULL (-1) for the root.
    """

    def __init__(self, ast, root, classes, search=False):
        ast = [tuple(int(v) for v in x) for x in ast]
        check_tree(ast, root)
        if search:
            ast, root, classes = search_wrap(ast, root, classes)
        self.root = root
        self.kind = [a[0] for a in ast]
        self.c0 = [a[3] for a in ast]
        self.c1 = [a[4] for a in ast]
        self.label = [label_of(a, classes) if a[0] in (BYTE, CLASS) else None for a in ast]
        self.companion = {}
        for p, a in enumerate(ast):
            if a[0] == PLUS:
                q = len(self.kind)
                self.companion[p] = q
                self.kind.append(_PLUSLOOP)
                self.c0.append(a[3])
                self.c1.append(-1)
                self.label.append(None)
        self.m = len(self.kind)
        self.cont = [None] * self.m
        self._wire_cont()

    def _wire_cont(self):
        """Def. 4.4: alt children inherit cont p; cat: cont p1 = p2, cont p2 = cont p;
        star: cont p1 = p; root: null.  OPT and PLUS follow the readings in the module header."""
        cont = self.cont
        cont[self.root] = NULL
        stack = [self.root]
        while stack:
            p = stack.pop()
            k = self.kind[p]
            if k == ALT:
                cont[self.c0[p]] = cont[p]
                cont[self.c1[p]] = cont[p]
                stack += [self.c0[p], self.c1[p]]
            elif k == CAT:
                cont[self.c0[p]] = self.c1[p]
                cont[self.c1[p]] = cont[p]
                stack += [self.c0[p], self.c1[p]]
            elif k == STAR:
                cont[self.c0[p]] = p
                stack.append(self.c0[p])
            elif k == OPT:
                cont[self.c0[p]] = cont[p]
                stack.append(self.c0[p])
            elif k == PLUS:
                q = self.companion[p]
                cont[q] = cont[p]
                cont[self.c0[p]] = q
                stack.append(self.c0[p])

    # -- Fig. 4.2 -------------------------------------------------------
    def eps_succ(self, p):
        """Pointers q with p --> q (no input consumed)."""
        if p == NULL:
            return []
        k = self.kind[p]
        if k == ALT:
            return [self.c0[p], self.c1[p]]
        if k == CAT:
            return [self.c0[p]]
        if k == STAR:
            return [self.c0[p], self.cont[p]]
        if k == EPS:
            return [self.cont[p]]
        if k == OPT:
            return [self.c0[p], self.cont[p]]
        if k == PLUS:
            return [self.c0[p]]
        if k == _PLUSLOOP:
            return [self.c0[p], self.cont[p]]
        return []  # leaves

    def is_leaf(self, p):
        return p != NULL and self.kind[p] in (BYTE, CLASS)

    def char_succ(self, p, a):
        """The pointer q with p --a--> q, or None."""
        if self.is_leaf(p) and a in self.label[p]:
            return self.cont[p]
        return None


def pwpi_accepts(heap: Heap, w: bytes) -> bool:
    """Def. 4.5: is there a run <p0; w> --> ... --> <null; eps>?

    Backtracking search over configurations (p, i) (i = input consumed) with a
    visited set, so the loops of Example 4.6 are cut.  A configuration
    <null; w'> with w' non-empty has no successor.
    """
    n = len(w)
    seen = set()
    stack = [(heap.root, 0)]
    while stack:
        p, i = stack.pop()
        if (p, i) in seen:
            continue
        seen.add((p, i))
        if p == NULL:
            if i == n:
                return True
            continue
        for q in heap.eps_succ(p):
            stack.append((q, i))
        if i < n:
            q = heap.char_succ(p, w[i])
            if q is not None:
                stack.append((q, i + 1))
    return False


def pwpi_step_ok(heap: Heap, cfg_from, cfg_to, w: bytes) -> bool:
    """Is <p; w[i:]> --> <q; w[j:]> a single PW-pi transition?  (used to replay Example 4.6)"""
    (p, i), (q, j) = cfg_from, cfg_to
    if j == i:
        return q in heap.eps_succ(p)
    if j == i + 1 and i < len(w):
        return heap.char_succ(p, w[i]) == q
    return False


# -- Section 5: generic lockstep ------------------------------------------
def evolve(heap: Heap, S):
    """Def. 5.1 (with null kept, see header): the leaves, plus null, reachable by --> steps from S."""
    out = set()
    seen = set()
    stack = list(S)
    while stack:
        p = stack.pop()
        if p in seen:
            continue
        seen.add(p)
        if p == NULL or heap.is_leaf(p):
            out.add(p)
            continue
        stack.extend(heap.eps_succ(p))
    return frozenset(out)


def advance(heap: Heap, S, a):
    """Def. 5.2, S ==a==> S': every pointer matching a moves to its continuation; the rest die."""
    return frozenset(q for p in S if (q := heap.char_succ(p, a)) is not None)


def lockstep_trace(heap: Heap, w: bytes):
    """The sets visited by the generic lockstep machine (Def. 5.3): [evolve S0, after a1, evolve, ...]."""
    S = evolve(heap, {heap.root})
    trace = [S]
    for a in w:
        S = advance(heap, S, a)
        trace.append(S)
        S = evolve(heap, S)
        trace.append(S)
    return trace


def lockstep_accepts(heap: Heap, w: bytes) -> bool:
    return NULL in lockstep_trace(heap, w)[-1]


# -- Section 6: sequential lockstep ----------------------------------------
def _psi(p, l1, l2):
    """Def. 6.1: push p onto l1 unless it already occurs in l1 @ l2."""
    return l1 if (p in l1 or p in l2) else [p] + l1


def seq_lockstep_accepts(heap: Heap, w: bytes) -> bool:
    """Def. 6.2 / Fig. 6.1 with three readings: the star rule enters the child;
    a leaf that does not match the next byte is dropped; at the end of input
    evolution continues and the string is accepted if null ever surfaces in c."""
    c, t, n = [heap.root], [], []
    i = 0
    while True:
        if not c:
            if i < len(w) and n:
                c, t, n = n, [], []
                i += 1
                continue
            return False
        p, c = c[0], c[1:]
        if p == NULL:
            if i == len(w):
                return True
            continue  # a null thread dies while input remains
        k = heap.kind[p]
        if k == ALT:
            c = _psi(heap.c1[p], _psi(heap.c0[p], c, t), t)
        elif k == CAT:
            c = _psi(heap.c0[p], c, t)
        elif k in (STAR, OPT, _PLUSLOOP):
            c = _psi(heap.cont[p], _psi(heap.c0[p], c, t), t)
        elif k == PLUS:
            c = _psi(heap.c0[p], c, t)
        elif k == EPS:
            c = _psi(heap.cont[p], c, t)
        else:  # leaf
            if i < len(w) and w[i] in heap.label[p]:
                n = _psi(heap.cont[p], n, [])
        t = [p] + t


# -- Section 2: big-step semantics -----------------------------------------
def bigstep_accepts(ast, root, classes, w: bytes, search=False) -> bool:
    """Fig. 2.1, e matches w, by memoised recursion over (node, i, j).

    Kleene1 is used with a non-empty first part, which leaves the language
    unchanged and makes the recursion well founded.  PLUS and OPT use
    e+ = e e* and e? = e | eps.
    """
    ast = [tuple(int(v) for v in x) for x in ast]
    check_tree(ast, root)
    if search:
        ast, root, classes = search_wrap(ast, root, classes)
    labels = [label_of(a, classes) if a[0] in (BYTE, CLASS) else None for a in ast]

    @lru_cache(maxsize=None)
    def star(c, i, j):  # (c)* matches w[i:j]
        if i == j:
            return True  # Kleene2
        return any(m(c, i, k) and star(c, k, j) for k in range(i + 1, j + 1))  # Kleene1

    @lru_cache(maxsize=None)
    def m(p, i, j):
        kind, _, _, c0, c1 = ast[p]
        if kind == EPS:
            return i == j
        if kind in (BYTE, CLASS):
            return j == i + 1 and w[i] in labels[p]
        if kind == CAT:
            return any(m(c0, i, k) and m(c1, k, j) for k in range(i, j + 1))
        if kind == ALT:
            return m(c0, i, j) or m(c1, i, j)
        if kind == STAR:
            return star(c0, i, j)
        if kind == PLUS:
            return any(m(c0, i, k) and star(c0, k, j) for k in range(i, j + 1))
        if kind == OPT:
            return i == j or m(c0, i, j)
        raise ValueError(kind)

    return m(root, 0, len(w))


# -- Section 3: EKW machine ------------------------------------------------
def ekw_accepts(ast, root, classes, w: bytes, search=False) -> bool:
    """Def. 3.1 / Fig. 3.1.  Expressions are ('n', p) for AST node p, ('s', p) for
    (body of p)* used when unfolding PLUS, and ('e',) for the constant eps.
    A visited set of configurations (e, k, i) cuts the loop of Example 3.3."""
    ast = [tuple(int(v) for v in x) for x in ast]
    check_tree(ast, root)
    if search:
        ast, root, classes = search_wrap(ast, root, classes)
    labels = [label_of(a, classes) if a[0] in (BYTE, CLASS) else None for a in ast]
    E = ("e",)
    n = len(w)
    start = (("n", root), (), 0)
    seen = set()
    stack = [start]
    while stack:
        cfg = stack.pop()
        if cfg in seen:
            continue
        seen.add(cfg)
        e, k, i = cfg
        if e == E and not k and i == n:
            return True
        succ = []
        if e == E:
            if k:
                succ.append((k[0], k[1:], i))
        elif e[0] == "s":  # a star whose body is node e[1]'s child
            body = ("n", ast[e[1]][3])
            succ.append((body, (e,) + k, i))
            succ.append((E, k, i))
        else:
            kind, _, _, c0, c1 = ast[e[1]]
            if kind == ALT:
                succ += [(("n", c0), k, i), (("n", c1), k, i)]
            elif kind == CAT:
                succ.append((("n", c0), (("n", c1),) + k, i))
            elif kind == STAR:
                succ.append((("n", c0), (e,) + k, i))
                succ.append((E, k, i))
            elif kind == PLUS:  # e+ = e e*
                succ.append((("n", c0), (("s", e[1]),) + k, i))
            elif kind == OPT:  # e? = e | eps
                succ += [(("n", c0), k, i), (E, k, i)]
            elif kind == EPS:
                succ.append((E, k, i))
            else:  # a w --> eps k w'
                if i < n and w[i] in labels[e[1]]:
                    succ.append((E, k, i + 1))
        stack.extend(succ)
    return False


# -- library special case ---------------------------------------------------
def to_python_regex(ast, root, classes) -> bytes:
    """Translate the AST to a Python bytes pattern (for re.fullmatch with DOTALL)."""
    ast = [tuple(int(v) for v in x) for x in ast]

    def cls_pat(s):
        if not s:
            return b"(?!)"
        return b"[" + b"".join(re.escape(bytes([b])) for b in sorted(s)) + b"]"

    def go(p):
        kind, byte, cls, c0, c1 = ast[p]
        if kind == EPS:
            return b"(?:)"
        if kind == BYTE:
            return b"(?:" + re.escape(bytes([byte])) + b")"
        if kind == CLASS:
            return cls_pat(_class_set(classes[cls]))
        if kind == CAT:
            return b"(?:" + go(c0) + go(c1) + b")"
        if kind == ALT:
            return b"(?:" + go(c0) + b"|" + go(c1) + b")"
        if kind == STAR:
            return b"(?:" + go(c0) + b")*"
        if kind == PLUS:
            return b"(?:" + go(c0) + b")+"
        if kind == OPT:
            return b"(?:" + go(c0) + b")?"
        raise ValueError(kind)

    return go(root)


def re_accepts(ast, root, classes, w: bytes, search=False) -> bool:
    pat = re.compile(to_python_regex(ast, root, classes), re.DOTALL)
    return (pat.search(w) if search else pat.fullmatch(w)) is not None
