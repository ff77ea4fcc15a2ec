"""Seeded synthetic workloads (regex ASTs and packed strings).

This module only draws inputs: random expression trees, character classes and
byte strings.  It does no matching.  Both the GPU library's callers and the CPU
oracle receive what it returns, so it imports neither.

The paper evaluates on no dataset; every workload here is synthetic:

* ``small``        -- a random expression over {a,b} (literal 0.3 / concat 0.3 /
  alternation 0.2 / star 0.2, depth <= 4 with a forced literal at depth 4,
  at most 16 nodes), 1,000 strings of length U{0..32} over {a,b}; anchored.
* ``single``       -- one ~200-node expression over bytes (literals a-z,
  8 character classes, concat, alternation, star, plus, optional) searched
  as .*(e).*; 1M strings of exactly 256 bytes of uniform a-z, 10% of them
  with a string drawn from the expression's language planted at a uniform
  offset.
* ``multi``        -- 16 expressions of U{16..512} nodes over printable ASCII
  (Zipf(1.1) literals, 8 classes each) searched; lines of log-normal length
  (mean 120, sigma 1, clipped to [1, 4096]) with Zipf(1.1) characters.
* ``serving``      -- requests of one expression (8..512 nodes, log-uniform)
  and 1..10,000 strings (log-uniform) of log-normal length (median 256,
  sigma 1, clipped to [16, 8192]).
* ``pathological`` -- ((a*)*)* or (a|aa)* repeated k times by left-deep
  concatenation and closed by 'b' / 'c'; strings a^n and a^(n-1)t.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

EPS, BYTE, CLASS, CAT, ALT, STAR, PLUS, OPT = range(8)

AST_DTYPE = np.dtype(
    [("kind", np.uint8), ("byte", np.uint8), ("cls", np.uint16), ("c0", np.int32), ("c1", np.int32)]
)

LOWER = np.arange(ord("a"), ord("z") + 1, dtype=np.int64)
PRINTABLE = np.arange(0x20, 0x7F, dtype=np.int64)  # 95 characters, Zipf rank r -> 0x1F + r


@dataclass
class Program:
    ast: np.ndarray  # AST_DTYPE records
    root: int
    classes: np.ndarray  # (n_classes, 4) uint64, byte b = bit (b & 63) of word b >> 6
    search: bool = False

    @property
    def n_nodes(self) -> int:
        return len(self.ast)


@dataclass
class Strings:
    data: np.ndarray  # uint8, all strings back to back
    offsets: np.ndarray  # int64, n + 1 entries

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def get(self, i: int) -> bytes:
        return self.data[self.offsets[i] : self.offsets[i + 1]].tobytes()


def pack(strings) -> Strings:
    lens = np.array([len(s) for s in strings], dtype=np.int64)
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    data = np.frombuffer(b"".join(bytes(s) for s in strings), dtype=np.uint8).copy()
    return Strings(data, offs)


def class_words(byte_set) -> np.ndarray:
    w = np.zeros(4, dtype=np.uint64)
    for b in byte_set:
        w[b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    return w


def class_members(words) -> list:
    return [b for b in range(256) if (int(words[b >> 6]) >> (b & 63)) & 1]


class _Builder:
    def __init__(self):
        self.nodes = []

    def add(self, kind, byte=0, cls=0, c0=-1, c1=-1) -> int:
        self.nodes.append((kind, byte, cls, c0, c1))
        return len(self.nodes) - 1

    def array(self) -> np.ndarray:
        return np.array(self.nodes, dtype=AST_DTYPE)


# ---------------------------------------------------------------------------
# small: grammar of literal / concat / alternation / star over {a,b}
# ---------------------------------------------------------------------------
def small_program(seed: int, max_nodes: int = 16, max_depth: int = 4) -> Program:
    rng = np.random.default_rng([seed, 0])
    while True:
        b = _Builder()

        def gen(depth):
            if depth >= max_depth:
                r = 0.0
            else:
                r = rng.random()
            if r < 0.3:
                return b.add(BYTE, byte=int(rng.choice([97, 98])))
            if r < 0.6:
                x = gen(depth + 1)
                y = gen(depth + 1)
                return b.add(CAT, c0=x, c1=y)
            if r < 0.8:
                x = gen(depth + 1)
                y = gen(depth + 1)
                return b.add(ALT, c0=x, c1=y)
            x = gen(depth + 1)
            return b.add(STAR, c0=x)

        root = gen(0)
        if len(b.nodes) <= max_nodes:
            return Program(b.array(), root, np.zeros((0, 4), np.uint64), False)


def small_strings(seed: int, n: int = 1000, max_len: int = 32, alphabet=b"ab") -> Strings:
    rng = np.random.default_rng([seed, 1])
    lens = rng.integers(0, max_len + 1, size=n)
    alpha = np.frombuffer(alphabet, np.uint8)
    offs = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    data = alpha[rng.integers(0, len(alpha), size=int(offs[-1]))]
    return Strings(data.astype(np.uint8), offs)


# ---------------------------------------------------------------------------
# random trees with an exact node count
# ---------------------------------------------------------------------------
def random_classes(rng, n: int, universe=PRINTABLE, must=LOWER) -> np.ndarray:
    """n classes, each a union of 1-3 byte ranges inside ``universe`` (width 1..12),
    holding at least one byte of ``must``; a quarter are complemented over 0..255
    when the complement still holds a byte of ``must``."""
    out = np.zeros((n, 4), np.uint64)
    must_set = set(int(x) for x in must)
    lo_u, hi_u = int(universe[0]), int(universe[-1])
    for i in range(n):
        s = set()
        for _ in range(int(rng.integers(1, 4))):
            lo = int(rng.integers(lo_u, hi_u + 1))
            hi = min(hi_u, lo + int(rng.integers(0, 12)))
            s.update(range(lo, hi + 1))
        if not (s & must_set):
            c = int(rng.choice(sorted(must_set)))
            s.update(range(c, min(c + int(rng.integers(1, 6)), max(must_set) + 1)))
        if rng.random() < 0.25:
            comp = set(range(256)) - s
            if comp & must_set:
                s = comp
        out[i] = class_words(s)
    return out


def random_tree(rng, n_nodes: int, leaf_byte, n_classes: int, p_class: float,
                weights=(("cat", 0.45), ("alt", 0.2), ("star", 0.1), ("plus", 0.1), ("opt", 0.15))):
    """A random AST with exactly ``n_nodes`` nodes.  Returns (builder, root, derives_empty).

    ``derives_empty`` (whether the tree's language holds the empty string) is
    tracked during generation so callers can reject trees whose search would be
    trivially true."""
    names = [w[0] for w in weights]
    probs = np.array([w[1] for w in weights], dtype=np.float64)
    probs /= probs.sum()
    unary_only = np.array([0.0 if nm in ("cat", "alt") else p for nm, p in zip(names, probs)])
    unary_only /= unary_only.sum()
    b = _Builder()
    # explicit post-order construction: frames of (budget, state, partial)
    result = []  # stack of (node_id, empty)
    work = [("gen", n_nodes)]
    while work:
        op = work.pop()
        if op[0] == "gen":
            budget = op[1]
            if budget == 1:
                if n_classes and rng.random() < p_class:
                    nid = b.add(CLASS, cls=int(rng.integers(0, n_classes)))
                else:
                    nid = b.add(BYTE, byte=int(leaf_byte(rng)))
                result.append((nid, False))
                continue
            pr = unary_only if budget == 2 else probs
            kind = names[int(rng.choice(len(names), p=pr))]
            if kind in ("cat", "alt"):
                left = int(rng.integers(1, budget - 1))
                work.append(("mk2", kind))
                work.append(("gen", budget - 1 - left))
                work.append(("gen", left))
            else:
                work.append(("mk1", kind))
                work.append(("gen", budget - 1))
        elif op[0] == "mk2":
            (y, ey), (x, ex) = result.pop(), result.pop()
            if op[1] == "cat":
                result.append((b.add(CAT, c0=x, c1=y), ex and ey))
            else:
                result.append((b.add(ALT, c0=x, c1=y), ex or ey))
        else:
            x, ex = result.pop()
            kind = {"star": STAR, "plus": PLUS, "opt": OPT}[op[1]]
            result.append((b.add(kind, c0=x), True if kind in (STAR, OPT) else ex))
    root, empty = result.pop()
    return b, root, empty


class _Uniforms:
    """Uniform [0, 1) draws served from bulk numpy blocks (fast in Python loops)."""

    def __init__(self, rng, block: int = 1 << 16):
        self.rng, self.block = rng, block
        self.buf, self.i = rng.random(block).tolist(), 0

    def __call__(self) -> float:
        if self.i == len(self.buf):
            self.buf, self.i = self.rng.random(self.block).tolist(), 0
        u = self.buf[self.i]
        self.i += 1
        return u


def sample_member(prog: Program, rng, max_len: int = 256, cap_rep: int = 4, _cache=None):
    """A random string of the expression's language by a random derivation:
    alternation uniform, star/plus repetitions geometric(1/2) capped at
    ``cap_rep``, optional a fair coin, classes a uniform member.  Returns None
    when the draw exceeds ``max_len``.  ``rng`` is a numpy Generator or a
    ``_Uniforms`` stream."""
    u = rng if isinstance(rng, _Uniforms) else _Uniforms(rng, 1024)
    if _cache is None:
        _cache = {}
    if "nodes" not in _cache:
        _cache["nodes"] = [tuple(int(v) for v in a) for a in prog.ast]
        _cache["members"] = [class_members(c) for c in prog.classes]
    nodes, members = _cache["nodes"], _cache["members"]
    out = bytearray()
    work = [int(prog.root)]
    while work:
        p = work.pop()
        if len(out) > max_len:
            return None
        k, byte, cls, c0, c1 = nodes[p]
        if k == BYTE:
            out.append(byte)
        elif k == CLASS:
            mem = members[cls]
            out.append(mem[int(u() * len(mem))])
        elif k == CAT:
            work += [c1, c0]
        elif k == ALT:
            work.append(c0 if u() < 0.5 else c1)
        elif k in (STAR, PLUS):
            reps = 0
            while reps < cap_rep and u() < 0.5:
                reps += 1
            if k == PLUS:
                reps = max(reps, 1)
            work += [c0] * reps
        elif k == OPT:
            if u() < 0.5:
                work.append(c0)
    return bytes(out) if len(out) <= max_len else None


# ---------------------------------------------------------------------------
# single: one ~200-node program, 1M x 256 B, 10% planted
# ---------------------------------------------------------------------------
def single_program(seed: int = 1, lo: int = 190, hi: int = 210) -> Program:
    rng = np.random.default_rng([seed, 10])
    classes = random_classes(rng, 8)
    while True:
        n_nodes = int(rng.integers(lo, hi + 1))
        b, root, empty = random_tree(rng, n_nodes, lambda r: int(r.integers(97, 123)), 8, 0.2)
        if not empty:
            return Program(b.array(), root, classes, True)


def single_strings(prog: Program, seed: int = 1, n: int = 1_000_000, length: int = 256,
                   plant_frac: float = 0.1):
    """Returns (strings, planted_ids)."""
    rng = np.random.default_rng([seed, 11])
    data = rng.integers(97, 123, size=n * length, dtype=np.uint8)
    offs = np.arange(n + 1, dtype=np.int64) * length
    n_plant = int(round(n * plant_frac))
    planted = np.sort(rng.choice(n, size=n_plant, replace=False)) if n_plant else np.zeros(0, np.int64)
    u = _Uniforms(rng)
    cache = {}
    for i in planted:
        while True:
            w = sample_member(prog, u, max_len=length, _cache=cache)
            if w is not None:
                break
        at = int(u() * (length - len(w) + 1))
        base = int(i) * length + at
        data[base : base + len(w)] = np.frombuffer(w, np.uint8)
    return Strings(data, offs), planted.astype(np.int64)


# ---------------------------------------------------------------------------
# multi: 16 programs over printable ASCII, log-normal Zipf lines
# ---------------------------------------------------------------------------
def zipf_cdf(s: float = 1.1, n: int = 95) -> np.ndarray:
    w = 1.0 / np.arange(1, n + 1, dtype=np.float64) ** s
    c = np.cumsum(w)
    return c / c[-1]


def zipf_bytes(rng, size: int, s: float = 1.1, chunk: int = 1 << 24) -> np.ndarray:
    cdf = zipf_cdf(s)
    out = np.empty(size, np.uint8)
    for a in range(0, size, chunk):
        e = min(size, a + chunk)
        u = rng.random(e - a)
        out[a:e] = (np.searchsorted(cdf, u, side="right") + 0x20).astype(np.uint8)
    return out


def multi_programs(seed: int = 2, count: int = 16, lo: int = 16, hi: int = 512):
    progs = []
    cdf = zipf_cdf()
    for p in range(count):
        rng = np.random.default_rng([seed + p, 20])
        classes = random_classes(rng, 8, universe=PRINTABLE, must=PRINTABLE)
        lit = lambda r: 0x20 + int(np.searchsorted(cdf, r.random(), side="right"))
        while True:
            n_nodes = int(rng.integers(lo, hi + 1))
            b, root, empty = random_tree(rng, n_nodes, lit, 8, 0.2)
            if not empty:
                break
        progs.append(Program(b.array(), root, classes, True))
    return progs


def lognormal_lengths(rng, n: int, mean: float, sigma: float, lo: int, hi: int, arithmetic_mean=True):
    mu = math.log(mean) - (sigma * sigma / 2 if arithmetic_mean else 0.0)
    lens = np.rint(rng.lognormal(mu, sigma, size=n)).astype(np.int64)
    return np.clip(lens, lo, hi)


def multi_lines(seed: int = 2, n: int = 4_000_000, mean: float = 120.0, sigma: float = 1.0,
                lo: int = 1, hi: int = 4096) -> Strings:
    rng = np.random.default_rng([seed, 21])
    lens = lognormal_lengths(rng, n, mean, sigma, lo, hi)
    offs = np.zeros(n + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    data = zipf_bytes(rng, int(offs[-1]))
    return Strings(data, offs)


# ---------------------------------------------------------------------------
# serving: request stream
# ---------------------------------------------------------------------------
@dataclass
class Request:
    program: Program
    strings: Strings
    arrival: float  # seconds from stream start


def serving_request(seed: int, idx: int, max_strings: int = 10_000) -> tuple:
    rng = np.random.default_rng([seed, 30, idx])
    n_nodes = int(round(math.exp(rng.uniform(math.log(8), math.log(512)))))
    cdf = zipf_cdf()
    lit = lambda r: 0x20 + int(np.searchsorted(cdf, r.random(), side="right"))
    classes = random_classes(rng, 8, universe=PRINTABLE, must=PRINTABLE)
    while True:
        b, root, empty = random_tree(rng, n_nodes, lit, 8, 0.2)
        if not empty:
            break
    prog = Program(b.array(), root, classes, True)
    count = int(round(math.exp(rng.uniform(0.0, math.log(max_strings)))))
    lens = lognormal_lengths(rng, count, 256.0, 1.0, 16, 8192, arithmetic_mean=False)
    offs = np.zeros(count + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    data = zipf_bytes(rng, int(offs[-1]))
    return prog, Strings(data, offs)


def poisson_arrivals(seed: int, n: int, rate: float) -> np.ndarray:
    rng = np.random.default_rng([seed, 31])
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


# ---------------------------------------------------------------------------
# pathological: X^k t
# ---------------------------------------------------------------------------
def pathological_program(family: str, k: int) -> Program:
    """family 'nested': (((a*)*)*)^k b  (5k+1 nodes); 'altstar': ((a|aa)*)^k c (7k+1 nodes)."""
    b = _Builder()
    acc = -1
    for _ in range(k):
        if family == "nested":
            x = b.add(BYTE, byte=97)
            for _ in range(3):
                x = b.add(STAR, c0=x)
        elif family == "altstar":
            a1 = b.add(BYTE, byte=97)
            a2 = b.add(BYTE, byte=97)
            a3 = b.add(BYTE, byte=97)
            aa = b.add(CAT, c0=a2, c1=a3)
            x = b.add(STAR, c0=b.add(ALT, c0=a1, c1=aa))
        else:
            raise ValueError(family)
        acc = x if acc < 0 else b.add(CAT, c0=acc, c1=x)
    t = b.add(BYTE, byte=98 if family == "nested" else 99)
    root = b.add(CAT, c0=acc, c1=t)
    return Program(b.array(), root, np.zeros((0, 4), np.uint64), False)


def pathological_strings(family: str, n_len: int, count: int = 256) -> Strings:
    """count strings of length n_len: the first half a^n, the second half a^(n-1) t."""
    t = 98 if family == "nested" else 99
    data = np.full(count * n_len, 97, np.uint8)
    offs = np.arange(count + 1, dtype=np.int64) * n_len
    if n_len > 0:
        for i in range(count // 2, count):
            data[(i + 1) * n_len - 1] = t
    return Strings(data, offs)
