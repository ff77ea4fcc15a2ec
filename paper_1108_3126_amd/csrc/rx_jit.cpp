// Bit-sliced node circuit: code generation and run-time compilation.
//
// The lockstep macro step (Def. 5.2) is evaluated as a boolean circuit over the
// node tree -- the per-node processes of Section 7 (each node forwards the
// thread to its children or its continuation; leaves wait for the input byte)
// with messages as bits.  One 32-bit word per node holds that node's signal for
// 32 strings at once, so every bitwise instruction advances 32 strings.
//
// For one input byte c and current leaf set S (X_x = S_x AND [c in label x]):
//   bottom-up  out(p): a thread that consumed c inside p's subtree reaches cont p
//     leaf x        out = X_x
//     eps           out = 0
//     cat(a, b)     out = out b  OR (nullable b AND out a)
//     alt(a, b)     out = out a  OR out b
//     star/plus/opt out = out a
//   top-down   in(p): a thread arrives at p during the evolution of this step
//     root          in = 0           (no thread re-enters the root)
//     cat(a, b)     in a = in p,  in b = out a OR (nullable a AND in p)
//     alt(a, b)     in a = in b = in p
//     star/plus     in a = in p OR out a   (the body loops back, Fig. 4.2)
//     opt           in a = in p
//   S'_x = in(x) for every leaf x; the accept bit (null reached) is out(root).
// Every non-consuming path of Fig. 4.2 is covered by these two passes, so no
// fixpoint iteration is needed even though cont pointers form cycles
// (Section 4 notes the cycle through a nested star).  OR-ing signals that
// arrive at the same node is the removal of duplicate threads by pointer
// equality.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "rx_internal.h"

namespace rx {

namespace {

// ---------------------------------------------------------------------------
// a tiny expression emitter with constant folding
// ---------------------------------------------------------------------------
struct V {
    int c;          // 0 or 1: constant all-zeros / all-ones; -1: a named value
    std::string n;  // C expression name when c == -1
};

struct Emitter {
    std::ostringstream code;
    int tmp = 0;
    int ops = 0;
    V zero{0, ""}, one{1, ""};

    std::unordered_map<std::string, std::string> memo;   // expression -> its temporary
    std::unordered_map<std::string, std::vector<int>> deps;   // temporary -> the state words it reads

    // the state words a value reads (sorted)
    std::vector<int> reads(const std::string& n) const {
        if (n.rfind("s[", 0) == 0) return {std::atoi(n.c_str() + 2)};
        auto it = deps.find(n);
        return it == deps.end() ? std::vector<int>{} : it->second;
    }
    V def(const std::string& expr, const std::string& a, const std::string& b = "") {
        auto it = memo.find(expr);
        if (it != memo.end()) return V{-1, it->second};
        const std::string name = "t" + std::to_string(tmp++);
        code << "    const u32 " << name << " = " << expr << ";\n";
        ++ops;
        memo.emplace(expr, name);
        std::vector<int> d = reads(a), e = reads(b), u;
        std::set_union(d.begin(), d.end(), e.begin(), e.end(), std::back_inserter(u));
        if (!u.empty()) deps.emplace(name, std::move(u));
        return V{-1, name};
    }
    static std::string str(const V& v) {
        if (v.c == 0) return "0u";
        if (v.c == 1) return "0xffffffffu";
        return v.n;
    }
    V AND(const V& a, const V& b) {
        if (a.c == 0 || b.c == 0) return zero;
        if (a.c == 1) return b;
        if (b.c == 1) return a;
        if (a.n == b.n) return a;
        return a.n < b.n ? def(a.n + " & " + b.n, a.n, b.n) : def(b.n + " & " + a.n, a.n, b.n);
    }
    V OR(const V& a, const V& b) {
        if (a.c == 1 || b.c == 1) return one;
        if (a.c == 0) return b;
        if (b.c == 0) return a;
        if (a.n == b.n) return a;
        return a.n < b.n ? def(a.n + " | " + b.n, a.n, b.n) : def(b.n + " | " + a.n, a.n, b.n);
    }
    V NOT(const V& a) {
        if (a.c == 0) return one;
        if (a.c == 1) return zero;
        return def("~" + a.n, a.n);
    }
};

// Bit-sliced membership of the input byte in a byte set, from the eight bit
// planes b0..b7 (plane k holds bit k of the current byte of 32 strings).
// Products over three fixed bit groups are shared between labels:
//   H[h]: bits 7..5 == h,  M[u]: bits 4..2 == u,  Q[v]: bits 1..0 == v.
struct Decoder {
    Emitter& E;
    V H[8], M[8], Q[4];
    bool hH[8] = {}, hM[8] = {}, hQ[4] = {};
    explicit Decoder(Emitter& e) : E(e) {}

    V lit(int bit, int val) { return val ? V{-1, "b" + std::to_string(bit)} : V{-1, "nb" + std::to_string(bit)}; }
    V prod3(int hi_bit, int v) {
        return E.AND(E.AND(lit(hi_bit, (v >> 2) & 1), lit(hi_bit - 1, (v >> 1) & 1)), lit(hi_bit - 2, v & 1));
    }
    V getH(int h) { if (!hH[h]) { H[h] = prod3(7, h); hH[h] = true; } return H[h]; }
    V getM(int u) { if (!hM[u]) { M[u] = prod3(4, u); hM[u] = true; } return M[u]; }
    V getQ(int v) {
        if (!hQ[v]) { Q[v] = E.AND(lit(1, (v >> 1) & 1), lit(0, v & 1)); hQ[v] = true; }
        return Q[v];
    }
    V decode(const std::array<uint64_t, 4>& set) {
        int cnt = 0;
        for (int w = 0; w < 4; ++w) cnt += __builtin_popcountll(set[w]);
        if (cnt == 0) return E.zero;
        if (cnt == 256) return E.one;
        if (cnt > 128) {
            std::array<uint64_t, 4> inv = {~set[0], ~set[1], ~set[2], ~set[3]};
            return E.NOT(decode(inv));
        }
        auto has = [&](int b) { return (set[b >> 6] >> (b & 63)) & 1; };
        V acc = E.zero;
        for (int h = 0; h < 8; ++h) {
            int n_h = 0;
            for (int b = h * 32; b < h * 32 + 32; ++b) n_h += (int)has(b);
            if (n_h == 0) continue;
            V term;
            if (n_h == 32) {
                term = getH(h);
            } else {
                V inner = E.zero;
                for (int u = 0; u < 8; ++u) {
                    const int b0 = h * 32 + u * 4;
                    int mask = 0;
                    for (int v = 0; v < 4; ++v) mask |= (int)has(b0 + v) << v;
                    if (!mask) continue;
                    V t;
                    if (mask == 15) {
                        t = getM(u);
                    } else {
                        V g = E.zero;
                        for (int v = 0; v < 4; ++v)
                            if (mask >> v & 1) g = E.OR(g, getQ(v));
                        t = E.AND(getM(u), g);
                    }
                    inner = E.OR(inner, t);
                }
                term = E.AND(getH(h), inner);
            }
            acc = E.OR(acc, term);
        }
        return acc;
    }
};

bool is_leaf_kind(int k) { return k == RX_BYTE || k == RX_CLASS; }

// The search prefix (any byte)* of RX_SEARCH keeps its leaf live forever:
// that leaf's state is the constant all-ones.
int search_prefix_leaf(const Program& P) {
    if (!(P.flags & RX_SEARCH) || P.kind[0] != RX_CAT) return -1;
    const int left = P.c0[0];
    if (left < 0 || P.kind[left] != RX_CAT) return -1;
    const int pre = P.c0[left];
    if (pre < 0 || P.kind[pre] != RX_STAR) return -1;
    const int dot = P.c0[pre];
    if (dot < 0 || P.kind[dot] != RX_CLASS) return -1;
    const auto& c = P.classes[P.label[dot]];
    if ((c[0] & c[1] & c[2] & c[3]) != ~0ull) return -1;
    return dot;
}

// The search suffix (any byte)* of RX_SEARCH: once its leaf is live it stays
// live and the string accepts.
int search_suffix_leaf(const Program& P) {
    if (search_prefix_leaf(P) < 0) return -1;
    const int suf = P.c1[0];
    if (suf < 0 || P.kind[suf] != RX_STAR) return -1;
    const int dot = P.c0[suf];
    if (dot < 0 || P.kind[dot] != RX_CLASS) return -1;
    const auto& c = P.classes[P.label[dot]];
    if ((c[0] & c[1] & c[2] & c[3]) != ~0ull) return -1;
    return dot;
}

std::array<uint64_t, 4> label_set(const Program& P, int p) {
    std::array<uint64_t, 4> s = {0, 0, 0, 0};
    if (P.kind[p] == RX_BYTE) s[P.label[p] >> 6] |= 1ull << (P.label[p] & 63);
    else s = P.classes[P.label[p]];
    return s;
}

}  // namespace

// Generates the step function (device/host neutral C++): rx_step(s, acc, b0..b7)
// plus the initial state.  Fills n_state (state words) and n_ops.
std::string jit_step_source(const Program& P, int* n_state, int* n_ops, int* suffix_slot) {
    const int nt = P.n_tree;
    std::vector<char> nu(nt, 0);
    for (int p = nt - 1; p >= 0; --p) {
        const int a = P.c0[p], b = P.c1[p];
        switch (P.kind[p]) {
        case RX_EPS: nu[p] = 1; break;
        case RX_BYTE: case RX_CLASS: nu[p] = 0; break;
        case RX_CAT: nu[p] = nu[a] && nu[b]; break;
        case RX_ALT: nu[p] = nu[a] || nu[b]; break;
        case RX_STAR: case RX_OPT: nu[p] = 1; break;
        case RX_PLUS: nu[p] = nu[a]; break;
        default: nu[p] = 0; break;
        }
    }
    auto is_first = [&](int r) { return ((P.first[r >> 5] >> (r & 31)) & 1) != 0; };
    // Leaves that hold the same word at every step share one state word, and
    // leaves that are constant need none.  The classes are found by partition
    // refinement: start optimistic (every leaf live at the start is the
    // constant all-ones, every other the constant zero), write the update of
    // each leaf in terms of the current classes, and split a class whose
    // leaves' updates differ (a constant class also loses the leaves whose
    // update is not that constant); when nothing splits, every leaf of a class
    // has its start value and its update in common, so by induction over the
    // steps they agree forever.  Last, a word that the accept bit does not
    // read, directly or through the updates of words it reads, is dropped
    // (read as zero): it cannot change the result.
    constexpr int kOne = -1, kZero = -2, kDead = -3;
    std::vector<int> grp(P.m, -1), kind;   // leaf -> class; class -> kOne, kZero, kDead or 0 (a word)
    kind = {kOne, kZero};
    for (int r = 0; r < P.L; ++r) grp[P.leaf_node[r]] = is_first(r) ? 0 : 1;
    std::vector<int> slot(P.m, kOne);
    int ns = 0;
    auto number = [&]() {
        std::vector<int> word(kind.size(), -1);
        ns = 0;
        for (int r = 0; r < P.L; ++r) {
            const int x = P.leaf_node[r], g = grp[x];
            if (kind[g] != 0) slot[x] = kind[g];
            else {
                if (word[g] < 0) word[g] = ns++;
                slot[x] = word[g];
            }
        }
    };
    number();
    for (;;) {
        Emitter E;
        E.code << "    const u32 nb0 = ~b0, nb1 = ~b1, nb2 = ~b2, nb3 = ~b3, nb4 = ~b4, nb5 = ~b5, nb6 = ~b6, nb7 = ~b7;\n";
        Decoder D(E);
        // one decoded mask per distinct label
        std::vector<std::array<uint64_t, 4>> seen_sets;
        std::vector<V> seen_vals;
        std::vector<V> lab(P.m, E.zero);
        for (int r = 0; r < P.L; ++r) {
            const int x = P.leaf_node[r];
            const auto set = label_set(P, x);
            int found = -1;
            for (size_t i = 0; i < seen_sets.size(); ++i)
                if (seen_sets[i] == set) { found = (int)i; break; }
            if (found < 0) {
                seen_sets.push_back(set);
                seen_vals.push_back(D.decode(set));
                found = (int)seen_vals.size() - 1;
            }
            lab[x] = seen_vals[found];
        }
        auto state = [&](int x) {
            return slot[x] == kOne ? E.one : slot[x] < 0 ? E.zero : V{-1, "s[" + std::to_string(slot[x]) + "]"};
        };
        std::vector<V> out(nt, E.zero), in(nt, E.zero);
        for (int p = nt - 1; p >= 0; --p) {
            const int a = P.c0[p], b = P.c1[p];
            switch (P.kind[p]) {
            case RX_BYTE: case RX_CLASS: out[p] = E.AND(state(p), lab[p]); break;
            case RX_EPS: out[p] = E.zero; break;
            case RX_CAT: out[p] = E.OR(out[b], nu[b] ? out[a] : E.zero); break;
            case RX_ALT: out[p] = E.OR(out[a], out[b]); break;
            case RX_STAR: case RX_PLUS: case RX_OPT: out[p] = out[a]; break;
            default: break;
            }
        }
        in[0] = E.zero;
        for (int p = 0; p < nt; ++p) {
            const int a = P.c0[p], b = P.c1[p];
            switch (P.kind[p]) {
            case RX_CAT:
                in[a] = in[p];
                in[b] = E.OR(out[a], nu[a] ? in[p] : E.zero);
                break;
            case RX_ALT: in[a] = in[p]; in[b] = in[p]; break;
            case RX_STAR: case RX_PLUS: in[a] = E.OR(in[p], out[a]); break;
            case RX_OPT: in[a] = in[p]; break;
            default: break;
            }
        }
        // refine: (class, update) -> class
        std::vector<int> ngrp(P.m, -1), nkind;
        std::unordered_map<std::string, int> cls;
        for (int r = 0; r < P.L; ++r) {
            const int x = P.leaf_node[r], g = grp[x];
            const std::string upd = Emitter::str(in[x]);
            auto it = cls.emplace(std::to_string(g) + ":" + upd, (int)nkind.size());
            if (it.second) {
                const bool stays = kind[g] == kDead || (kind[g] == kOne && in[x].c == 1) ||
                                   (kind[g] == kZero && in[x].c == 0);
                nkind.push_back(stays ? kind[g] : 0);
            }
            ngrp[x] = it.first->second;
        }
        bool same = nkind.size() == kind.size();
        for (int r = 0; same && r < P.L; ++r) {
            const int x = P.leaf_node[r];
            same = kind[grp[x]] == nkind[ngrp[x]];
        }
        if (!same) {
            grp = ngrp;
            kind = nkind;
            number();
            continue;
        }
        // the words the accept bit reads
        std::vector<V> upd(ns > 0 ? ns : 1, E.zero);
        for (int r = 0; r < P.L; ++r) {
            const int x = P.leaf_node[r];
            if (slot[x] >= 0) upd[slot[x]] = in[x];
        }
        std::vector<char> live(ns > 0 ? ns : 1, 0);
        std::vector<int> todo = out[0].c < 0 ? E.reads(out[0].n) : std::vector<int>{};
        while (!todo.empty()) {
            const int k = todo.back();
            todo.pop_back();
            if (live[k]) continue;
            live[k] = 1;
            if (upd[k].c < 0)
                for (int j : E.reads(upd[k].n)) todo.push_back(j);
        }
        bool dropped = false;
        for (int r = 0; r < P.L; ++r) {
            const int x = P.leaf_node[r];
            if (slot[x] >= 0 && !live[slot[x]]) {
                kind[grp[x]] = kDead;
                dropped = true;
            }
        }
        if (dropped) {
            number();
            continue;
        }
        // commit the new state after every value is computed
        std::ostringstream tail;
        std::vector<char> done(ns > 0 ? ns : 1, 0);
        for (int r = 0; r < P.L; ++r) {
            const int x = P.leaf_node[r];
            if (slot[x] < 0 || done[slot[x]]) continue;
            done[slot[x]] = 1;
            tail << "    s[" << slot[x] << "] = " << Emitter::str(in[x]) << ";\n";
        }
        tail << "    acc = " << Emitter::str(out[0]) << ";\n";
        std::ostringstream src;
        src << "#define RX_NS " << (ns > 0 ? ns : 1) << "\n";
        src << "__device__ __forceinline__ void rx_step(u32 (&s)[RX_NS], u32& acc, u32 b0, u32 b1, u32 b2, u32 b3,"
               " u32 b4, u32 b5, u32 b6, u32 b7) {\n";
        src << E.code.str() << tail.str() << "}\n";
        src << "__device__ __forceinline__ void rx_init(u32 (&s)[RX_NS], u32& acc) {\n";
        for (int k = 0; k < (ns > 0 ? ns : 1); ++k) src << "    s[" << k << "] = 0u;\n";
        std::fill(done.begin(), done.end(), 0);
        for (int r = 0; r < P.L; ++r) {
            const int x = P.leaf_node[r];
            if (slot[x] >= 0 && !done[slot[x]] && is_first(r)) {
                done[slot[x]] = 1;
                src << "    s[" << slot[x] << "] = 0xffffffffu;\n";
            }
        }
        src << "    acc = " << (P.nullable ? "0xffffffffu" : "0u") << ";\n}\n";
        if (n_state) *n_state = ns;
        if (n_ops) *n_ops = E.ops;
        if (suffix_slot) {
            const int suf = search_suffix_leaf(P);
            *suffix_slot = suf >= 0 && slot[suf] >= 0 ? slot[suf] : -1;
        }
        return src.str();
    }
}

// 32x32 bit transpose: afterwards a[k] bit j == (before) a[j] bit k.  The two
// byte-granular stages are byte permutes (v_perm_b32, one instruction per
// word); the three bit stages are a shift plus a bit-field insert per word.
const char* kTransposeSource = R"RX(
#ifndef RX_PERM
#define RX_PERM(hi, lo, sel) __builtin_amdgcn_perm((hi), (lo), (sel))
#endif
// bit select (a & m) | (b & ~m) as one 3-input bit operation; the table
// 0xE4 is that function evaluated on the operand patterns a = 0xF0,
// b = 0xCC, m = 0xAA
#ifndef RX_SEL
#define RX_SEL(a, b, m) __builtin_amdgcn_bitop3_b32((a), (b), (m), 0xE4)
#endif
__device__ __forceinline__ void rx_transpose32(u32 (&a)[32]) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const u32 x = a[j], y = a[j + 16];
        a[j] = RX_PERM(y, x, 0x05040100u);
        a[j + 16] = RX_PERM(y, x, 0x07060302u);
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        if ((j & 8) == 0) {
            const u32 x = a[j], y = a[j + 8];
            a[j] = RX_PERM(y, x, 0x06020400u);
            a[j + 8] = RX_PERM(y, x, 0x07030501u);
        }
    }
#pragma unroll
    for (unsigned d = 4, m = 0x0f0f0f0fu; d > 0; d >>= 1, m ^= (m << d)) {
#pragma unroll
        for (unsigned j = 0; j < 32; ++j) {
            if ((j & d) == 0) {
                const u32 x = a[j], y = a[j + d];
                a[j] = RX_SEL(x, y << d, m);
                a[j + d] = RX_SEL(x >> d, y, m);
            }
        }
    }
}
)RX";

// Chunk-parallel form of a circuit of at most two state words.  The step of
// Def. 5.1 maps (state, byte) to a state and an accept bit, so a chunk of a
// string is a map from the R = 2^NS states to states, with the accept bit
// after its last byte; running the chunk once from each of the R states (all
// 32 chunks of a lane from the same state, word k all-ones where bit k of
// the state index is set) gives it, and the maps of consecutive chunks
// compose.  A map is one word: bits 2r, 2r+1 the state after the chunk from
// state r, bit 8 + r the accept bit after its last byte, bit 12 set when the
// chunk has bytes (clear: the identity).
const char* kChunkSource = R"RX(
// Bytes [off, off + 16) of a chunk of len bytes at c, little-endian in four
// words (bytes at or past len unspecified); only the 16-byte aligned blocks
// that hold a byte of the chunk are read.
__device__ __forceinline__ void rx_chunk_window16(const unsigned char* c, long long len, long long off,
                                                  u32 (&w)[4]) {
    w[0] = w[1] = w[2] = w[3] = 0u;
    if (off >= len) return;
    const unsigned long long addr = (unsigned long long)(c + off), end = (unsigned long long)(c + len);
    const unsigned long long a = addr & ~15ull;
    const u32 sh = (u32)(addr & 15ull);
    u32 b[8];
    const u32* p0 = (const u32*)a;
    b[0] = p0[0]; b[1] = p0[1]; b[2] = p0[2]; b[3] = p0[3];
    if (a + 16 < end) {
        const u32* p1 = (const u32*)(a + 16);
        b[4] = p1[0]; b[5] = p1[1]; b[6] = p1[2]; b[7] = p1[3];
    } else {
        b[4] = b[5] = b[6] = b[7] = 0u;
    }
    if (sh & 8) {
#pragma unroll
        for (int k = 0; k < 6; ++k) b[k] = b[k + 2];
    }
    if (sh & 4) {
#pragma unroll
        for (int k = 0; k < 5; ++k) b[k] = b[k + 1];
    }
    const u32 r = (sh & 3) * 8;
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = r ? (b[k] >> r) | (b[k + 1] << (32 - r)) : b[k];
}

#if RX_NS <= 2
#define RX_R (1 << RX_NS)
__device__ __forceinline__ u32 rx_fn_compose(u32 f, u32 g) {   // f, then g
    if (!(g & 0x1000u)) return f;
    if (!(f & 0x1000u)) return g;
    u32 h = 0x1000u;
#pragma unroll
    for (int r = 0; r < RX_R; ++r) {
        const u32 m = (f >> (2 * r)) & 3u;
        h |= ((g >> (2 * m)) & 3u) << (2 * r);
        h |= ((g >> (8 + m)) & 1u) << (8 + r);
    }
    return h;
}

// The composed map of chunks 32 lane .. 32 lane + 31 (Lc bytes each) of the
// string at s of `length` bytes.
__device__ __forceinline__ u32 rx_chunk_lane(const unsigned char* s, long long length, long long Lc, int lane) {
    int len[32];   // Lc < 2^31 (the host allows strings of up to 2^40 bytes)
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const long long start = (32ll * lane + j) * Lc;
        len[j] = start < length ? (int)(length - start < Lc ? length - start : Lc) : 0;
    }
    u32 st[RX_R][RX_NS], acc[RX_R];
#pragma unroll
    for (int r = 0; r < RX_R; ++r) {
#pragma unroll
        for (int k = 0; k < RX_NS; ++k) st[r][k] = ((r >> k) & 1) ? 0xffffffffu : 0u;
        acc[r] = 0u;
    }
    for (long long p = 0; p < Lc && p < len[0]; p += 16) {
        u32 win[32][4];
#pragma unroll
        for (int j = 0; j < 32; ++j) rx_chunk_window16(s + (32ll * lane + j) * Lc, len[j], p, win[j]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            u32 x[32];
#pragma unroll
            for (int j = 0; j < 32; ++j) x[j] = win[j][q];
            rx_transpose32(x);   // x[8 i + b]: bit b of byte i of the four, bit j = chunk j
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long pos = p + 4 * q + i;
                u32 v = 0u;
#pragma unroll
                for (int j = 0; j < 32; ++j) v |= (len[j] > pos ? 1u : 0u) << j;
#pragma unroll
                for (int r = 0; r < RX_R; ++r) {
                    u32 ns[RX_NS];
#pragma unroll
                    for (int k = 0; k < RX_NS; ++k) ns[k] = st[r][k];
                    u32 a = acc[r];
                    rx_step(ns, a, x[8 * i], x[8 * i + 1], x[8 * i + 2], x[8 * i + 3], x[8 * i + 4], x[8 * i + 5],
                            x[8 * i + 6], x[8 * i + 7]);
#pragma unroll
                    for (int k = 0; k < RX_NS; ++k) st[r][k] = (ns[k] & v) | (st[r][k] & ~v);
                    acc[r] = (a & v) | (acc[r] & ~v);
                }
            }
        }
    }
    u32 f = 0u;
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        if (len[j] == 0) continue;
        u32 g = 0x1000u;
#pragma unroll
        for (int r = 0; r < RX_R; ++r) {
            u32 m = 0u;
#pragma unroll
            for (int k = 0; k < RX_NS; ++k) m |= ((st[r][k] >> j) & 1u) << k;
            g |= m << (2 * r);
            g |= ((acc[r] >> j) & 1u) << (8 + r);
        }
        f = rx_fn_compose(f, g);
    }
    return f;
}

// The result of a string from the composed map of all its chunks.
__device__ __forceinline__ unsigned char rx_chunk_result(u32 f) {
    u32 s0[RX_NS], a0;
    rx_init(s0, a0);
    u32 r0 = 0u;
#pragma unroll
    for (int k = 0; k < RX_NS; ++k) r0 |= (s0[k] & 1u) << k;
    return (unsigned char)((f & 0x1000u) ? (f >> (8 + r0)) & 1u : a0 & 1u);
}
#endif

#if RX_NS <= 31
#define RX_M (RX_NS + 1)
// Affine maps of the state words.  Every update of the step is an OR of
// terms that read at most one word (a leaf's word AND its label, or a label
// alone), and so is the accept bit, so a chunk maps a state T (bit k: word
// k) to m[0] | the m[k + 1] of T's words: m[0] the image of the empty state,
// m[k + 1] of word k alone, bit 31 of each the accept bit after the chunk's
// last byte.  NS + 1 runs of a chunk give its map, and maps compose.
__device__ __forceinline__ u32 rx_aff_apply(const u32 (&m)[RX_M], u32 t) {
    u32 r = m[0];
#pragma unroll
    for (int k = 0; k < RX_NS; ++k) r |= (0u - ((t >> k) & 1u)) & m[k + 1];
    return r;
}
__device__ __forceinline__ void rx_aff_compose(u32 (&f)[RX_M], const u32 (&g)[RX_M]) {   // f := f, then g
#pragma unroll
    for (int i = 0; i < RX_M; ++i) f[i] = rx_aff_apply(g, f[i] & 0x7fffffffu);
}

// The lengths (at most Lc) of chunks 32 lane .. 32 lane + 31 of a segment of
// seglen bytes.
__device__ __forceinline__ void rx_aff_lens(long long seglen, long long Lc, int lane, int (&len)[32]) {
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const long long start = (32ll * lane + j) * Lc;
        len[j] = start < seglen ? (int)(seglen - start < Lc ? seglen - start : Lc) : 0;   // Lc < 2^31
    }
}

// Positions p .. p + 15 of those chunks as bit planes: y[q][8 i + b] is bit b
// of byte 4 q + i of every chunk (bit j = chunk 32 lane + j).
__device__ __forceinline__ void rx_aff_planes(const unsigned char* s, long long Lc, int lane, const int (&len)[32],
                                              long long p, u32 (&y)[4][32]) {
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        u32 w[4];
        rx_chunk_window16(s + (32ll * lane + j) * Lc, len[j], p, w);
#pragma unroll
        for (int q = 0; q < 4; ++q) y[q][j] = w[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) rx_transpose32(y[q]);
}

// The chunks that still have bytes at positions p .. p + 15 (vm[t]: bit j
// for chunk 32 lane + j at position p + t).
__device__ __forceinline__ void rx_aff_masks(const int (&len)[32], long long p, u32 (&vm)[16]) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        u32 v = 0u;
#pragma unroll
        for (int j = 0; j < 32; ++j) v |= (len[j] > p + t ? 1u : 0u) << j;
        vm[t] = v;
    }
}

// The circuit over those 16 positions, each chunk's state frozen once it has
// ended.
__device__ __forceinline__ void rx_aff_steps(const u32 (&y)[4][32], const u32 (&vm)[16], u32 (&st)[RX_NS],
                                             u32& acc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const u32 v = vm[4 * q + i];
            u32 ns[RX_NS];
#pragma unroll
            for (int k = 0; k < RX_NS; ++k) ns[k] = st[k];
            u32 a = acc;
            rx_step(ns, a, y[q][8 * i], y[q][8 * i + 1], y[q][8 * i + 2], y[q][8 * i + 3], y[q][8 * i + 4],
                    y[q][8 * i + 5], y[q][8 * i + 6], y[q][8 * i + 7]);
#pragma unroll
            for (int k = 0; k < RX_NS; ++k) st[k] = (ns[k] & v) | (st[k] & ~v);
            acc = (a & v) | (acc & ~v);
        }
    }
}

// Word r of the maps of the lane's 32 chunks from a run's final words: bit k
// word k, bit 31 the accept bit, to out[(r * 32 + j) * stride].
__device__ __forceinline__ void rx_aff_store(const u32 (&st)[RX_NS], u32 acc, int r, u32* out, int stride) {
    u32 x[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) x[k] = k < RX_NS ? st[k] : k == 31 ? acc : 0u;
    rx_transpose32(x);
#pragma unroll
    for (int j = 0; j < 32; ++j) out[(r * 32 + j) * stride] = x[j];
}

// The maps of chunks 32 lane .. 32 lane + 31 of the seglen bytes at s: run r
// (0: from the empty state, k + 1: from word k alone) gives word r of every
// chunk's map, written to out[(r * 32 + j) * stride] for chunk 32 lane + j
// (bit k: word k after the chunk, bit 31: the accept bit after its last
// byte).  Chunks of 16 bytes are one window: its planes are made once and
// every run reuses them (a loop of its own, so the other form's values are
// not live there).
__device__ __forceinline__ void rx_aff_lane_maps(const unsigned char* s, long long seglen, long long Lc, int lane,
                                                 u32* out, int stride) {
    int len[32];
    rx_aff_lens(seglen, Lc, lane, len);
    u32 y[4][32], vm[16];
    if (Lc == 16) {
        // one window: its planes and masks made once, kept for every run
        const bool live = len[0] > 0;
        rx_aff_planes(s, Lc, lane, len, 0, y);
        rx_aff_masks(len, 0, vm);
#pragma clang loop unroll(disable)
        for (int r = 0; r < RX_M; ++r) {
            u32 st[RX_NS], acc = 0u;
#pragma unroll
            for (int k = 0; k < RX_NS; ++k) st[k] = r == k + 1 ? 0xffffffffu : 0u;
            if (live) rx_aff_steps(y, vm, st, acc);
            rx_aff_store(st, acc, r, out, stride);
        }
        return;
    }
#pragma clang loop unroll(disable)
    for (int r = 0; r < RX_M; ++r) {
        u32 st[RX_NS], acc = 0u;
#pragma unroll
        for (int k = 0; k < RX_NS; ++k) st[k] = r == k + 1 ? 0xffffffffu : 0u;
        for (long long p = 0; p < Lc && p < len[0]; p += 16) {
            rx_aff_planes(s, Lc, lane, len, p, y);
            rx_aff_masks(len, p, vm);
            rx_aff_steps(y, vm, st, acc);
        }
        rx_aff_store(st, acc, r, out, stride);
    }
}

// The start state as a word set, and the result of a string from the
// composed map of its chunks (any: the string has bytes).
__device__ __forceinline__ unsigned char rx_aff_result(const u32 (&f)[RX_M], bool any) {
    u32 s0[RX_NS], a0;
    rx_init(s0, a0);
    u32 t0 = 0u;
#pragma unroll
    for (int k = 0; k < RX_NS; ++k) t0 |= (s0[k] & 1u) << k;
    return (unsigned char)(any ? rx_aff_apply(f, t0) >> 31 : a0 & 1u);
}
#endif
)RX";

// One wavefront per string; lane l runs chunks 32 l .. 32 l + 31 of 2,048
// chunks of Lc bytes (a multiple of 16), and the lanes' maps compose in lane
// order in six shuffle steps (after step d, lane l with l % 2d == 0 holds the
// map of lanes l .. l + 2d - 1).
const char* kChunkKernelSource = R"RX(
#if RX_NS <= 2
extern "C" __global__ __launch_bounds__(64) void rx_sliced_chunks(const unsigned char* __restrict__ bytes,
                                                                  long long length, long long n,
                                                                  unsigned char* __restrict__ out) {
    const long long i = blockIdx.x;
    if (i >= n) return;
    const int lane = threadIdx.x;
    const long long Lc = ((length + 2047) / 2048 + 15) / 16 * 16;
    u32 f = rx_chunk_lane(bytes + i * length, length, Lc, lane);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const u32 g = __shfl_down(f, d, 64);
        if ((lane & (2 * d - 1)) == 0) f = rx_fn_compose(f, g);
    }
    if (lane == 0) out[i] = rx_chunk_result(f);
}
#endif

#if RX_NS <= 31
// One long string: one wavefront per segment of 2,048 chunks of Lc bytes.
// Lane l runs the NS + 1 runs of its 32 chunks, keeping every chunk's map in
// the workspace (chunk_maps, 2,048 x (NS + 1) words per segment; word r of
// chunk 32 l + j at ((g (NS + 1) + r) 32 + j) 64 + l, so a wavefront's stores
// and loads are coalesced), composes its chunks in order, and the lanes' maps
// compose in lane order in six shuffle steps; the segment's map goes to
// seg_maps[g * (NS + 1) ..].
extern "C" __global__ __launch_bounds__(64) void rx_long_chunks(const unsigned char* __restrict__ bytes,
                                                                long long length, long long Lc,
                                                                u32* __restrict__ seg_maps,
                                                                u32* __restrict__ chunk_maps) {
    const long long g = blockIdx.x;
    const int lane = threadIdx.x;
    const long long base = g * 2048 * Lc;
    const long long seglen = length - base < 2048 * Lc ? length - base : 2048 * Lc;
    u32* maps = chunk_maps + g * RX_M * 2048;
    rx_aff_lane_maps(bytes + base, seglen, Lc, lane, maps + lane, 64);
    u32 f[RX_M];
    bool any = false;
    for (int j = 0; j < 32; ++j) {
        if ((32ll * lane + j) * Lc >= seglen) break;
        u32 h[RX_M];
#pragma unroll
        for (int i = 0; i < RX_M; ++i) h[i] = maps[(i * 32 + j) * 64 + lane];
        if (any) rx_aff_compose(f, h);
        else {
#pragma unroll
            for (int i = 0; i < RX_M; ++i) f[i] = h[i];
            any = true;
        }
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        u32 h[RX_M];
#pragma unroll
        for (int i = 0; i < RX_M; ++i) h[i] = __shfl_down(any ? f[i] : 0u, d, 64);
        const int ha = __shfl_down(any ? 1 : 0, d, 64);
        if ((lane & (2 * d - 1)) == 0 && lane + d < 64 && ha) {
            if (any) rx_aff_compose(f, h);
            else {
#pragma unroll
                for (int i = 0; i < RX_M; ++i) f[i] = h[i];
                any = true;
            }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < RX_M; ++i) seg_maps[g * RX_M + i] = f[i];
    }
}

// The G segments' maps in order (one wavefront: lane l composes a run of
// consecutive segments, then the lanes in order), applied to the start state.
extern "C" __global__ __launch_bounds__(64) void rx_long_compose(const u32* __restrict__ seg_maps, long long G,
                                                                 unsigned char* __restrict__ out) {
    const int lane = threadIdx.x;
    const long long per = (G + 63) / 64, g0 = lane * per, g1 = g0 + per < G ? g0 + per : G;
    u32 f[RX_M];
    bool any = false;
    for (long long g = g0; g < g1; ++g) {
        u32 h[RX_M];
#pragma unroll
        for (int i = 0; i < RX_M; ++i) h[i] = seg_maps[g * RX_M + i];
        if (any) rx_aff_compose(f, h);
        else {
#pragma unroll
            for (int i = 0; i < RX_M; ++i) f[i] = h[i];
            any = true;
        }
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        u32 h[RX_M];
#pragma unroll
        for (int i = 0; i < RX_M; ++i) h[i] = __shfl_down(any ? f[i] : 0u, d, 64);
        const int ha = __shfl_down(any ? 1 : 0, d, 64);
        if ((lane & (2 * d - 1)) == 0 && lane + d < 64 && ha) {
            if (any) rx_aff_compose(f, h);
            else {
#pragma unroll
                for (int i = 0; i < RX_M; ++i) f[i] = h[i];
                any = true;
            }
        }
    }
    if (lane == 0) out[0] = rx_aff_result(f, any);
}
#endif
)RX";

// Fixed-length strings: string i is bytes[i*length, (i+1)*length).  One
// wavefront runs 2048 strings: lane l owns bit j of every word for string
// base + 64 j + l.  32-byte tiles of every string are staged in LDS by
// asynchronous 16-byte global->LDS loads, then each lane reads 4 bytes of its
// 32 strings, transposes them into bit planes and runs four macro steps.
const char* kFixedKernelSource = R"RX(
// ---- device kernel ----
typedef __attribute__((address_space(1))) void rx_gvoid;
typedef __attribute__((address_space(3))) void rx_lvoid;
typedef __attribute__((address_space(3))) u32 rx_lds_u32;
typedef unsigned int rx_v4 __attribute__((ext_vector_type(4)));
#define RX_WAVE_STRINGS 2048
#define RX_TILE 32

// Runs the macro step over positions [0, np) of the staged 32-byte tile.
__device__ __forceinline__ void rx_run_tile(const u32* rx_tile, int lane, int np, u32 (&s)[RX_NS], u32& acc) {
    for (int pq = 0; pq < np; pq += 4) {
        u32 w[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) w[j] = rx_tile[(j * 64 + lane) * 8 + (pq >> 2)];
        rx_transpose32(w);
        rx_step(s, acc, w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7]);
        if (pq + 1 < np) rx_step(s, acc, w[8], w[9], w[10], w[11], w[12], w[13], w[14], w[15]);
        if (pq + 2 < np) rx_step(s, acc, w[16], w[17], w[18], w[19], w[20], w[21], w[22], w[23]);
        if (pq + 3 < np) rx_step(s, acc, w[24], w[25], w[26], w[27], w[28], w[29], w[30], w[31]);
    }
}

__device__ __forceinline__ void rx_store_result(unsigned char* __restrict__ out, long long base, long long n, int lane,
                                                 u32 acc) {
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const long long sid = base + j * 64 + lane;
        if (sid < n) out[sid] = (unsigned char)((acc >> j) & 1u);
    }
}

// 32-byte bursts: each tile is fetched straight into LDS.
extern "C" __global__ __launch_bounds__(64, 1) void rx_sliced_fixed(const unsigned char* __restrict__ bytes,
        long long length, long long n, unsigned char* __restrict__ out) {
    extern __shared__ u32 rx_tile[];   // RX_WAVE_STRINGS * RX_TILE bytes
    const int lane = threadIdx.x;
    const long long base = (long long)blockIdx.x * RX_WAVE_STRINGS;
    u32 s[RX_NS];
    u32 acc;
    rx_init(s, acc);
    const long long ntiles = (length + RX_TILE - 1) / RX_TILE;
    for (long long t = 0; t < ntiles; ++t) {
        const long long off = t * RX_TILE + 16 * (lane & 1);
        __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the previous tile has been read
        if (off < length) {
#pragma unroll 8
            for (int q = 0; q < RX_WAVE_STRINGS / 32; ++q) {
                long long sid = base + q * 32 + (lane >> 1);
                if (sid > n - 1) sid = n - 1;
                __builtin_amdgcn_global_load_lds((rx_gvoid*)(bytes + sid * length + off),
                                                 (rx_lvoid*)(rx_tile + q * 256), 16, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the tile has landed
        const long long left = length - t * RX_TILE;
        rx_run_tile(rx_tile, lane, left < RX_TILE ? (int)left : RX_TILE, s, acc);
    }
    rx_store_result(out, base, n, lane, acc);
}

// Prefetching: the next 32-byte tile of every string streams into
// accumulation registers (unused by this kernel otherwise) while the current
// tile is matched from LDS, so load latency hides behind the circuit.
// At a tile boundary the registers are written to LDS and the following
// tile's loads are issued before matching starts.
__device__ __forceinline__ void rx_issue_tile(const unsigned char* __restrict__ bytes, long long length, long long n,
                                              long long base, int lane, long long t, rx_v4 (&nx)[RX_WAVE_STRINGS / 32]) {
    long long off = t * RX_TILE + 16 * (lane & 1);
    if (off >= length) off = t * RX_TILE;   // past a string's end: an in-bounds duplicate, never matched
#pragma unroll
    for (int q = 0; q < RX_WAVE_STRINGS / 32; ++q) {
        long long sid = base + q * 32 + (lane >> 1);
        if (sid > n - 1) sid = n - 1;
        const unsigned char* p = bytes + sid * length + off;
        asm volatile("global_load_dwordx4 %0, %1, off" : "=a"(nx[q]) : "v"(p) : "memory");
    }
}

// Two waves per workgroup: every string's next 64 bytes are requested as one
// burst, its first 32 bytes by the matching wave (into accumulation
// registers) and its second 32 by a loader wave (into its registers), so a
// cache line is fetched in two halves at about the same time instead of four
// quarters a tile apart.  The halves are written to LDS in turn; the next
// burst is in flight while the matching wave works on the second half.
__device__ __forceinline__ void rx_issue_half(const unsigned char* __restrict__ bytes, long long length, long long n,
                                              long long base, int lane, long long off_half,
                                              rx_v4 (&nx)[RX_WAVE_STRINGS / 32]) {
    long long off = off_half + 16 * (lane & 1);
    if (off >= length) off = length - 16;   // past a string's end: an in-bounds duplicate, never matched
#pragma unroll
    for (int q = 0; q < RX_WAVE_STRINGS / 32; ++q) {
        long long sid = base + q * 32 + (lane >> 1);
        if (sid > n - 1) sid = n - 1;
        const unsigned char* p = bytes + sid * length + off;
        asm volatile("global_load_dwordx4 %0, %1, off" : "=a"(nx[q]) : "v"(p) : "memory");
    }
}

__device__ __forceinline__ void rx_regs_to_tile(u32* rx_tile, int lane, rx_v4 (&nx)[RX_WAVE_STRINGS / 32]) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
    for (int q = 0; q < RX_WAVE_STRINGS / 32; ++q) {
        const u32 a = (u32)(unsigned long long)(rx_lds_u32*)(rx_tile + q * 256 + 4 * lane);
        asm volatile("ds_write_b128 %0, %1" ::"v"(a), "a"(nx[q]) : "memory");
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

extern "C" __global__ __launch_bounds__(128, 1) void rx_sliced_fixed_duo(const unsigned char* __restrict__ bytes,
        long long length, long long n, unsigned char* __restrict__ out) {
    extern __shared__ u32 rx_tile[];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const long long base = (long long)blockIdx.x * RX_WAVE_STRINGS;
    u32 s[RX_NS];
    u32 acc;
    rx_init(s, acc);
    const long long nbursts = (length + 63) / 64;
    const long long nhalves = (length + 31) / 32;
    rx_v4 nx[RX_WAVE_STRINGS / 32];
    rx_issue_half(bytes, length, n, base, lane, wave * 32, nx);
    for (long long h = 0; h < nhalves; ++h) {
        const long long k = h >> 1;
        const int half = (int)(h & 1);
        if (wave == half) rx_regs_to_tile(rx_tile, lane, nx);   // this half of burst k
        __syncthreads();
        if (half == 1 && k + 1 < nbursts) rx_issue_half(bytes, length, n, base, lane, (k + 1) * 64 + wave * 32, nx);
        const long long left = length - h * 32;
        if (wave == 0) rx_run_tile(rx_tile, lane, left < 32 ? (int)left : 32, s, acc);
        __syncthreads();
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // a trailing half that was never matched has landed
    if (wave == 0) rx_store_result(out, base, n, lane, acc);
}

// Transposer and circuit on two SIMDs.  Data move as in the two-wave kernel
// (64-byte bursts split between the waves' registers, written to the LDS tile
// in halves), but the second wave also turns the tile into bit planes, four
// positions at a time, into a two-slot ring; the first wave runs the circuit
// one slot behind.  Slot layout: 8 quads of plane words per lane, quad-major,
// so both sides move 16 bytes per lane per access without bank conflicts.
#define RX_SLOT_WORDS (32 * 64)
__device__ __forceinline__ void rx_tile_to_planes(const u32* rx_tile, u32* slot, int lane, int grp) {
    u32 w[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) w[j] = rx_tile[(j * 64 + lane) * 8 + grp];
    rx_transpose32(w);
    rx_v4* d = reinterpret_cast<rx_v4*>(slot);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        rx_v4 v;
        v.x = w[4 * k];
        v.y = w[4 * k + 1];
        v.z = w[4 * k + 2];
        v.w = w[4 * k + 3];
        d[k * 64 + lane] = v;
    }
}

__device__ __forceinline__ void rx_run_planes(const u32* slot, int lane, u32 (&s)[RX_NS], u32& acc) {
    const rx_v4* q = reinterpret_cast<const rx_v4*>(slot);
    u32 w[32];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const rx_v4 v = q[k * 64 + lane];
        w[4 * k] = v.x;
        w[4 * k + 1] = v.y;
        w[4 * k + 2] = v.z;
        w[4 * k + 3] = v.w;
    }
    rx_step(s, acc, w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7]);
    rx_step(s, acc, w[8], w[9], w[10], w[11], w[12], w[13], w[14], w[15]);
    rx_step(s, acc, w[16], w[17], w[18], w[19], w[20], w[21], w[22], w[23]);
    rx_step(s, acc, w[24], w[25], w[26], w[27], w[28], w[29], w[30], w[31]);
}

// As rx_run_planes, also recording each string's earliest accept.  After the
// step that consumes byte k0 + t (t = 0..3) of the first set's strings (bits
// 0-15) and byte k1 + t of the second set's (bits 16-31), bits of vmask whose
// accept appears for the first time get first[string] = that count + 1.
__device__ __forceinline__ void rx_note_first(u32 nw, int t, long long k0, long long k1, long long base, long long n,
                                              int lane, long long* __restrict__ first) {
    while (nw) {
        const int j = __builtin_ctz(nw);
        nw &= nw - 1;
        const long long sid = base + j * 64 + lane;
        if (sid < n) first[sid] = (j < 16 ? k0 : k1) + t + 1;
    }
}
__device__ __forceinline__ void rx_run_planes_first(const u32* slot, int lane, u32 (&s)[RX_NS], u32& acc, u32& seen,
                                                    u32 vmask, long long k0, long long k1, long long base,
                                                    long long n, long long* __restrict__ first) {
    const rx_v4* q = reinterpret_cast<const rx_v4*>(slot);
    u32 w[32];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const rx_v4 v = q[k * 64 + lane];
        w[4 * k] = v.x;
        w[4 * k + 1] = v.y;
        w[4 * k + 2] = v.z;
        w[4 * k + 3] = v.w;
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        rx_step(s, acc, w[8 * t], w[8 * t + 1], w[8 * t + 2], w[8 * t + 3], w[8 * t + 4], w[8 * t + 5], w[8 * t + 6],
                w[8 * t + 7]);
        const u32 nw = acc & ~seen & vmask;
        if (nw) {
            seen |= nw;
            rx_note_first(nw, t, k0, k1, base, n, lane, first);
        }
    }
}

// length must be a multiple of 16 (whole 4-position groups, whole 16-byte loads).
extern "C" __global__ __launch_bounds__(128, 1) void rx_sliced_fixed_split(const unsigned char* __restrict__ bytes,
        long long length, long long n, unsigned char* __restrict__ out) {
    extern __shared__ u32 rx_tile[];                   // 32-byte tile of every string, then the ring
    u32* rx_ring = rx_tile + RX_WAVE_STRINGS * 8;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const long long base = (long long)blockIdx.x * RX_WAVE_STRINGS;
    u32 s[RX_NS];
    u32 acc;
    rx_init(s, acc);
    const long long nbursts = (length + 63) / 64;
    const long long ngroups = length / 4;
    rx_v4 nx[RX_WAVE_STRINGS / 32];
    rx_issue_half(bytes, length, n, base, lane, wave * 32, nx);
    // tick g: wave 1 transposes group g, wave 0 runs group g - 1
    for (long long g = 0; g <= ngroups; ++g) {
        if ((g & 7) == 0 && g < ngroups) {
            // group g opens half h of the string; the tile's previous half was
            // last read by wave 1 in the tick before
            const long long h = g >> 3;
            const long long k = h >> 1;
            const int half = (int)(h & 1);
            if (wave == half) rx_regs_to_tile(rx_tile, lane, nx);
            __syncthreads();
            if (half == 1 && k + 1 < nbursts) rx_issue_half(bytes, length, n, base, lane, (k + 1) * 64 + wave * 32, nx);
        }
        if (wave == 1) {
            if (g < ngroups) rx_tile_to_planes(rx_tile, rx_ring + (int)(g & 1) * RX_SLOT_WORDS, lane, (int)(g & 7));
        } else if (g > 0) {
            rx_run_planes(rx_ring + (int)((g - 1) & 1) * RX_SLOT_WORDS, lane, s, acc);
        }
        __syncthreads();
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // a trailing half that was never matched has landed
    if (wave == 0) rx_store_result(out, base, n, lane, acc);
}

// Skewed sets.  The 2048 strings of a workgroup form two sets: bits 0-15 of
// every word (strings 0-1023) and bits 16-31 (strings 1024-2047).  The circuit
// wave fetches the first set's 64-byte bursts, the transposing wave the
// second's, and the second set runs one 32-byte half behind the first.  A
// wave requests its set's next burst as soon as the previous one has moved to
// the tile, so the two sets' requests alternate from half to half and one is
// always in flight while the circuit runs.  The second set's bits take
// garbage during the first half and are reset to the start state before its
// first byte; the first set's accept bits are taken after its last byte.
#define RX_SET_STRINGS 1024
// Burst (off / 64) of every string of one set: instruction q takes 16 bytes
// (chunk lane / 32) of string q * 32 + lane % 32 into nx[q] (first 32 bytes of
// the burst) and into nx[q + 32] (second 32), back to back.  Addresses are a uniform base (scalar
// registers) plus a 32-bit per-lane offset, formed at the load, so no address
// stays live across the loop.  off < length and length % 16 == 0.
__device__ __forceinline__ void rx_gload(rx_v4& dst, const unsigned char* sp, u32 voff) {
    asm volatile("global_load_dwordx4 %0, %1, %2" : "=a"(dst) : "v"(voff), "s"(sp) : "memory");
}
// B = 0: strings q < 16 (32 loads), B = 1: strings q >= 16, B < 0: all 64.
template <int B>
__device__ __forceinline__ void rx_issue_set(const unsigned char* __restrict__ bytes, long long length, long long n,
                                             long long sbase, int lane, long long off, rx_v4 (&nx)[64]) {
    const long long room = length - 16 - off;   // >= 0; past a string's end: an in-bounds duplicate, never matched
    const int c = lane >> 5;
    const long long da = 16 * c < room ? 16 * c : room;
    const long long db = 32 + 16 * c < room ? 32 + 16 * c : room;
    if (sbase + RX_SET_STRINGS <= n) {
        const u32 va = (u32)((lane & 31) * length + da), vb = (u32)((lane & 31) * length + db);
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            if ((B == 0 && q >= 16) || (B == 1 && q < 16)) continue;
            const unsigned char* sp = bytes + (sbase + q * 32) * length + off;
            rx_gload(nx[q], sp, va);
            rx_gload(nx[q + 32], sp, vb);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            if ((B == 0 && q >= 16) || (B == 1 && q < 16)) continue;
            long long bq = sbase + q * 32;
            if (bq > n - 1) bq = n - 1;
            long long r = lane & 31;
            if (r > n - 1 - bq) r = n - 1 - bq;
            const unsigned char* sp = bytes + bq * length + off;
            rx_gload(nx[q], sp, (u32)(r * length + da));
            rx_gload(nx[q + 32], sp, (u32)(r * length + db));
        }
    }
}

// Moves one half of the set's burst (SECOND = its last 32 bytes) to the tile,
// which holds the current 32 bytes of every string as two 16-byte chunks,
// chunk-major: chunk c of string s (0 .. 2047) at 16-byte slot c * 2048 + s.
// Consecutive lanes write consecutive slots, and the transposing wave reads
// one dword of 64 consecutive slots at a time.
template <int SECOND>
__device__ __forceinline__ void rx_set_to_tile(u32* rx_tile, int set_off, int lane, rx_v4 (&nx)[64]) {
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const int slot = (lane >> 5) * RX_WAVE_STRINGS + set_off + q * 32 + (lane & 31);
        const u32 a = (u32)(unsigned long long)(rx_lds_u32*)(rx_tile + slot * 4);
        asm volatile("ds_write_b128 %0, %1" ::"v"(a), "a"(nx[q + 32 * SECOND]) : "memory");
    }
    // the writes have read their registers before any load refills them
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// Plane groups of the chunk-major tile.  At an even group g the transposing
// lane reads dwords g % 4 and g % 4 + 1 of chunk g / 4 of its 32 strings
// (string j * 64 + lane) as one 8-byte access each and makes group g from the
// first; group g + 1 comes from the second, already in registers.
typedef unsigned int rx_v2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void rx_read_pairs(const u32* rx_tile, int g, int lane, rx_v2 (&raw)[32]) {
    const rx_v2* t = reinterpret_cast<const rx_v2*>(rx_tile) + (g >> 2) * (RX_WAVE_STRINGS * 2) + ((g & 3) >> 1);
#pragma unroll
    for (int j = 0; j < 32; ++j) raw[j] = t[(j * 64 + lane) * 2];
}
// Plane group g read one dword per string (the variant for programs whose
// circuit leaves no room for the pair registers).
__device__ __forceinline__ void rx_words_to_planes(const u32* rx_tile, u32* slot, int lane, int g) {
    u32 w[32];
    const u32* t = rx_tile + (g >> 2) * (RX_WAVE_STRINGS * 4) + (g & 3);
#pragma unroll
    for (int j = 0; j < 32; ++j) w[j] = t[(j * 64 + lane) * 4];
    rx_transpose32(w);
    rx_v4* d = reinterpret_cast<rx_v4*>(slot);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        rx_v4 v;
        v.x = w[4 * k];
        v.y = w[4 * k + 1];
        v.z = w[4 * k + 2];
        v.w = w[4 * k + 3];
        d[k * 64 + lane] = v;
    }
}
template <int E>
__device__ __forceinline__ void rx_pairs_to_planes(const rx_v2 (&raw)[32], u32* slot, int lane) {
    u32 w[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) w[j] = E == 0 ? raw[j].x : raw[j].y;
    rx_transpose32(w);
    rx_v4* d = reinterpret_cast<rx_v4*>(slot);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        rx_v4 v;
        v.x = w[4 * k];
        v.y = w[4 * k + 1];
        v.z = w[4 * k + 2];
        v.w = w[4 * k + 3];
        d[k * 64 + lane] = v;
    }
}

// length must be a multiple of 16.  PAIRS: the transposing wave reads dword
// pairs (fewer LDS accesses, 64 more registers) rather than single dwords.
template <bool PAIRS, bool FIRST>
__device__ __forceinline__ void rx_skew(const unsigned char* __restrict__ bytes, long long length, long long n,
                                        unsigned char* __restrict__ out, long long* __restrict__ first,
                                        u32* rx_tile) {
    u32* rx_ring = rx_tile + RX_WAVE_STRINGS * 8;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const long long base = (long long)blockIdx.x * RX_WAVE_STRINGS;
    const long long sbase = base + (long long)wave * RX_SET_STRINGS;
    const long long nbursts = (length + 63) / 64;
    const long long nhalves = (length + 31) / 32;
    const long long ngroups = length / 4;
    const long long nticks = ngroups + 8;   // the second set's groups come 8 ticks late
    u32 s[RX_NS];
    u32 acc;
    rx_init(s, acc);
    u32 acc_first = 0;
    u32 seen = 0;   // FIRST: strings whose accept has appeared
    rx_v4 nx[64];
    // The first set's first burst is needed at once; the second set's half
    // goes out now and half two ticks in, so the first set's requests reach
    // memory ahead of it.
    if (wave == 0) rx_issue_set<-1>(bytes, length, n, sbase, lane, 0, nx);
    else rx_issue_set<0>(bytes, length, n, sbase, lane, 0, nx);
    // tick T: the transposing wave makes plane group T (first set: group T of
    // its string, second set: group T - 8), the circuit wave runs group T - 1
    rx_v2 raw[32];
    long long hh = 0;   // the half this wave's set is in
    for (long long T = 0; T <= nticks; ++T) {
        if ((T & 7) == 0 && T < nticks) {
            hh = (T >> 3) - wave;
            if (hh >= 0 && hh < nhalves) {
                if ((hh & 1) == 0) {
                    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                    rx_set_to_tile<0>(rx_tile, wave * RX_SET_STRINGS, lane, nx);
                } else {
                    // the burst landed with its first half
                    rx_set_to_tile<1>(rx_tile, wave * RX_SET_STRINGS, lane, nx);
                }
            }
            // The registers are free once the burst's second half is in the
            // tile.  The next burst goes out in two halves, here and two
            // ticks later: a wave may hold 63 loads in flight, and a wave
            // whose requests back up in a busy memory system stalls at issue
            // (holding the other wave at the next barrier), so shorter
            // batches keep both waves computing.
            if (hh >= 0 && hh < nhalves && (hh & 1) == 1 && (hh >> 1) + 1 < nbursts)
                rx_issue_set<0>(bytes, length, n, sbase, lane, ((hh >> 1) + 1) * 64, nx);
            __syncthreads();
        }
        // (hh = -1: the second set's first burst, whose first half went out
        // before the loop)
        if ((T & 7) == 2 && T < nticks && hh >= -1 && hh < nhalves && (hh & 1) == 1 && (hh >> 1) + 1 < nbursts)
            rx_issue_set<1>(bytes, length, n, sbase, lane, ((hh >> 1) + 1) * 64, nx);
        if (wave == 1) {
            if (T < nticks) {
                if (!PAIRS) {
                    rx_words_to_planes(rx_tile, rx_ring + (int)(T & 1) * RX_SLOT_WORDS, lane, (int)(T & 7));
                } else if ((T & 1) == 0) {
                    rx_read_pairs(rx_tile, (int)(T & 7), lane, raw);
                    rx_pairs_to_planes<0>(raw, rx_ring + (int)(T & 1) * RX_SLOT_WORDS, lane);
                } else {
                    rx_pairs_to_planes<1>(raw, rx_ring + (int)(T & 1) * RX_SLOT_WORDS, lane);
                }
            }
        } else if (T > 0) {
            const long long P = T - 1;
            if (P == 8) {
                // the second set's first byte: its bits restart from the start state
                u32 s0[RX_NS];
                u32 a0;
                rx_init(s0, a0);
#pragma unroll
                for (int i = 0; i < RX_NS; ++i) s[i] = (s[i] & 0x0000ffffu) | (s0[i] & 0xffff0000u);
                acc = (acc & 0x0000ffffu) | (a0 & 0xffff0000u);
            }
            if (FIRST) {
                // the first set is real for groups [0, ngroups), the second from group 8 on
                const u32 vmask = (P < ngroups ? 0x0000ffffu : 0u) | (P >= 8 ? 0xffff0000u : 0u);
                rx_run_planes_first(rx_ring + (int)(P & 1) * RX_SLOT_WORDS, lane, s, acc, seen, vmask, P * 4,
                                    (P - 8) * 4, base, n, first);
            } else {
                rx_run_planes(rx_ring + (int)(P & 1) * RX_SLOT_WORDS, lane, s, acc);
            }
            if (P == ngroups - 1) acc_first = acc;
        }
        __syncthreads();
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // loads past the last matched half have landed
    if (wave != 0) return;
    if (!FIRST) {
        rx_store_result(out, base, n, lane, (acc_first & 0x0000ffffu) | (acc & 0xffff0000u));
        return;
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) {   // strings whose accept never appeared
        const long long sid = base + j * 64 + lane;
        if (sid < n && !((seen >> j) & 1u)) first[sid] = -1;
    }
}

extern "C" __global__ __launch_bounds__(128, 1) void rx_sliced_fixed_skew(const unsigned char* __restrict__ bytes,
        long long length, long long n, unsigned char* __restrict__ out) {
    extern __shared__ u32 rx_tile[];   // 32-byte tile of every string, then the ring
    rx_skew<true, false>(bytes, length, n, out, nullptr, rx_tile);
}

extern "C" __global__ __launch_bounds__(128, 1) void rx_sliced_fixed_skew_w(const unsigned char* __restrict__ bytes,
        long long length, long long n, unsigned char* __restrict__ out) {
    extern __shared__ u32 rx_tile[];
    rx_skew<false, false>(bytes, length, n, out, nullptr, rx_tile);
}

// rx_match's equal-length strings: the layout slot of call `id` (see the
// layout check: {id, length, first offset, flaw}) holds the length and the
// first string's offset; the kernel does nothing unless the slot is this
// call's and has no flaw (the table form then matches the strings).
extern "C" __global__ __launch_bounds__(128, 1) void rx_sliced_offsets_skew(const unsigned char* __restrict__ bytes,
        const long long* __restrict__ slot, long long id, long long n, unsigned char* __restrict__ out) {
    extern __shared__ u32 rx_tile[];
    if (slot[0] != id || slot[3] != 0) return;
    rx_skew<true, false>(bytes + slot[2], slot[1], n, out, nullptr, rx_tile);
}

extern "C" __global__ __launch_bounds__(128, 1) void rx_sliced_offsets_skew_w(const unsigned char* __restrict__ bytes,
        const long long* __restrict__ slot, long long id, long long n, unsigned char* __restrict__ out) {
    extern __shared__ u32 rx_tile[];
    if (slot[0] != id || slot[3] != 0) return;
    rx_skew<false, false>(bytes + slot[2], slot[1], n, out, nullptr, rx_tile);
}

// Earliest accepting prefix of every string (the root is not nullable:
// the caller answers 0 for every string otherwise).
extern "C" __global__ __launch_bounds__(128, 1) void rx_sliced_first_skew(const unsigned char* __restrict__ bytes,
        long long length, long long n, long long* __restrict__ first) {
    extern __shared__ u32 rx_tile[];
    rx_skew<true, true>(bytes, length, n, nullptr, first, rx_tile);
}

extern "C" __global__ __launch_bounds__(128, 1) void rx_sliced_first_skew_w(const unsigned char* __restrict__ bytes,
        long long length, long long n, long long* __restrict__ first) {
    extern __shared__ u32 rx_tile[];
    rx_skew<false, true>(bytes, length, n, nullptr, first, rx_tile);
}

extern "C" __global__ __launch_bounds__(64, 1) void rx_sliced_fixed_pf(const unsigned char* __restrict__ bytes,
        long long length, long long n, unsigned char* __restrict__ out) {
    extern __shared__ u32 rx_tile[];
    const int lane = threadIdx.x;
    const long long base = (long long)blockIdx.x * RX_WAVE_STRINGS;
    u32 s[RX_NS];
    u32 acc;
    rx_init(s, acc);
    const long long ntiles = (length + RX_TILE - 1) / RX_TILE;
    rx_v4 nx[RX_WAVE_STRINGS / 32];
    rx_issue_tile(bytes, length, n, base, lane, 0, nx);
    for (long long t = 0; t < ntiles; ++t) {
        // tile t has landed in registers; the previous tile's LDS reads are done
        asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
#pragma unroll
        for (int q = 0; q < RX_WAVE_STRINGS / 32; ++q) {
            const u32 a = (u32)(unsigned long long)(rx_lds_u32*)(rx_tile + q * 256 + 4 * lane);
            asm volatile("ds_write_b128 %0, %1" ::"v"(a), "a"(nx[q]) : "memory");
        }
        // the writes have read their registers before the next loads refill them
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        if (t + 1 < ntiles) rx_issue_tile(bytes, length, n, base, lane, t + 1, nx);
        const long long left = length - t * RX_TILE;
        rx_run_tile(rx_tile, lane, left < RX_TILE ? (int)left : RX_TILE, s, acc);
    }
    rx_store_result(out, base, n, lane, acc);
}
)RX";

// Plane form: circuits driven by bit planes that a separate kernel has
// already gathered and transposed (rx_multi.hip), for strings of any length.
// A slab is 2048 strings (lane l holds strings 64 j + l in bit j); tick t of a
// slab is positions 4t .. 4t+3 as 36 words per lane: w[8i + b] = bit plane b
// of position 4t + i, w[32 + i] = the strings whose length exceeds 4t + i.
// In memory a tick is nine groups of four words, group q of lane l at
// u32 index ((t * 9 + q) * 64 + l) * 4.  After each step a string's accept
// bit is taken only while the string still has bytes, so it holds the value
// after the string's last byte (the start value for the empty string).
//
// One module holds the circuits of every program of a call (one struct per
// program), so one launch runs every (program, slab) pair of a range of
// slabs: the longest slabs of all programs start first, and the programs of
// one slab run side by side on one XCD (workgroups go to the XCDs in turn,
// blockIdx mod 8), where they share that slab's planes in the XCD's L2.
const char* kPlanesTickSource = R"RX(
template <class PR>
__device__ __forceinline__ void rx_planes_tick(u32 (&s)[PR::NS], u32& acc, u32& accf, const u32 (&w)[36]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        PR::step(s, acc, w[8 * i], w[8 * i + 1], w[8 * i + 2], w[8 * i + 3], w[8 * i + 4], w[8 * i + 5],
                 w[8 * i + 6], w[8 * i + 7]);
        const u32 v = w[32 + i];
        accf = (acc & v) | (accf & ~v);
    }
}
)RX";

const char* kPlanesKernelSource = R"RX(
// ---- device kernel ----
typedef unsigned int rx_pv4 __attribute__((ext_vector_type(4)));
// Ticks [t0, t1) of a slab (p: the slab's planes at tick 0, this lane's
// column) through program PR's circuit.  Each tick is rx_planes_tick's (four
// steps, the accept bit kept where a string still has bytes), with its loads
// spread through it: the registers of a position's planes are refilled with
// the next tick's as soon as that position is done, so every load has a whole
// tick to arrive and no second set of registers is needed.  The first tick's
// values get a use of their own before the loop: the compiler then keeps the
// loop's loads where they are instead of merging each with the first tick's
// into one load at the top of the loop, next to its first use.
template <class PR>
__device__ __forceinline__ void rx_ticks(const rx_pv4* p, long long t0, long long t1, u32 (&st)[PR::NS], u32& acc,
                                         u32& accf) {
    if (t0 >= t1) return;
    rx_pv4 cur[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) cur[q] = p[t0 * (9 * 64) + q * 64];
#pragma unroll
    for (int q = 0; q < 9; ++q) asm volatile("" ::"v"(cur[q]));
    for (long long t = t0; t < t1; ++t) {
        const rx_pv4* pn = p + (t + 1 < t1 ? t + 1 : t) * (9 * 64);
        const u32 v[4] = {cur[8].x, cur[8].y, cur[8].z, cur[8].w};
        cur[8] = pn[8 * 64];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            PR::step(st, acc, cur[2 * i].x, cur[2 * i].y, cur[2 * i].z, cur[2 * i].w, cur[2 * i + 1].x,
                     cur[2 * i + 1].y, cur[2 * i + 1].z, cur[2 * i + 1].w);
            accf = (acc & v[i]) | (accf & ~v[i]);
            cur[2 * i] = pn[(2 * i) * 64];
            cur[2 * i + 1] = pn[(2 * i + 1) * 64];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Slab s (ticks slab_tick[s] .. slab_tick[s+1] of `planes`) for program PR;
// lane l writes its 32 results (bit j: the slab's entry 64 j + l) to
// res[l * RX_NPROGS] (the programs' words of one lane side by side).
template <class PR>
__device__ __forceinline__ void rx_run_slab(const u32* __restrict__ planes, const long long* __restrict__ slab_tick,
                                            long long s, u32* __restrict__ res) {
    const int lane = threadIdx.x & 63;
    const long long t0 = slab_tick[s], T = slab_tick[s + 1] - t0;
    const rx_pv4* p = reinterpret_cast<const rx_pv4*>(planes) + t0 * (9 * 64) + lane;
    u32 st[PR::NS];
    u32 acc;
    PR::init(st, acc);
    u32 accf = acc;
    rx_ticks<PR>(p, 0, T, st, acc, accf);
    res[lane * RX_NPROGS] = accf;
}

// A long slab of a searched program on up to PR::NW wavefronts (8, 4 or 2,
// as many as leave room in LDS for the kept states; the launch has
// RX_SPEC_WAVES).  The slab's T ticks are cut into ws segments of at least 64
// ticks; wavefront i
// starts at tick i * T / ws, the first from the start as usual, the others
// from the start state, and each of those leaves copies of its state in LDS
// after 4, 8, 16, 32 of its ticks.  Wavefront i runs on past its segment and,
// at each of the next one's copies, compares its state with the copy: once
// they are equal for every string they stay equal (the step depends on the
// state and the byte alone, Def. 5.1), so it stops there, and from that tick
// on the next wavefront holds the true state.  Strings that have ended by
// then, and strings already in the any-byte loop of the search suffix (they
// accept whatever follows), are left out of the comparison.  A searched
// program's start state lies in every state it reaches (the any-byte loop of
// its prefix leads back to it after every byte), so two neighbours meet as
// soon as the matches begun before the later one's start have died or joined
// those begun after it -- usually at the first copy.  Each string then takes
// the accept bit of the wavefront that holds the true state at its last
// byte.  A wavefront waits for a copy a bounded time; past that it runs on to
// the end, with the same bits.  One call of the tick loop serves every
// wavefront and every segment.
template <class PR>
__device__ __forceinline__ void rx_run_slab_spec(const u32* __restrict__ planes,
                                                 const long long* __restrict__ slab_tick, long long s,
                                                 u32* __restrict__ res, u32* lds) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const long long t0 = slab_tick[s], T = slab_tick[s + 1] - t0;
    const rx_pv4* p = reinterpret_cast<const rx_pv4*>(planes) + t0 * (9 * 64) + lane;
    constexpr int NS = PR::NS, NCP = PR::NCP, NW = RX_SPEC_WAVES;
    volatile u32* flags = lds;          // flags[8 i + c]: wavefront i's copy c is in place
    volatile u32* met = lds + 8 * NW;   // met[i]: wavefront i met wavefront i + 1
    u32* accx = lds + 9 * NW;           // per wavefront and lane: accept bits,
    u32* vnx = accx + 64 * NW;          // the strings with bytes at the meeting tick,
    u32* surex = vnx + 64 * NW;         // the strings in the suffix loop there
    u32* ck = surex + 64 * NW;          // wavefront i >= 1, copy c, word k, lane l at (((i-1) NCP + c) NS + k) 64 + l
    int ws = PR::SPEC && NCP > 0 ? PR::NW : 1;
    while (ws > 1 && T < 64 * ws) ws >>= 1;
    if (threadIdx.x < 9 * NW) lds[threadIdx.x] = 0u;
    __syncthreads();
    if (wave < ws) {
        const long long seg = T / ws, start = wave * seg, next = wave + 1 < ws ? start + seg : T;
        u32 st[NS];
        u32 acc;
        PR::init(st, acc);
        u32 accf = wave == 0 ? acc : 0u;
        u32 vnext = 0u, sure = 0u;
        bool same = false;
        long long t = start;
        // phase 0: own copies (not the first wavefront); 1: to the segment's
        // end; 2: the next wavefront's copies (not the last), then the end
        int phase = wave == 0 ? 1 : 0, c = 0;
#pragma clang loop unroll(disable)
        for (;;) {
            long long te;
            if (phase == 0) te = start + (4ll << c);
            else if (phase == 1) te = next;
            else te = c < NCP ? next + (4ll << c) : T;
            if (te > T) te = T;
            rx_ticks<PR>(p, t, te, st, acc, accf);
            t = te;
            if (phase == 0) {
#pragma unroll
                for (int k = 0; k < NS; ++k) ck[(((wave - 1) * NCP + c) * NS + k) * 64 + lane] = st[k];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                if (lane == 0) flags[8 * wave + c] = 1u;
                if (++c == NCP) {
                    phase = 1;
                    c = 0;
                }
            } else if (phase == 1) {
                if (wave + 1 == ws) break;
                phase = 2;
            } else {
                if (c == NCP || t >= T) break;
                int spin = 0;
                while (flags[8 * (wave + 1) + c] == 0u && spin < (1 << 22)) {
                    __builtin_amdgcn_s_sleep(2);
                    ++spin;
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                if (flags[8 * (wave + 1) + c] != 0u) {
                    vnext = p[t * (9 * 64) + 8 * 64].x;
                    sure = PR::SUF >= 0 ? st[PR::SUF >= 0 ? PR::SUF : 0] : 0u;
                    u32 diff = 0u;
#pragma unroll
                    for (int k = 0; k < NS; ++k) diff |= st[k] ^ ck[((wave * NCP + c) * NS + k) * 64 + lane];
                    same = __builtin_amdgcn_ballot_w64((diff & vnext & ~sure) != 0u) == 0ull;
                }
                if (same) break;
                ++c;
            }
        }
        accx[wave * 64 + lane] = accf;
        vnx[wave * 64 + lane] = vnext;
        surex[wave * 64 + lane] = sure;
        if (lane == 0) met[wave] = same ? 1u : 0u;
    }
    __syncthreads();
    if (wave == 0) {
        // wavefront i holds the true state from where wavefront i - 1 met it
        // to where it meets wavefront i + 1 (or the end)
        u32 r = 0u, live = 0xffffffffu;
        for (int i = 0; i < ws; ++i) {
            const u32 a = accx[i * 64 + lane];
            if (i + 1 == ws || met[i] == 0u) {
                r |= a & live;
                break;
            }
            const u32 vn = vnx[i * 64 + lane], su = surex[i * 64 + lane];
            r |= (a & live & ~vn) | (su & vn & live);
            live &= vn & ~su;
        }
        res[lane * RX_NPROGS] = r;
    }
}

// One wavefront per (program, slab) for the slabs of rank r_lo <= r < r_hi
// (rank 0 = the longest slab).  Workgroup b runs on XCD b mod 8; its slab
// rank is r_lo + 8 * ((b / 8) / n_progs) + b mod 8 and its program (b / 8)
// mod n_progs.  info[0] = strings in slabs; the results of program p and
// slab s, lane l go to res[(s * 64 + l) * RX_NPROGS + p].
extern "C" __global__ __launch_bounds__(64) void rx_planes_multi(const u32* __restrict__ planes,
        const long long* __restrict__ slab_tick, const long long* __restrict__ info, u32* __restrict__ res,
        long long max_slabs, long long r_lo, long long r_hi) {
    const long long b = blockIdx.x;
    const long long k = b >> 3;
    const int p = (int)(k % RX_NPROGS);
    const long long r = r_lo + (k / RX_NPROGS) * 8 + (b & 7);
    const long long n_sliced = info[0];
    const long long S = (n_sliced + 2047) / 2048;
    if (r >= S || r >= r_hi) return;
    // the longest slabs set the kernel's length: their wavefronts issue first on their SIMDs
    if (r < 16) __builtin_amdgcn_s_setprio(3);
    rx_dispatch(p, planes, slab_tick, S - 1 - r, res + (S - 1 - r) * 64 * RX_NPROGS + p);
}

// The same slabs with RX_SPEC_WAVES wavefronts per (program, slab): a
// searched program's slab of 128 ticks or more is cut into segments run side
// by side (rx_run_slab_spec); otherwise the first wavefront runs it whole.  Dynamic LDS: RX_SPEC_LDS
// bytes (flags, B's accept bits, the checkpoints).
extern "C" __global__ __launch_bounds__(64 * RX_SPEC_WAVES) void rx_planes_spec(const u32* __restrict__ planes,
        const long long* __restrict__ slab_tick, const long long* __restrict__ info, u32* __restrict__ res,
        long long max_slabs, long long r_lo, long long r_hi) {
    extern __shared__ u32 rx_spec_lds[];
    const long long b = blockIdx.x;
    const long long k = b >> 3;
    const int p = (int)(k % RX_NPROGS);
    const long long r = r_lo + (k / RX_NPROGS) * 8 + (b & 7);
    const long long n_sliced = info[0];
    const long long S = (n_sliced + 2047) / 2048;
    if (r >= S || r >= r_hi) return;
    __builtin_amdgcn_s_setprio(3);
    rx_dispatch_spec(p, planes, slab_tick, S - 1 - r, res + (S - 1 - r) * 64 * RX_NPROGS + p, rx_spec_lds);
}
)RX";

// The plane-form source for a list of programs: program k's circuit as
// struct RxProgk (its step and start state in namespace rxqk), the tick
// template, a dispatch over the programs and the kernel.
std::string jit_multi_planes_source(const Program* const* progs, int n, int* max_state, int* spec_lds) {
    std::ostringstream s;
    s << "typedef unsigned int u32;\n#define RX_NPROGS " << n << "\n#define RX_SPEC_WAVES " << kSpecWaves << "\n";
    int mx = 0;
    int64_t ck_words = 0;   // the largest checkpoint area of a split slab
    for (int k = 0; k < n; ++k) {
        int ns = 0, suf = -1;
        std::string step = jit_step_source(*progs[k], &ns, nullptr, &suf);
        if (ns < 1) ns = 1;
        mx = std::max(mx, ns);
        // a searched program's long slabs may be split in two; as many
        // checkpoints (after 4, 8, 16, ... ticks) as the LDS budget holds
        const bool spec = search_prefix_leaf(*progs[k]) >= 0;
        // as many wavefronts per long slab (8, 4, 2) as leave room in LDS for
        // two kept states of each but the first, and as many kept states
        // (up to kSpecCheckpoints) as then fit
        auto fits = [&](int w) { return kSpecLdsBudget / (4 * 64 * (int64_t)ns * (w - 1)); };
        int nw = kSpecWaves;
        while (nw > 2 && fits(nw) < 2) nw >>= 1;
        const int ncp = spec ? (int)std::min<int64_t>(kSpecCheckpoints, fits(nw)) : 0;
        ck_words = std::max<int64_t>(ck_words, (int64_t)ncp * ns * 64 * (nw - 1));
        // the step source opens with its own #define of RX_NS
        const size_t eol = step.find('\n');
        s << "#define RX_NS " << ns << "\nnamespace rxq" << k << " {\n" << step.substr(eol + 1) << "}\n#undef RX_NS\n";
        s << "struct RxProg" << k << " {\n    static constexpr int NS = " << ns << ";\n"
          << "    static constexpr bool SPEC = " << (spec ? "true" : "false") << ";\n"
          << "    static constexpr int NCP = " << ncp << ";\n"
          << "    static constexpr int NW = " << nw << ";\n"
          << "    static constexpr int SUF = " << suf << ";\n"
          << "    __device__ static __forceinline__ void init(u32 (&s)[NS], u32& acc) { rxq" << k << "::rx_init(s, acc); }\n"
          << "    __device__ static __forceinline__ void step(u32 (&s)[NS], u32& acc, u32 b0, u32 b1, u32 b2, u32 b3, "
             "u32 b4, u32 b5, u32 b6, u32 b7) {\n        rxq" << k << "::rx_step(s, acc, b0, b1, b2, b3, b4, b5, b6, b7);\n    }\n};\n";
    }
    s << kPlanesTickSource;
    // the kernel part starts with the device-only marker; the dispatch sits just after it
    std::string kern = kPlanesKernelSource;
    const std::string marker = "// ---- device kernel ----\n";
    const size_t at = kern.find(marker) + marker.size();
    std::ostringstream disp;
    disp << kern.substr(0, kern.find("extern \"C\""));
    disp << "__device__ __forceinline__ void rx_dispatch(int p, const u32* __restrict__ planes, const long long* "
            "__restrict__ slab_tick, long long s, u32* __restrict__ res) {\n    switch (p) {\n";
    for (int k = 0; k < n; ++k)
        disp << "    case " << k << ": rx_run_slab<RxProg" << k << ">(planes, slab_tick, s, res); break;\n";
    disp << "    default: break;\n    }\n}\n";
    disp << "__device__ __forceinline__ void rx_dispatch_spec(int p, const u32* __restrict__ planes, const long long* "
            "__restrict__ slab_tick, long long s, u32* __restrict__ res, u32* lds) {\n    switch (p) {\n";
    for (int k = 0; k < n; ++k)
        disp << "    case " << k << ": rx_run_slab_spec<RxProg" << k << ">(planes, slab_tick, s, res, lds); break;\n";
    disp << "    default: break;\n    }\n}\n";
    disp << kern.substr(kern.find("extern \"C\""));
    (void)at;
    s << disp.str();
    if (max_state) *max_state = mx;
    // flags and meeting marks (9 words per wavefront), three words per lane and wavefront, the copies
    if (spec_lds) *spec_lds = (int)(4 * (9 * kSpecWaves + 3 * 64 * kSpecWaves + ck_words));
    return s.str();
}

// Loaded plane-form modules by (device, source): one per distinct program
// list, kept until the process ends (a module may be running on a stream).
struct PlaneModule {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    hipFunction_t fn_spec = nullptr;   // two wavefronts per (program, slab), long slabs split in two
    int spec_lds = 0;                  // its dynamic LDS bytes
    int scratch = 0;
};
namespace {
std::mutex g_plane_mu;
std::unordered_map<std::string, PlaneModule*> g_plane_mods;
}  // namespace

struct JitKernel {
    hipModule_t mod = nullptr;
    hipFunction_t fixed = nullptr;
    hipFunction_t fixed64 = nullptr;
    hipFunction_t duo = nullptr;
    hipFunction_t split = nullptr;
    hipFunction_t skew = nullptr;
    bool skew_words = false;   // skew is the single-dword-read form
    hipFunction_t skew_offsets = nullptr;   // the same form for rx_match's equal-length strings
    hipFunction_t first = nullptr;   // the skewed kernel's earliest-accept form
    bool first_words = false;
    hipFunction_t chunks = nullptr;   // chunk-parallel form (circuits of at most two words)
    hipFunction_t long_chunks = nullptr, long_compose = nullptr;   // one long string (at most 31 words)
    int dev = -1;
    int n_state = 0, n_ops = 0;
    std::string arch;
    // static check of the register-staged kernels (rx_isa_guard.cpp), per
    // kernel of kStagedKernels: -1 not checked, else the number of
    // compiler-made instructions that touch an accumulation register
    int guard_ran = 0;
    int guard_violations[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    int guard_dropped = 0;   // bit k: kernel k was dropped by the check
    // run-time check (jit_selfcheck): 1 when it ran on the device; bit k of
    // selfcheck_dropped: staged kernel k gave other bits than the table step
    int selfcheck_ran = 0;
    int selfcheck_dropped = 0;
};

// The kernels that keep in-flight loads in accumulation registers.
const char* const kStagedKernels[] = {"rx_sliced_fixed_pf", "rx_sliced_fixed_duo", "rx_sliced_fixed_split",
                                      "rx_sliced_fixed_skew", "rx_sliced_fixed_skew_w", "rx_sliced_first_skew",
                                      "rx_sliced_first_skew_w"};
constexpr int kNumStaged = (int)(sizeof(kStagedKernels) / sizeof(kStagedKernels[0]));

std::string jit_full_source(const Program& P, int* n_state, int* n_ops) {
    std::ostringstream s;
    s << "typedef unsigned int u32;\n";
    s << jit_step_source(P, n_state, n_ops);
    s << kTransposeSource;
    s << kChunkSource;
    s << kFixedKernelSource;
    s << kChunkKernelSource;
    return s.str();
}

// Code objects by (architecture, source): a program whose circuit text was
// compiled before in this process skips the device compiler.  Bounded; when
// full it is emptied and refilled.
namespace {
std::mutex g_code_mu;
std::unordered_map<std::string, std::vector<char>> g_code_cache;
constexpr size_t kCodeCacheEntries = 64;
}  // namespace

// The device's architecture name (arch_in when given: compile only, dev = -1).
int jit_target(const char* arch_in, std::string* arch, int* dev) {
    *dev = -1;
    if (arch_in && *arch_in) {
        *arch = arch_in;
        return RX_OK;
    }
    if (hipGetDevice(dev) != hipSuccess) return fail(RX_EHIP, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return fail(RX_EHIP, "hipGetDeviceProperties failed");
    *arch = prop.gcnArchName;
    return RX_OK;
}

// Compiles `src` for `arch` with hiprtc (or takes the cached code object).
int jit_code(const std::string& src, const std::string& arch, std::vector<char>* out) {
    const std::string key = arch + '\n' + src;
    std::vector<char> code;
    {
        std::lock_guard<std::mutex> lk(g_code_mu);
        auto it = g_code_cache.find(key);
        if (it != g_code_cache.end()) code = it->second;
    }
    if (code.empty()) {
        hiprtcProgram prog;
        if (hiprtcCreateProgram(&prog, src.c_str(), "rx_sliced.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
            return fail(RX_EJIT, "hiprtcCreateProgram failed");
        const std::string arch_opt = "--gpu-architecture=" + arch;
        const char* opts[] = {arch_opt.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
        const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
        if (rc != HIPRTC_SUCCESS) {
            size_t n = 0;
            hiprtcGetProgramLogSize(prog, &n);
            std::string log(n, '\0');
            if (n) hiprtcGetProgramLog(prog, &log[0]);
            hiprtcDestroyProgram(&prog);
            return fail(RX_EJIT, "hiprtc compile failed: " + log.substr(0, 2000));
        }
        size_t code_size = 0;
        hiprtcGetCodeSize(prog, &code_size);
        code.resize(code_size);
        hiprtcGetCode(prog, code.data());
        hiprtcDestroyProgram(&prog);
        std::lock_guard<std::mutex> lk(g_code_mu);
        if (g_code_cache.size() >= kCodeCacheEntries) g_code_cache.clear();
        g_code_cache.emplace(key, code);
    }
    *out = std::move(code);
    return RX_OK;
}

std::string jit_planes_source(const Program& P, int* n_state) {
    const Program* one[1] = {&P};
    return jit_multi_planes_source(one, 1, n_state, nullptr);
}

namespace {
// modules are looked up by device and the programs' identities, so a launch
// does not regenerate the source
std::string plane_key(int dev, const Program* const* progs, int n) {
    std::string k = std::to_string(dev);
    for (int i = 0; i < n; ++i) k += ':' + std::to_string(progs[i]->uid);
    return k;
}
}  // namespace

int jit_prepare_planes(const Program* const* progs, int n, const char* arch_in, int* spill_bytes) {
    int mx = 0, spec_lds = 0;
    const std::string src = jit_multi_planes_source(progs, n, &mx, &spec_lds);
    if (mx > kJitPlanesMaxState)
        return fail(RX_ETOOBIG, "the plane-form circuit keeps at most " + std::to_string(kJitPlanesMaxState) +
                                    " state words; a program needs " + std::to_string(mx));
    std::string arch;
    int dev = -1;
    if (int rc = jit_target(arch_in, &arch, &dev)) return rc;
    if (dev >= 0) {
        std::lock_guard<std::mutex> lk(g_plane_mu);
        auto it = g_plane_mods.find(plane_key(dev, progs, n));
        if (it != g_plane_mods.end()) {
            if (spill_bytes) *spill_bytes = it->second->scratch;
            return RX_OK;
        }
    }
    std::vector<char> code;
    if (int rc = jit_code(src, arch, &code)) return rc;
    if (dev < 0) return RX_OK;
    PlaneModule* K = new PlaneModule;
    hipError_t e = hipModuleLoadData(&K->mod, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&K->fn, K->mod, "rx_planes_multi");
    if (e == hipSuccess) e = hipModuleGetFunction(&K->fn_spec, K->mod, "rx_planes_spec");
    K->spec_lds = spec_lds;
    if (e == hipSuccess) e = hipFuncGetAttribute(&K->scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, K->fn);
    if (e != hipSuccess) {
        if (K->mod) hipModuleUnload(K->mod);
        delete K;
        return fail(RX_EHIP, std::string("plane-form module: ") + hipGetErrorString(e));
    }
    if (spill_bytes) *spill_bytes = K->scratch;
    std::lock_guard<std::mutex> lk(g_plane_mu);
    auto ins = g_plane_mods.emplace(plane_key(dev, progs, n), K);
    if (!ins.second) {   // another thread loaded the same list meanwhile
        hipModuleUnload(K->mod);
        delete K;
    }
    return RX_OK;
}

bool jit_planes_prepared(const Program* const* progs, int n) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lk(g_plane_mu);
    return g_plane_mods.count(plane_key(dev, progs, n)) > 0;
}

int launch_planes_circuits(const Program* const* progs, int n, const uint32_t* planes, const int64_t* slab_tick,
                           const int64_t* info, uint32_t* res, int64_t max_slabs, int64_t r_lo, int64_t r_hi,
                           bool split, void* stream) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return (int)hipErrorInvalidDevice;
    PlaneModule* K = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_plane_mu);
        auto it = g_plane_mods.find(plane_key(dev, progs, n));
        if (it != g_plane_mods.end()) K = it->second;
    }
    if (!K) return -1;   // not prepared
    const int64_t hi = r_hi < max_slabs ? r_hi : max_slabs;
    if (hi <= r_lo) return 0;
    const long long per = (hi - r_lo + 7) / 8;
    const unsigned grid = (unsigned)(8 * per * n);
    const void* a0 = planes;
    const void* a1 = slab_tick;
    const void* a2 = info;
    void* a3 = res;
    long long a4 = max_slabs, a5 = r_lo, a6 = hi;
    void* args[] = {&a0, &a1, &a2, &a3, &a4, &a5, &a6};
    if (split)
        return (int)hipModuleLaunchKernel(K->fn_spec, grid, 1, 1, 64 * kSpecWaves, 1, 1, (unsigned)K->spec_lds,
                                          (hipStream_t)stream,
                                          args, nullptr);
    return (int)hipModuleLaunchKernel(K->fn, grid, 1, 1, 64, 1, 1, 0, (hipStream_t)stream, args, nullptr);
}

namespace {
// A seeded batch for the run-time check of the staged kernels: strings that
// walk the automaton (each byte, with probability 7/8, one that a live leaf's
// label holds, so accepts are reached and left), and the table step of
// Def. 5.1 on the host over them: S = First, then S' = union of Follow[x]
// over the leaves x in S whose label holds the byte; the accept bit is rank L.
struct SelfCheckBatch {
    int64_t n = 0, length = 0;
    std::vector<uint8_t> bytes;
    std::vector<uint8_t> accept;    // accept bit after the last byte
    std::vector<int64_t> first;     // fewest bytes after which the accept bit is set, or -1
};

SelfCheckBatch selfcheck_batch(const Program& P, int64_t n, int64_t length) {
    SelfCheckBatch B;
    B.n = n;
    B.length = length;
    B.bytes.resize((size_t)(n * length));
    B.accept.resize((size_t)n);
    B.first.resize((size_t)n);
    const int W = P.W, L = P.L;
    std::vector<std::vector<uint8_t>> label_bytes((size_t)L);
    for (int b = 0; b < 256; ++b)
        for (int r = 0; r < L; ++r)
            if ((P.bytemask[(size_t)b * W + (r >> 5)] >> (r & 31)) & 1u) label_bytes[(size_t)r].push_back((uint8_t)b);
    uint64_t z = 0x243f6a8885a308d3ull;   // splitmix64 (Steele, Lea, Flood 2014)
    auto next = [&z]() {
        uint64_t x = (z += 0x9e3779b97f4a7c15ull);
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        return x ^ (x >> 31);
    };
    std::vector<uint32_t> S((size_t)W), T((size_t)W);
    std::vector<int> live;
    const bool acc0 = (P.first[(size_t)(L >> 5)] >> (L & 31)) & 1u;
    for (int64_t i = 0; i < n; ++i) {
        for (int w = 0; w < W; ++w) S[(size_t)w] = P.first[(size_t)w];
        int64_t firstpos = acc0 ? 0 : -1;
        for (int64_t k = 0; k < length; ++k) {
            live.clear();
            for (int w = 0; w < W; ++w)
                for (uint32_t x = S[(size_t)w]; x; x &= x - 1) {
                    const int r = w * 32 + __builtin_ctz(x);
                    if (r < L && !label_bytes[(size_t)r].empty()) live.push_back(r);
                }
            uint8_t c;
            const uint64_t u = next();
            if (live.empty() || (u & 7) == 0) {
                c = (uint8_t)(u >> 8);
            } else {
                const auto& lb = label_bytes[(size_t)live[(size_t)((u >> 8) % live.size())]];
                c = lb[(size_t)((u >> 32) % lb.size())];
            }
            B.bytes[(size_t)(i * length + k)] = c;
            std::fill(T.begin(), T.end(), 0u);
            for (int w = 0; w < W; ++w) {
                uint32_t x = S[(size_t)w] & P.bytemask[(size_t)c * W + w];
                while (x) {
                    const int r = w * 32 + __builtin_ctz(x);
                    x &= x - 1;
                    if (r >= L) continue;
                    for (int v = 0; v < W; ++v) T[(size_t)v] |= P.follow[(size_t)r * W + v];
                }
            }
            S.swap(T);
            if (firstpos < 0 && ((S[(size_t)(L >> 5)] >> (L & 31)) & 1u)) firstpos = k + 1;
        }
        B.accept[(size_t)i] = (uint8_t)((S[(size_t)(L >> 5)] >> (L & 31)) & 1u);
        B.first[(size_t)i] = firstpos;
    }
    return B;
}

// Runs every kept register-staged kernel of K (and the LDS-staged one) on the
// batch; a staged kernel whose bits differ from the table step is dropped.
// Returns nonzero when the check itself could not run or the LDS-staged
// kernel disagrees.
int jit_selfcheck(const Program& P, JitKernel* K, hipFunction_t* const* staged, int n_staged,
                  hipFunction_t* offsets_twin, hipFunction_t* offsets_twin_w) {
    const int64_t n = 4096, length = 256;
    const SelfCheckBatch B = selfcheck_batch(P, n, length);
    uint8_t* d_bytes = nullptr;
    uint8_t* d_out = nullptr;
    int64_t* d_first = nullptr;
    int64_t* d_slot = nullptr;
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&d_bytes, (size_t)(n * length));
    if (e == hipSuccess) e = hipMalloc(&d_out, (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&d_first, 8 * (size_t)n);
    if (e == hipSuccess) e = hipMalloc(&d_slot, 4 * sizeof(int64_t));
    const int64_t slot[4] = {1, length, 0, 0};   // an equal-length batch, as the layout check would find it
    if (e == hipSuccess) e = hipMemcpy(d_bytes, B.bytes.data(), (size_t)(n * length), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_slot, slot, sizeof(slot), hipMemcpyHostToDevice);
    std::vector<uint8_t> out((size_t)n);
    std::vector<int64_t> fp((size_t)n);
    // threads, LDS bytes and output of each kernel form
    auto run = [&](hipFunction_t f, int threads, unsigned lds, int kind) -> int {
        // kind 0: accept bits (bytes, length, n, out); 1: earliest accepts; 2: the offsets twin
        long long len = length, nn = n, id = 1;
        const void* b = d_bytes;
        void* o = d_out;
        void* fo = d_first;
        const void* sl = d_slot;
        void* a0[] = {&b, &len, &nn, &o};
        void* a1[] = {&b, &len, &nn, &fo};
        void* a2[] = {&b, &sl, &id, &nn, &o};
        hipError_t r = hipMemsetAsync(kind == 1 ? (void*)d_first : (void*)d_out, 0xff,
                                      kind == 1 ? 8 * (size_t)n : (size_t)n, st);
        if (r == hipSuccess)
            r = hipModuleLaunchKernel(f, (unsigned)((n + 2047) / 2048), 1, 1, threads, 1, 1, lds, st,
                                      kind == 0 ? a0 : kind == 1 ? a1 : a2, nullptr);
        if (r == hipSuccess) r = hipStreamSynchronize(st);
        if (r == hipSuccess && kind != 1) r = hipMemcpy(out.data(), d_out, (size_t)n, hipMemcpyDeviceToHost);
        if (r == hipSuccess && kind == 1) r = hipMemcpy(fp.data(), d_first, 8 * (size_t)n, hipMemcpyDeviceToHost);
        if (r != hipSuccess) return -1;
        if (kind == 1) return fp == B.first ? 0 : 1;
        return out == B.accept ? 0 : 1;
    };
    int rc = e == hipSuccess ? 0 : -1;
    if (!rc && K->fixed) {
        const int bad = run(K->fixed, 64, 2048 * 32, 0);
        if (bad) rc = bad < 0 ? -1 : -2;
    }
    if (!rc) {
        // staged kernels in the order of kStagedKernels: modes 1, 3, 4, 5 (pairs), 5 (words), earliest (pairs, words)
        const int threads[7] = {64, 128, 128, 128, 128, 128, 128};
        const unsigned lds[7] = {2048 * 32, 2048 * 32, 2048 * 32 + 2 * 2048 * 4, 2048 * 32 + 2 * 2048 * 4,
                                 2048 * 32 + 2 * 2048 * 4, 2048 * 32 + 2 * 2048 * 4, 2048 * 32 + 2 * 2048 * 4};
        for (int k = 0; k < n_staged && !rc; ++k) {
            hipFunction_t* f = staged[k];
            // the earliest-accept kernels serve programs whose root is not
            // nullable (the caller answers 0 for every string otherwise)
            if (!*f || (k >= 5 && P.nullable)) continue;
            const int bad = run(*f, threads[k], lds[k], k >= 5 ? 1 : 0);
            if (bad < 0) rc = -1;
            if (bad > 0) {
                *f = nullptr;
                K->selfcheck_dropped |= 1 << k;
            }
        }
        for (hipFunction_t* t : {offsets_twin, offsets_twin_w}) {
            if (rc || !*t) continue;
            const int bad = run(*t, 128, 2048 * 32 + 2 * 2048 * 4, 2);
            if (bad < 0) rc = -1;
            if (bad > 0) {
                *t = nullptr;
                K->selfcheck_dropped |= 1 << (t == offsets_twin ? 3 : 4);   // reported with its kernel
            }
        }
    }
    if (d_bytes) (void)hipFree(d_bytes);
    if (d_out) (void)hipFree(d_out);
    if (d_first) (void)hipFree(d_first);
    if (d_slot) (void)hipFree(d_slot);
    if (st) (void)hipStreamDestroy(st);
    if (!rc) K->selfcheck_ran = 1;
    return rc;
}
}  // namespace

int jit_compile(Program* P, const char* arch_in) {
    int ns = 0, nops = 0;
    const std::string src = jit_full_source(*P, &ns, &nops);
    if (ns > kJitMaxState)
        return fail(RX_ETOOBIG, "the bit-sliced circuit keeps at most " + std::to_string(kJitMaxState) +
                                    " state words in registers; this program needs " + std::to_string(ns));
    std::string arch;
    int dev = -1;
    if (int rc = jit_target(arch_in, &arch, &dev)) return rc;
    std::vector<char> code;
    if (int rc = jit_code(src, arch, &code)) return rc;
    JitKernel* K = new JitKernel;
    K->arch = arch;
    K->n_state = ns;
    K->n_ops = nops;
    // Disassemble the staged kernels: each must leave its accumulation
    // registers to its own loads and LDS writes.
    K->guard_ran = 1;
    for (int k = 0; k < kNumStaged; ++k) {
        int v = 0;
        if (isa_check_agpr_staging(code, arch, kStagedKernels[k], &v, nullptr) != 0) {
            K->guard_ran = 0;   // the check could not run: every staged kernel is dropped
            K->guard_violations[k] = -1;
            continue;
        }
        // the skewed kernels' twins for rx_match's equal-length strings are
        // checked with them (and dropped with them)
        const char* twin = k == 3 ? "rx_sliced_offsets_skew" : k == 4 ? "rx_sliced_offsets_skew_w" : nullptr;
        int vt = 0;
        if (twin && isa_check_agpr_staging(code, arch, twin, &vt, nullptr) != 0) {
            K->guard_ran = 0;
            K->guard_violations[k] = -1;
            continue;
        }
        K->guard_violations[k] = v + vt;
    }
    if (dev >= 0) {
        hipError_t e = hipModuleLoadData(&K->mod, code.data());
        if (e != hipSuccess) { delete K; return fail(RX_EHIP, std::string("hipModuleLoadData: ") + hipGetErrorString(e)); }
        e = hipModuleGetFunction(&K->fixed, K->mod, "rx_sliced_fixed");
        if (e == hipSuccess) e = hipModuleGetFunction(&K->fixed64, K->mod, "rx_sliced_fixed_pf");
        if (e == hipSuccess) e = hipModuleGetFunction(&K->duo, K->mod, "rx_sliced_fixed_duo");
        if (e == hipSuccess) e = hipModuleGetFunction(&K->split, K->mod, "rx_sliced_fixed_split");
        hipFunction_t skew_w = nullptr, first_w = nullptr, off = nullptr, off_w = nullptr;
        if (e == hipSuccess) e = hipModuleGetFunction(&K->skew, K->mod, "rx_sliced_fixed_skew");
        if (e == hipSuccess) e = hipModuleGetFunction(&skew_w, K->mod, "rx_sliced_fixed_skew_w");
        if (e == hipSuccess) e = hipModuleGetFunction(&off, K->mod, "rx_sliced_offsets_skew");
        if (e == hipSuccess) e = hipModuleGetFunction(&off_w, K->mod, "rx_sliced_offsets_skew_w");
        if (e == hipSuccess) e = hipModuleGetFunction(&K->first, K->mod, "rx_sliced_first_skew");
        if (e == hipSuccess) e = hipModuleGetFunction(&first_w, K->mod, "rx_sliced_first_skew_w");
        if (e == hipSuccess && K->n_state <= 2 && hipModuleGetFunction(&K->chunks, K->mod, "rx_sliced_chunks") != hipSuccess) {
            K->chunks = nullptr;
            (void)hipGetLastError();
        }
        if (e == hipSuccess && K->n_state <= kLongChunkMaxState &&
            (hipModuleGetFunction(&K->long_chunks, K->mod, "rx_long_chunks") != hipSuccess ||
             hipModuleGetFunction(&K->long_compose, K->mod, "rx_long_compose") != hipSuccess)) {
            K->long_chunks = K->long_compose = nullptr;
            (void)hipGetLastError();
        }
        if (e != hipSuccess) {
            hipModuleUnload(K->mod);
            delete K;
            return fail(RX_EHIP, std::string("hipModuleGetFunction: ") + hipGetErrorString(e));
        }
        // The staged kernels keep in-flight loads in registers the compiler
        // believes already hold their data; a kernel that spills could move
        // such a register before its load lands.  Those kernels are dropped
        // for this program and the LDS-staged kernel runs instead.
        // Kernels that failed the static check are dropped as well.
        hipFunction_t* staged[kNumStaged] = {&K->fixed64, &K->duo, &K->split, &K->skew, &skew_w, &K->first, &first_w};
        for (int k = 0; k < kNumStaged; ++k) {
            hipFunction_t* f = staged[k];
            int scratch = 1;
            if (hipFuncGetAttribute(&scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, *f) != hipSuccess || scratch != 0)
                *f = nullptr;
            if (*f && (!K->guard_ran || K->guard_violations[k] != 0)) {
                *f = nullptr;
                K->guard_dropped |= 1 << k;
            }
        }
        // the twins share their kernel's fate: no scratch and the static check passed
        for (hipFunction_t* t : {&off, &off_w}) {
            int scratch = 1;
            if (hipFuncGetAttribute(&scratch, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, *t) != hipSuccess || scratch != 0)
                *t = nullptr;
        }
        if (!K->skew) off = nullptr;
        if (!skew_w) off_w = nullptr;
        // Every kernel that is kept runs once on a seeded batch against the
        // table step; one that gives other bits is dropped as well.
        const int sc = jit_selfcheck(*P, K, staged, kNumStaged, &off, &off_w);
        if (sc == -2) {
            hipModuleUnload(K->mod);
            delete K;
            return fail(RX_EJIT, "the bit-sliced kernel gives other bits than the table step on the check batch");
        }
        if (sc != 0) {
            hipModuleUnload(K->mod);
            delete K;
            return fail(RX_EHIP, "the run-time check of the bit-sliced kernels could not run");
        }
        if (!K->skew) off = nullptr;
        if (!skew_w) off_w = nullptr;
        K->skew_words = !K->skew && skew_w;
        K->skew_offsets = K->skew ? off : off_w;
        if (!K->skew) K->skew = skew_w;   // the skewed kernel with single-dword transposer reads
        K->first_words = !K->first && first_w;
        if (!K->first) K->first = first_w;
        K->dev = dev;
    }
    if (P->jit) jit_free(P);
    P->jit = K;
    return RX_OK;
}

void jit_free(Program* P) {
    JitKernel* K = static_cast<JitKernel*>(P->jit);
    if (!K) return;
    if (K->mod) hipModuleUnload(K->mod);
    delete K;
    P->jit = nullptr;
}

bool jit_ready(const Program* P, int* n_state, int* n_ops) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    if (n_state) *n_state = K ? K->n_state : 0;
    if (n_ops) *n_ops = K ? K->n_ops : 0;
    return K && K->fixed;
}

int jit_default_staging(const Program* P) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    if (!K || !K->fixed) return 0;
    return K->skew ? 5 : K->duo ? 3 : 2;
}

void jit_staging(const Program* P, int32_t staged[7]) {
    for (int u = 0; u < 7; ++u) staged[u] = 0;
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    if (!K || !K->fixed) return;
    staged[0] = jit_default_staging(P);
    staged[1] = K->fixed64 ? 1 : 0;
    staged[2] = 1;
    staged[3] = K->duo ? 1 : 0;
    staged[4] = K->split ? 1 : 0;
    staged[5] = K->skew ? (K->skew_words ? 2 : 1) : 0;
    staged[6] = K->first ? (K->first_words ? 2 : 1) : 0;
}

void jit_selfcheck_report(const Program* P, int32_t* ran, int32_t* dropped) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    *ran = K ? K->selfcheck_ran : 0;
    *dropped = K ? K->selfcheck_dropped : 0;
}

void jit_guard(const Program* P, int32_t* ran, int32_t violations[8], int32_t* dropped) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    *ran = K ? K->guard_ran : 0;
    *dropped = K ? K->guard_dropped : 0;
    for (int k = 0; k < 8; ++k) violations[k] = K ? K->guard_violations[k] : -1;
}

bool jit_first_ready(const Program* P) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    return K && K->first;
}

int launch_sliced_first(const Program* P, const uint8_t* bytes, int64_t length, int64_t n, int64_t* first,
                        void* stream) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    if (!K || !K->first || length > (1 << 26)) return (int)hipErrorInvalidValue;
    const long long grid = (n + 2047) / 2048;
    const unsigned lds = 2048 * 32 + 2 * 2048 * 4;
    long long len = length, nn = n;
    const void* b = bytes;
    void* f = first;
    void* args[] = {&b, &len, &nn, &f};
    return (int)hipModuleLaunchKernel(K->first, (unsigned)grid, 1, 1, 128, 1, 1, lds, (hipStream_t)stream, args,
                                      nullptr);
}

bool jit_offsets_ready(const Program* P) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    return K && K->skew_offsets;
}

int launch_sliced_offsets(const Program* P, const uint8_t* bytes, const int64_t* slot, int64_t id, int64_t n,
                          uint8_t* out, void* stream) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    if (!K || !K->skew_offsets) return (int)hipErrorInvalidValue;
    const long long grid = (n + 2047) / 2048;
    const unsigned lds = 2048 * 32 + 2 * 2048 * 4;
    long long i = id, nn = n;
    const void* b = bytes;
    const void* sl = slot;
    void* o = out;
    void* args[] = {&b, &sl, &i, &nn, &o};
    return (int)hipModuleLaunchKernel(K->skew_offsets, (unsigned)grid, 1, 1, 128, 1, 1, lds, (hipStream_t)stream,
                                      args, nullptr);
}

int launch_sliced_fixed(const Program* P, const uint8_t* bytes, int64_t length, int64_t n, uint8_t* out,
                        int burst, void* stream) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    if (!K || !K->fixed) return (int)hipErrorInvalidValue;
    if (burst == 5 && length > (1 << 26)) burst = 4;   // the skewed kernel forms 32-bit per-lane offsets
    hipFunction_t fn = burst == 1 ? K->fixed64 : burst == 3 ? K->duo : burst == 4 ? K->split : burst == 5 ? K->skew
                                                                                                          : K->fixed;
    if (!fn) {   // dropped for this program
        fn = K->fixed;
        burst = 2;
    }
    const unsigned threads = burst >= 3 ? 128 : 64;
    const long long grid = (n + 2047) / 2048;
    // raw tile: 2048 strings x 32 bytes; the transposing kernels add two 8 KiB plane slots
    const unsigned lds = 2048 * 32 + (burst >= 4 ? 2 * 2048 * 4 : 0);
    long long len = length, nn = n;
    const void* b = bytes;
    void* o = out;
    void* args[] = {&b, &len, &nn, &o};
    return (int)hipModuleLaunchKernel(fn, (unsigned)grid, 1, 1, threads, 1, 1, lds, (hipStream_t)stream, args, nullptr);
}

// Chunk length (a multiple of 16) and segments of the long-string form: up to
// about 2,048 segments of 2,048 chunks (two wavefronts per SIMD), chunks of
// at least 16 bytes.
void long_chunk_shape(int64_t length, int64_t* Lc, int64_t* G) {
    int64_t c = (length + 2048 * 2048 - 1) / (2048 * 2048);
    c = (c + 15) / 16 * 16;
    if (c < 16) c = 16;
    *Lc = c;
    *G = (length + 2048 * c - 1) / (2048 * c);
}

// The segments' maps, then every chunk's map (256-byte aligned).
int64_t long_chunk_work_bytes(const Program* P, int64_t length) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    if (!K || !K->long_chunks) return -1;
    int64_t Lc, G;
    long_chunk_shape(length, &Lc, &G);
    const int64_t seg = (4 * G * (K->n_state + 1) + 255) & ~int64_t(255);
    return seg + 4 * G * 2048 * (K->n_state + 1);
}

int launch_long_chunks(const Program* P, const uint8_t* bytes, int64_t length, void* work, uint8_t* out,
                       void* stream) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    if (!K || !K->long_chunks || !K->long_compose) return (int)hipErrorInvalidValue;
    int64_t Lc, G;
    long_chunk_shape(length, &Lc, &G);
    if (G > 0x7fffffffll) return (int)hipErrorInvalidValue;
    long long len = length, lc = Lc, gg = G;
    const void* b = bytes;
    void* w = work;
    void* cm = static_cast<uint8_t*>(work) + ((4 * G * (K->n_state + 1) + 255) & ~int64_t(255));
    void* o = out;
    if (G > 0) {
        void* args[] = {&b, &len, &lc, &w, &cm};
        if (hipError_t e = hipModuleLaunchKernel(K->long_chunks, (unsigned)G, 1, 1, 64, 1, 1, 0, (hipStream_t)stream,
                                                 args, nullptr))
            return (int)e;
    }
    void* args2[] = {&w, &gg, &o};
    return (int)hipModuleLaunchKernel(K->long_compose, 1, 1, 1, 64, 1, 1, 0, (hipStream_t)stream, args2, nullptr);
}

bool jit_chunks_ready(const Program* P) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    return K && K->chunks;
}

int launch_sliced_chunks(const Program* P, const uint8_t* bytes, int64_t length, int64_t n, uint8_t* out,
                         void* stream) {
    const JitKernel* K = static_cast<const JitKernel*>(P->jit);
    if (!K || !K->chunks) return (int)hipErrorInvalidValue;
    if (n > 0x7fffffffll) return (int)hipErrorInvalidValue;
    long long len = length, nn = n;
    const void* b = bytes;
    void* o = out;
    void* args[] = {&b, &len, &nn, &o};
    return (int)hipModuleLaunchKernel(K->chunks, (unsigned)n, 1, 1, 64, 1, 1, 0, (hipStream_t)stream, args, nullptr);
}

}  // namespace rx
