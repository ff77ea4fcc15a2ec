// Host compiler: AST -> node array with continuation pointers -> evolution
// tables.  Follows Section 4 (heap, Def. 4.1; tree shape, Def. 4.3; cont,
// Def. 4.4), the two passes of Section 8 (pack the nodes, then wire cont) and
// Def. 5.1 (evolution) of Rathnayake & Thielecke, SOS 2011.
#include <atomic>
#include <algorithm>
#include <cstring>
#include <new>

#include "rx_internal.h"

namespace rx {

namespace {

bool is_leaf(int k) { return k == RX_BYTE || k == RX_CLASS; }
bool is_unary(int k) { return k == RX_STAR || k == RX_PLUS || k == RX_OPT; }
bool is_binary(int k) { return k == RX_CAT || k == RX_ALT; }

struct Tree {
    std::vector<int32_t> kind, c0, c1, label;
    int32_t root = -1;
};

// A1: validate the caller's AST (Def. 4.3: each node belongs to exactly one
// subtree, no cycles along child pointers).
int validate(const rx_ast_node* ast, int32_t n_ast, int32_t root, int32_t n_classes) {
    if (!ast || n_ast <= 0) return fail(RX_EINVAL, "empty AST");
    if (n_ast > kMaxNodes) return fail(RX_ETOOBIG, "AST has more than 2^20 nodes");
    if (root < 0 || root >= n_ast) return fail(RX_EINVAL, "root index out of range");
    if (n_classes < 0) return fail(RX_EINVAL, "negative class count");
    std::vector<int32_t> parents(n_ast, 0);
    for (int32_t i = 0; i < n_ast; ++i) {
        const rx_ast_node& a = ast[i];
        const int k = a.kind;
        if (k > RX_OPT) return fail(RX_EINVAL, "node " + std::to_string(i) + ": bad kind " + std::to_string(k));
        if (k == RX_CLASS && a.cls >= n_classes)
            return fail(RX_EINVAL, "node " + std::to_string(i) + ": class index out of range");
        if (is_unary(k) || is_binary(k)) {
            if (a.c0 < 0 || a.c0 >= n_ast)
                return fail(RX_EINVAL, "node " + std::to_string(i) + ": child 0 out of range");
            ++parents[a.c0];
        }
        if (is_binary(k)) {
            if (a.c1 < 0 || a.c1 >= n_ast)
                return fail(RX_EINVAL, "node " + std::to_string(i) + ": child 1 out of range");
            ++parents[a.c1];
        }
    }
    for (int32_t i = 0; i < n_ast; ++i) {
        const int want = i == root ? 0 : 1;
        if (parents[i] != want) {
            if (i == root) return fail(RX_EINVAL, "root has a parent (cycle through the root)");
            if (parents[i] == 0) return fail(RX_EINVAL, "node " + std::to_string(i) + " is unreachable from the root");
            return fail(RX_EINVAL, "node " + std::to_string(i) + " is shared by " + std::to_string(parents[i]) +
                                       " parents (not a tree)");
        }
    }
    // with parent counts exact, any node not reached from the root lies on a cycle
    std::vector<int32_t> stack{root};
    int32_t seen = 0;
    while (!stack.empty()) {
        const int32_t p = stack.back();
        stack.pop_back();
        if (++seen > n_ast) break;
        const rx_ast_node& a = ast[p];
        if (is_unary(a.kind) || is_binary(a.kind)) stack.push_back(a.c0);
        if (is_binary(a.kind)) stack.push_back(a.c1);
    }
    if (seen != n_ast) return fail(RX_EINVAL, "child pointers form a cycle");
    return RX_OK;
}

}  // namespace

int compile(const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes,
            int32_t n_classes, uint32_t flags, Program** out) {
    if (!out) return fail(RX_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_classes > 0 && !classes) return fail(RX_EINVAL, "classes is NULL");
    if (flags & ~uint32_t(RX_SEARCH)) return fail(RX_EINVAL, "unknown flags");
    if (int rc = validate(ast, n_ast, root, n_classes)) return rc;

    Program* P = new (std::nothrow) Program;
    if (!P) return fail(RX_ENOMEM, "out of host memory");
    static std::atomic<uint64_t> next_uid{1};
    P->uid = next_uid++;
    P->flags = flags;
    for (int32_t i = 0; i < n_classes; ++i) {
        std::array<uint64_t, 4> c;
        std::memcpy(c.data(), classes[i].bits, sizeof(c));
        P->classes.push_back(c);
    }

    // The tree as given, plus the search wrapper ((any)* e)(any)* when asked.
    Tree T;
    T.kind.resize(n_ast);
    T.c0.resize(n_ast);
    T.c1.resize(n_ast);
    T.label.resize(n_ast);
    for (int32_t i = 0; i < n_ast; ++i) {
        const rx_ast_node& a = ast[i];
        T.kind[i] = a.kind;
        T.c0[i] = (is_unary(a.kind) || is_binary(a.kind)) ? a.c0 : -1;
        T.c1[i] = is_binary(a.kind) ? a.c1 : -1;
        T.label[i] = a.kind == RX_BYTE ? a.byte : a.kind == RX_CLASS ? a.cls : -1;
    }
    T.root = root;
    if (flags & RX_SEARCH) {
        const int32_t any = (int32_t)P->classes.size();
        P->classes.push_back({~0ull, ~0ull, ~0ull, ~0ull});
        auto add = [&](int k, int32_t a, int32_t b, int32_t lab) {
            T.kind.push_back(k);
            T.c0.push_back(a);
            T.c1.push_back(b);
            T.label.push_back(lab);
            return (int32_t)T.kind.size() - 1;
        };
        const int32_t dot1 = add(RX_CLASS, -1, -1, any);
        const int32_t pre = add(RX_STAR, dot1, -1, -1);
        const int32_t left = add(RX_CAT, pre, root, -1);
        const int32_t dot2 = add(RX_CLASS, -1, -1, any);
        const int32_t post = add(RX_STAR, dot2, -1, -1);
        T.root = add(RX_CAT, left, post, -1);
    }

    // A2: pack into d[] breadth-first from the root (d[0] = root).
    const int32_t nt = (int32_t)T.kind.size();
    std::vector<int32_t> order;
    order.reserve(nt);
    std::vector<int32_t> newid(nt, -1), depth_of(nt, 0);
    order.push_back(T.root);
    for (size_t h = 0; h < order.size(); ++h) {
        const int32_t p = order[h];
        newid[p] = (int32_t)h;
        if (T.c0[p] >= 0) { depth_of[T.c0[p]] = depth_of[p] + 1; order.push_back(T.c0[p]); }
        if (T.c1[p] >= 0) { depth_of[T.c1[p]] = depth_of[p] + 1; order.push_back(T.c1[p]); }
    }
    int32_t n_plus = 0;
    for (int32_t p = 0; p < nt; ++p) n_plus += T.kind[p] == RX_PLUS;
    const int32_t m = nt + n_plus;
    P->m = m;
    P->n_tree = nt;
    P->kind.assign(m, 0);
    P->c0.assign(m, -1);
    P->c1.assign(m, -1);
    P->label.assign(m, -1);
    P->cont.assign(m, -1);
    P->depth.assign(m, 0);
    std::vector<int32_t> companion(m, -1);
    int32_t next_comp = nt;
    for (int32_t h = 0; h < nt; ++h) {
        const int32_t p = order[h];
        P->kind[h] = T.kind[p];
        P->c0[h] = T.c0[p] >= 0 ? newid[T.c0[p]] : -1;
        P->c1[h] = T.c1[p] >= 0 ? newid[T.c1[p]] : -1;
        P->label[h] = T.label[p];
        P->depth[h] = depth_of[p];
        P->height = std::max(P->height, depth_of[p]);
        if (T.kind[p] == RX_PLUS) {
            const int32_t q = next_comp++;
            companion[h] = q;
            P->kind[q] = RX_PLUSLOOP;
            P->c0[q] = P->c0[h];
            P->depth[q] = depth_of[p];
        }
    }

    // A3: wire cont (Def. 4.4) in one top-down pass; breadth-first order
    // visits every parent before its children, so no recursion is needed.
    P->cont[0] = -1;
    for (int32_t p = 0; p < nt; ++p) {
        const int32_t a = P->c0[p], b = P->c1[p];
        switch (P->kind[p]) {
        case RX_ALT: P->cont[a] = P->cont[p]; P->cont[b] = P->cont[p]; break;
        case RX_CAT: P->cont[a] = b; P->cont[b] = P->cont[p]; break;
        case RX_STAR: P->cont[a] = p; break;
        case RX_OPT: P->cont[a] = P->cont[p]; break;
        case RX_PLUS: {
            const int32_t q = companion[p];
            P->cont[q] = P->cont[p];
            P->cont[a] = q;
            break;
        }
        default: break;
        }
    }

    // leaf ranks in d[] order; the accept bit is rank L
    P->leaf_rank.assign(m, -1);
    for (int32_t p = 0; p < m; ++p)
        if (is_leaf(P->kind[p])) {
            P->leaf_rank[p] = (int32_t)P->leaf_node.size();
            P->leaf_node.push_back(p);
        }
    P->L = (int32_t)P->leaf_node.size();
    if (P->L > kMaxLeaves) {
        const std::string msg = "program has " + std::to_string(P->L) + " leaves; the limit is 4095";
        delete P;
        return fail(RX_ETOOBIG, msg);
    }
    const int32_t L = P->L;
    const int32_t W = (L + 1 + 31) / 32;
    P->W = W;

    // A4: evolution of a single pointer (Def. 5.1 with null kept as the
    // accept bit).  Entering node p reaches the leaves first(p) inside its
    // subtree and, when p can be passed without consuming input (nullable),
    // everything reached from cont p:
    //     E(p) = first(p) OR (nullable(p) ? E(cont p) : 0),   E(null) = {accept}
    // first/nullable are computed bottom-up (reverse breadth-first order puts
    // children before parents); E is memoised along cont chains, which never
    // cycle back to their start.  O(m * W) words.
    std::vector<char> nu(m, 0);
    std::vector<uint32_t> first_of((size_t)m * W, 0);
    auto row = [&](std::vector<uint32_t>& v, int32_t p) { return &v[(size_t)p * W]; };
    for (int32_t p = m - 1; p >= 0; --p) {
        const int32_t a = P->c0[p], b = P->c1[p];
        uint32_t* f = row(first_of, p);
        switch (P->kind[p]) {
        case RX_EPS: nu[p] = 1; break;
        case RX_BYTE:
        case RX_CLASS: {
            const int32_t r = P->leaf_rank[p];
            f[r >> 5] |= 1u << (r & 31);
            break;
        }
        case RX_CAT:
            nu[p] = nu[a] && nu[b];
            for (int w = 0; w < W; ++w) f[w] = row(first_of, a)[w] | (nu[a] ? row(first_of, b)[w] : 0u);
            break;
        case RX_ALT:
            nu[p] = nu[a] || nu[b];
            for (int w = 0; w < W; ++w) f[w] = row(first_of, a)[w] | row(first_of, b)[w];
            break;
        case RX_STAR:
        case RX_OPT:
        case RX_PLUSLOOP:
            nu[p] = 1;
            for (int w = 0; w < W; ++w) f[w] = row(first_of, a)[w];
            break;
        case RX_PLUS:
            nu[p] = nu[a];
            for (int w = 0; w < W; ++w) f[w] = row(first_of, a)[w];
            break;
        default: break;
        }
    }
    // PLUS companions sit after the tree in d[] but read their child's first
    // set, which the loop above filled before reaching them only if the child
    // index is larger; recompute them now that every tree node is done.
    for (int32_t p = nt; p < m; ++p)
        for (int w = 0; w < W; ++w) row(first_of, p)[w] = row(first_of, P->c0[p])[w];
    std::vector<uint32_t> E((size_t)m * W, 0);
    std::vector<char> have(m, 0);
    std::vector<int32_t> chain;
    auto evolve_into = [&](int32_t q, uint32_t* out) {
        // walk q, cont q, ... while nullable, then fold the first sets back
        chain.clear();
        int32_t p = q;
        while (p >= 0 && !have[p]) {
            chain.push_back(p);
            if (!nu[p]) break;
            p = P->cont[p];
        }
        for (size_t k = chain.size(); k-- > 0;) {
            const int32_t c = chain[k];
            uint32_t* e = row(E, c);
            const uint32_t* f = row(first_of, c);
            for (int w = 0; w < W; ++w) e[w] = f[w];
            if (nu[c]) {
                const int32_t nx = P->cont[c];
                if (nx < 0) e[L >> 5] |= 1u << (L & 31);
                else
                    for (int w = 0; w < W; ++w) e[w] |= row(E, nx)[w];
            }
            have[c] = 1;
        }
        if (q < 0) {
            for (int w = 0; w < W; ++w) out[w] = 0;
            out[L >> 5] |= 1u << (L & 31);
        } else {
            for (int w = 0; w < W; ++w) out[w] = row(E, q)[w];
        }
    };
    P->first.assign(W, 0);
    evolve_into(0, P->first.data());
    P->follow.assign((size_t)L * W, 0);
    for (int32_t r = 0; r < L; ++r) evolve_into(P->cont[P->leaf_node[r]], &P->follow[(size_t)r * W]);
    P->bytemask.assign((size_t)256 * W, 0);
    for (int32_t r = 0; r < L; ++r) {
        const int32_t p = P->leaf_node[r];
        if (P->kind[p] == RX_BYTE) {
            P->bytemask[(size_t)P->label[p] * W + (r >> 5)] |= 1u << (r & 31);
            continue;
        }
        const auto& c = P->classes[P->label[p]];
        for (int b = 0; b < 256; ++b)
            if ((c[b >> 6] >> (b & 63)) & 1) P->bytemask[(size_t)b * W + (r >> 5)] |= 1u << (r & 31);
    }
    P->nullable = (P->first[L >> 5] >> (L & 31)) & 1;
    // (e)(any)*: once the accept bit is set it stays set
    {
        bool sa = false;
        if (P->kind[0] == RX_CAT) {
            const int32_t s = P->c1[0];
            if (P->kind[s] == RX_STAR) {
                const int32_t x = P->c0[s];
                if (P->kind[x] == RX_CLASS) {
                    const auto& c = P->classes[P->label[x]];
                    sa = (c[0] & c[1] & c[2] & c[3]) == ~0ull;
                }
            }
        }
        P->suffix_any = sa;
    }

    // device image
    auto align = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    DevLayout& D = P->layout;
    D.first = 0;
    D.follow = align(D.first + 4 * (int64_t)W);
    D.bytemask = align(D.follow + 4 * (int64_t)L * W);
    D.total = align(D.bytemask + 4 * 256 * (int64_t)W);
    // Large programs (run one wavefront per string) also get chunk unions:
    // row (k, v) is the OR of Follow over the leaves 8k + i with bit i set in
    // v, so a byte step reads one row per non-zero survivor byte instead of
    // one per survivor.  Built incrementally: T[k][v] = T[k][v & (v-1)] | Follow[8k + ctz v].
    D.chunks = 0;
    D.n_chunks = 0;
    if (W > kLaneMaxWords) {
        D.n_chunks = 4 * W;  // every byte of every word has a chunk, so no lookup leaves the table
        D.chunks = D.total;
        D.total = align(D.chunks + 4 * (int64_t)D.n_chunks * 256 * W);
    }
    P->blob.assign(D.total, 0);
    std::memcpy(P->blob.data() + D.first, P->first.data(), 4 * (size_t)W);
    if (L) std::memcpy(P->blob.data() + D.follow, P->follow.data(), 4 * (size_t)L * W);
    std::memcpy(P->blob.data() + D.bytemask, P->bytemask.data(), 4 * 256 * (size_t)W);
    if (D.n_chunks) {
        uint32_t* T = reinterpret_cast<uint32_t*>(P->blob.data() + D.chunks);
        for (int32_t k = 0; k < D.n_chunks; ++k) {
            uint32_t* base = T + (size_t)k * 256 * W;
            for (int v = 1; v < 256; ++v) {
                const int i = __builtin_ctz(v);
                const int32_t r = 8 * k + i;
                uint32_t* dst = base + (size_t)v * W;
                const uint32_t* prev = base + (size_t)(v & (v - 1)) * W;
                for (int w = 0; w < W; ++w) dst[w] = prev[w] | (r < L ? P->follow[(size_t)r * W + w] : 0u);
            }
        }
    }

    *out = P;
    return RX_OK;
}

}  // namespace rx
