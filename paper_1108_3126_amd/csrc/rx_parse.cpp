// Regular-expression text -> the AST rows rx_compile takes.
//
// The text form of the Section 2 grammar (bytes, concatenation, '|', '*', the
// empty string) plus the extensions the AST carries: byte classes ('.', [...],
// \d \w \s and their complements), '+', '?', and bounded repetition e{m,n},
// which expands into copies of e (every node has one parent, Def. 4.2, so a
// repeated subexpression is copied, never shared).  Matching is of the whole
// string, or of any substring with RX_SEARCH, so '^' and '$' are refused
// rather than given a meaning of their own.  '.' matches every byte,
// newline included.
//
//   alt  := cat ('|' cat)*
//   cat  := post*                                   (nothing: the empty string)
//   post := atom ('*' | '+' | '?' | '{m}' | '{m,}' | '{m,n}' | '{,n}')*
//   atom := byte | '\' escape | '.' | '[' ['^'] items ']' | '(' alt ')'
//
// A '{' that does not open a well-formed bound is an ordinary byte, as is a
// lone '}' or ']'.
#include <array>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "rx.h"
#include "rx_internal.h"

namespace rx {
namespace {

constexpr size_t kMaxParseNodes = size_t(1) << 20;
constexpr int kMaxBound = 1000;
constexpr int kMaxDepth = 2000;

using Bits = std::array<uint64_t, 4>;

Bits bits_of(const char* members) {
    Bits b{};
    for (const unsigned char* p = reinterpret_cast<const unsigned char*>(members); *p; ++p)
        b[*p >> 6] |= uint64_t(1) << (*p & 63);
    return b;
}
Bits bits_range(int lo, int hi) {
    Bits b{};
    for (int c = lo; c <= hi; ++c) b[c >> 6] |= uint64_t(1) << (c & 63);
    return b;
}
Bits operator|(Bits a, const Bits& b) {
    for (int w = 0; w < 4; ++w) a[w] |= b[w];
    return a;
}
Bits complement(Bits a) {
    for (int w = 0; w < 4; ++w) a[w] = ~a[w];
    return a;
}
const Bits kDigit = bits_range('0', '9');
const Bits kWord = bits_range('a', 'z') | bits_range('A', 'Z') | kDigit | bits_of("_");
const Bits kSpace = bits_of(" \t\n\r\f\v");

struct ParseError {
    size_t pos;
    std::string msg;
    int code;
};

struct Parser {
    const unsigned char* s;
    size_t n;
    size_t i = 0;
    int depth = 0;
    std::vector<rx_ast_node> ast;
    std::vector<Bits> classes;
    std::map<Bits, int> class_id;

    [[noreturn]] void error(const std::string& m, int code = RX_EINVAL) { throw ParseError{i, m, code}; }
    bool at_end() const { return i >= n; }
    int peek() const { return i < n ? s[i] : -1; }

    int node(int kind, int byte, int cls, int c0, int c1) {
        if (ast.size() >= kMaxParseNodes)
            error("the expression expands to more than " + std::to_string(kMaxParseNodes) + " nodes", RX_ETOOBIG);
        rx_ast_node a;
        a.kind = (uint8_t)kind;
        a.byte = (uint8_t)byte;
        a.cls = (uint16_t)cls;
        a.c0 = c0;
        a.c1 = c1;
        ast.push_back(a);
        return (int)ast.size() - 1;
    }
    int byte_node(int b) { return node(RX_BYTE, b, 0, -1, -1); }
    int class_node(const Bits& b) {
        auto it = class_id.find(b);
        int id;
        if (it != class_id.end()) {
            id = it->second;
        } else {
            if (classes.size() >= 65536) error("more than 65536 distinct byte classes", RX_ETOOBIG);
            id = (int)classes.size();
            classes.push_back(b);
            class_id.emplace(b, id);
        }
        return node(RX_CLASS, 0, id, -1, -1);
    }

    // a fresh copy of the subtree at r (iterative: chains can be deep)
    int copy(int r) {
        std::vector<std::pair<int, int>> todo;   // (source node, destination node)
        const int root = node(ast[r].kind, ast[r].byte, ast[r].cls, -1, -1);
        todo.push_back({r, root});
        while (!todo.empty()) {
            const auto [src, dst] = todo.back();
            todo.pop_back();
            const int c0 = ast[src].c0, c1 = ast[src].c1;
            if (c0 >= 0) {
                const int d = node(ast[c0].kind, ast[c0].byte, ast[c0].cls, -1, -1);
                ast[dst].c0 = d;
                todo.push_back({c0, d});
            }
            if (c1 >= 0) {
                const int d = node(ast[c1].kind, ast[c1].byte, ast[c1].cls, -1, -1);
                ast[dst].c1 = d;
                todo.push_back({c1, d});
            }
        }
        return root;
    }

    int parse_alt() {
        if (++depth > kMaxDepth) error("groups nested more than " + std::to_string(kMaxDepth) + " deep", RX_ETOOBIG);
        int left = parse_cat();
        while (peek() == '|') {
            ++i;
            const int right = parse_cat();
            left = node(RX_ALT, 0, 0, left, right);
        }
        --depth;
        return left;
    }

    int parse_cat() {
        int left = -1;
        while (!at_end() && peek() != '|' && peek() != ')') {
            const int p = parse_post();
            left = left < 0 ? p : node(RX_CAT, 0, 0, left, p);
        }
        return left < 0 ? node(RX_EPS, 0, 0, -1, -1) : left;
    }

    // reads {m}, {m,}, {m,n} or {,n} at i (pointing at '{'); false (i unchanged) if not one
    bool bound(int* m, int* nmax) {
        size_t j = i + 1;
        auto digits = [&](int* v) {
            size_t k = j;
            long long x = 0;
            while (j < n && s[j] >= '0' && s[j] <= '9') {
                x = x * 10 + (s[j] - '0');
                if (x > kMaxBound) x = kMaxBound + 1;
                ++j;
            }
            *v = (int)x;
            return j > k;
        };
        int lo = 0, hi = -1;
        const bool has_lo = digits(&lo);
        if (j < n && s[j] == ',') {
            ++j;
            const bool has_hi = digits(&hi);
            if (!has_lo && !has_hi) return false;
            if (!has_hi) hi = -1;   // unbounded
        } else {
            if (!has_lo) return false;
            hi = lo;
        }
        if (j >= n || s[j] != '}') return false;
        if (lo > kMaxBound || hi > kMaxBound) error("repetition bounds above " + std::to_string(kMaxBound), RX_ETOOBIG);
        if (hi >= 0 && hi < lo) error("repetition {m,n} with n < m");
        i = j + 1;
        *m = lo;
        *nmax = hi;
        return true;
    }

    // e{m,n} = e ... e (m copies) followed by n - m optional copies; e{m,} = e^m e*
    int repeat(int e, int m, int hi) {
        std::vector<int> parts;
        bool used = false;
        auto take = [&]() {
            const int c = used ? copy(e) : e;
            used = true;
            return c;
        };
        for (int k = 0; k < m; ++k) parts.push_back(take());
        if (hi < 0) {
            parts.push_back(node(RX_STAR, 0, 0, take(), -1));
        } else {
            for (int k = m; k < hi; ++k) parts.push_back(node(RX_OPT, 0, 0, take(), -1));
        }
        if (parts.empty()) return node(RX_EPS, 0, 0, -1, -1);   // e{0} and e{0,0}
        int left = parts[0];
        for (size_t k = 1; k < parts.size(); ++k) left = node(RX_CAT, 0, 0, left, parts[k]);
        return left;
    }

    int parse_post() {
        int a = parse_atom();
        for (;;) {
            const int c = peek();
            if (c == '*') {
                ++i;
                a = node(RX_STAR, 0, 0, a, -1);
            } else if (c == '+') {
                ++i;
                a = node(RX_PLUS, 0, 0, a, -1);
            } else if (c == '?') {
                ++i;
                a = node(RX_OPT, 0, 0, a, -1);
            } else if (c == '{') {
                int m, hi;
                if (!bound(&m, &hi)) break;   // a literal '{' starts the next atom
                a = repeat(a, m, hi);
            } else {
                break;
            }
        }
        return a;
    }

    int hex_digit(int c) {
        if (c >= '0' && c <= '9') return c - '0';
        if (c >= 'a' && c <= 'f') return c - 'a' + 10;
        if (c >= 'A' && c <= 'F') return c - 'A' + 10;
        return -1;
    }

    // an escape after '\' (i points past the backslash): a single byte (returned,
    // *set untouched) or a class (returns -1 and fills *set).  Inside brackets
    // \b is the backspace byte.
    int escape(Bits* set, bool in_class = false) {
        if (at_end()) error("trailing backslash");
        const int c = s[i++];
        if (in_class && c == 'b') return 8;
        switch (c) {
        case 'n': return '\n';
        case 't': return '\t';
        case 'r': return '\r';
        case 'f': return '\f';
        case 'v': return '\v';
        case 'a': return 7;
        case '0': return 0;
        case 'x': {
            const int h = i < n ? hex_digit(s[i]) : -1, l = i + 1 < n ? hex_digit(s[i + 1]) : -1;
            if (h < 0 || l < 0) error("\\x needs two hex digits");
            i += 2;
            return h * 16 + l;
        }
        case 'd': *set = kDigit; return -1;
        case 'D': *set = complement(kDigit); return -1;
        case 'w': *set = kWord; return -1;
        case 'W': *set = complement(kWord); return -1;
        case 's': *set = kSpace; return -1;
        case 'S': *set = complement(kSpace); return -1;
        default:
            if ((c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || (c >= '0' && c <= '9')) {
                --i;
                error(std::string("unsupported escape \\") + (char)c);
            }
            return c;   // any other byte stands for itself
        }
    }

    int parse_class() {   // i points past '['
        bool negate = false;
        if (peek() == '^') {
            negate = true;
            ++i;
        }
        Bits set{};
        bool first = true;
        for (;;) {
            if (at_end()) error("unterminated [ ... ] class");
            int c = s[i];
            if (c == ']' && !first) {
                ++i;
                break;
            }
            first = false;
            int lo;
            ++i;
            if (c == '\\') {
                Bits esc{};
                lo = escape(&esc, true);
                if (lo < 0) {   // \d, \w, \s ... inside the brackets
                    set = set | esc;
                    continue;
                }
            } else {
                lo = c;
            }
            // a range lo-hi (a '-' before ']' or at the end is itself a member)
            if (peek() == '-' && i + 1 < n && s[i + 1] != ']') {
                ++i;
                int hi = s[i++];
                if (hi == '\\') {
                    Bits esc{};
                    hi = escape(&esc, true);
                    if (hi < 0) error("a class escape cannot end a range");
                }
                if (hi < lo) error("range out of order in [ ... ]");
                set = set | bits_range(lo, hi);
            } else {
                set[lo >> 6] |= uint64_t(1) << (lo & 63);
            }
        }
        return class_node(negate ? complement(set) : set);
    }

    int parse_atom() {
        const int c = s[i];
        switch (c) {
        case '(': {
            ++i;
            if (peek() == '?') error("group flags (?...) are not supported");
            const int a = parse_alt();
            if (peek() != ')') error("missing )");
            ++i;
            return a;
        }
        case '[': ++i; return parse_class();
        case '.': ++i; return class_node(complement(Bits{}));
        case '\\': {
            ++i;
            Bits set{};
            const int b = escape(&set);
            return b >= 0 ? byte_node(b) : class_node(set);
        }
        case '*': case '+': case '?': error("nothing to repeat");
        case '^': case '$':
            error("anchors are implicit: matching is of the whole string, or of any substring with RX_SEARCH");
        default: ++i; return byte_node(c);
        }
    }
};

}  // namespace
}  // namespace rx

using namespace rx;

int rx_parse(const char* pattern, size_t len, rx_ast_node* ast, int32_t ast_cap, int32_t* n_ast, int32_t* root,
             rx_class* classes, int32_t class_cap, int32_t* n_classes) {
    try {
        if (!pattern && len) return fail(RX_EINVAL, "pattern is NULL");
        if (!n_ast || !root || !n_classes) return fail(RX_EINVAL, "NULL output argument");
        if (ast_cap < 0 || class_cap < 0) return fail(RX_EINVAL, "negative capacity");
        Parser P;
        P.s = reinterpret_cast<const unsigned char*>(pattern ? pattern : "");
        P.n = len;
        int r;
        try {
            r = P.parse_alt();
            if (!P.at_end()) P.error("unbalanced )");
        } catch (const ParseError& e) {
            return fail(e.code, "regex at byte " + std::to_string(e.pos) + ": " + e.msg);
        }
        // e{0} leaves its operand unreferenced: keep only the nodes reachable from the root
        {
            std::vector<int> order, map(P.ast.size(), -1);
            order.push_back(r);
            map[r] = 0;
            for (size_t k = 0; k < order.size(); ++k) {
                for (int c : {P.ast[order[k]].c0, P.ast[order[k]].c1}) {
                    if (c >= 0 && map[c] < 0) {
                        map[c] = (int)order.size();
                        order.push_back(c);
                    }
                }
            }
            std::vector<rx_ast_node> kept(order.size());
            for (size_t k = 0; k < order.size(); ++k) {
                kept[k] = P.ast[order[k]];
                if (kept[k].c0 >= 0) kept[k].c0 = map[kept[k].c0];
                if (kept[k].c1 >= 0) kept[k].c1 = map[kept[k].c1];
            }
            P.ast.swap(kept);
            r = 0;
        }
        *n_ast = (int32_t)P.ast.size();
        *n_classes = (int32_t)P.classes.size();
        *root = r;
        if ((int64_t)P.ast.size() > ast_cap || (int64_t)P.classes.size() > class_cap)
            return fail(RX_ETOOBIG, "the AST needs " + std::to_string(P.ast.size()) + " nodes and " +
                                        std::to_string(P.classes.size()) + " classes");
        if (!P.ast.empty()) {
            if (!ast) return fail(RX_EINVAL, "ast is NULL");
            std::memcpy(ast, P.ast.data(), P.ast.size() * sizeof(rx_ast_node));
        }
        if (!P.classes.empty()) {
            if (!classes) return fail(RX_EINVAL, "classes is NULL");
            for (size_t k = 0; k < P.classes.size(); ++k)
                for (int w = 0; w < 4; ++w) classes[k].bits[w] = P.classes[k][w];
        }
        return RX_OK;
    } catch (const std::bad_alloc&) {
        return fail(RX_ENOMEM, "out of host memory");
    } catch (...) {
        return fail(RX_EINVAL, "internal error");
    }
}
