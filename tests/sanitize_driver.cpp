// Host-only driver for address / undefined-behaviour sanitizer builds of the
// library's host code (the text front end and the compiler) and of the C
// oracle.  It is built with g++/gcc by tests/test_host_sanitizers.py, never
// with the device compiler, and links no HIP code: the error-message helpers
// that the C interface normally provides are defined here.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "rx.h"
#include "rx_internal.h"

namespace rx {
static thread_local std::string g_msg;
int fail(int code, const std::string& msg) {
    g_msg = msg;
    return code;
}
void clear_error() { g_msg.clear(); }
const char* last_error_cstr() { return g_msg.c_str(); }
}  // namespace rx

extern "C" {
typedef struct {
    uint8_t kind, byte;
    uint16_t cls;
    int32_t c0, c1;
} rxo_ast;
int rxo_match(const rxo_ast* ast, int n_ast, int root, const uint64_t* classes, int n_classes, int search,
              const uint8_t* bytes, const int64_t* offsets, const int64_t* index, int64_t n, uint8_t* out,
              int threads);
}

static std::mt19937_64 rng(1108);
static int pick(int n) { return (int)(rng() % (uint64_t)n); }

static std::string random_pattern(int depth) {
    static const char* atoms[] = {"a", "b", ".", "[ab]", "[^a]", "\\d", "[a-c1]", "\\x41", "()", "\\w"};
    const int r = pick(100);
    if (depth >= 4 || r < 30) return atoms[pick(10)];
    if (r < 50) return random_pattern(depth + 1) + random_pattern(depth + 1);
    if (r < 65) return "(" + random_pattern(depth + 1) + "|" + random_pattern(depth + 1) + ")";
    static const char* q[] = {"*", "+", "?", "{2}", "{1,3}", "{0,2}", "{2,}", "{,2}"};
    return "(" + random_pattern(depth + 1) + ")" + q[pick(8)];
}

// Compile, read back nodes and sets, free.  Returns the compile status.
static int compile_and_read(const std::vector<rx_ast_node>& ast, int32_t root, const std::vector<rx_class>& cls,
                            uint32_t flags) {
    rx::Program* P = nullptr;
    const int rc = rx::compile(ast.data(), (int32_t)ast.size(), root, cls.data(), (int32_t)cls.size(), flags, &P);
    if (rc != RX_OK) return rc;
    volatile uint64_t sum = 0;
    for (int32_t i = 0; i < P->m; ++i) sum += (uint64_t)(P->kind[i] + P->c0[i] + P->c1[i] + P->cont[i]);
    for (uint32_t w : P->follow) sum += w;
    for (uint32_t w : P->bytemask) sum += w;
    for (uint8_t b : P->blob) sum += b;
    delete P;
    return RX_OK;
}

int main() {
    int parsed = 0, refused = 0, compiled = 0, rejected = 0, matched = 0;
    // 1. random and malformed pattern text through rx_parse, then the compiler
    const char* bad[] = {"a(b", "ab)", "*a", "a|+", "^ab", "[ab", "a\\", "\\q", "\\x4", "[z-a]", "a{3,2}",
                         "(?:a)", "a{1001}", "((a{1000}){1000}){1000}", "[", "]", "{", "a{2", "\\", ""};
    std::vector<std::string> pats;
    for (const char* b : bad) pats.push_back(b);
    for (int i = 0; i < 400; ++i) pats.push_back(random_pattern(0));
    for (int i = 0; i < 200; ++i) {   // random bytes
        std::string s;
        const int len = pick(12);
        for (int k = 0; k < len; ++k) s.push_back((char)("ab()[]{}|*+?.\\^-,0123x"[pick(23)]));
        pats.push_back(s);
    }
    for (const std::string& pat : pats) {
        int32_t n_ast = 0, root = 0, n_cls = 0;
        int rc = rx_parse(pat.data(), pat.size(), nullptr, 0, &n_ast, &root, nullptr, 0, &n_cls);
        if (rc != RX_OK && !(rc == RX_ETOOBIG && n_ast > 0)) { ++refused; continue; }
        std::vector<rx_ast_node> ast(n_ast > 0 ? n_ast : 1);
        std::vector<rx_class> cls(n_cls > 0 ? n_cls : 1);
        rc = rx_parse(pat.data(), pat.size(), ast.data(), n_ast, &n_ast, &root, cls.data(), n_cls, &n_cls);
        if (rc != RX_OK) { ++refused; continue; }
        ast.resize(n_ast);
        cls.resize(n_cls);
        ++parsed;
        for (uint32_t flags : {0u, (uint32_t)RX_SEARCH}) {
            if (compile_and_read(ast, root, cls, flags) == RX_OK) ++compiled; else ++rejected;
        }
    }
    // 2. random ASTs, many of them malformed (bad kinds, children out of range,
    //    shared children, cycles, bad class ids): the compiler must refuse
    //    them without touching memory it does not own
    for (int it = 0; it < 3000; ++it) {
        const int n = 1 + pick(12);
        std::vector<rx_ast_node> ast(n);
        for (int i = 0; i < n; ++i) {
            ast[i].kind = (uint8_t)pick(10);
            ast[i].byte = (uint8_t)pick(256);
            ast[i].cls = (uint16_t)pick(3);
            ast[i].c0 = pick(n + 2) - 1;
            ast[i].c1 = pick(n + 2) - 1;
        }
        std::vector<rx_class> cls(pick(3));
        for (auto& c : cls)
            for (auto& w : c.bits) w = rng();
        if (compile_and_read(ast, pick(n + 1) - (it % 7 == 0 ? 1 : 0), cls, it & 1 ? RX_SEARCH : 0) == RX_OK)
            ++compiled;
        else
            ++rejected;
    }
    // 3. the oracle on random well-formed programs (from the front end) and
    //    strings, single- and multi-threaded, which must agree
    for (int it = 0; it < 150; ++it) {
        const std::string pat = random_pattern(0);
        int32_t n_ast = 0, root = 0, n_cls = 0;
        const int q = rx_parse(pat.data(), pat.size(), nullptr, 0, &n_ast, &root, nullptr, 0, &n_cls);
        if (q != RX_OK && !(q == RX_ETOOBIG && n_ast > 0)) continue;   // sizes only: no buffers given
        std::vector<rx_ast_node> ast(n_ast);
        std::vector<rx_class> cls(n_cls > 0 ? n_cls : 1);
        if (rx_parse(pat.data(), pat.size(), ast.data(), n_ast, &n_ast, &root, cls.data(), n_cls, &n_cls) != RX_OK)
            continue;
        const int ns = 200;
        std::vector<int64_t> off(ns + 1, 0);
        std::vector<uint8_t> bytes;
        for (int s = 0; s < ns; ++s) {
            const int len = pick(20);
            for (int k = 0; k < len; ++k) bytes.push_back((uint8_t)"ab1A\n"[pick(5)]);
            off[s + 1] = (int64_t)bytes.size();
        }
        if (bytes.empty()) bytes.push_back(0);
        std::vector<uint8_t> o1(ns), o4(ns);
        const int search = it & 1;
        const uint64_t* cw = n_cls ? &cls[0].bits[0] : nullptr;
        const auto* oa = reinterpret_cast<const rxo_ast*>(ast.data());
        if (rxo_match(oa, n_ast, root, cw, n_cls, search, bytes.data(), off.data(), nullptr, ns, o1.data(), 1) ||
            rxo_match(oa, n_ast, root, cw, n_cls, search, bytes.data(), off.data(), nullptr, ns, o4.data(), 4)) {
            std::printf("oracle failed on %s\n", pat.c_str());
            return 1;
        }
        if (o1 != o4) {
            std::printf("oracle threads disagree on %s\n", pat.c_str());
            return 1;
        }
        ++matched;
    }
    std::printf("ok parsed=%d refused=%d compiled=%d rejected=%d matched=%d\n", parsed, refused, compiled, rejected,
                matched);
    return (parsed > 300 && refused > 10 && compiled > 500 && rejected > 500 && matched > 100) ? 0 : 2;
}
