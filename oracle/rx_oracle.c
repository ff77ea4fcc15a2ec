/*
 * rx_oracle.c -- plain, slow CPU oracle for regular expression matching.
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never links or calls this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no source with the HIP library: it parses the AST
 * records itself, builds its own heap, wires its own continuations and runs
 * its own search.
 *
 * What it computes: whether the PW-pi machine of Rathnayake & Thielecke
 * (SOS 2011), Def. 4.5 with the pointer transitions of Fig. 4.2, has a run
 *     <root; w> --> ... --> <null; eps>
 * over the heap of Def. 4.1 with the continuation function of Def. 4.4.
 * The search is plain backtracking over configurations (p, i) -- node p
 * (or null) with i input bytes consumed -- with a visited bitmap, so every
 * configuration is expanded at most once: O((m+1)(n+1)) per string.
 *
 * Extensions beyond the grammar of Section 2 (readings):
 *   CLASS leaf x: x --a--> cont x for every byte a in its 256-bit set.
 *   OPT  p:  p --> child, p --> cont p; cont child = cont p.
 *   PLUS p:  p --> child; cont child = q, a companion loop node with
 *            q --> child and q --> cont p.
 *   search mode: the expression is wrapped as (.* e) .*, '.' = any byte.
 * A configuration <null; w'> with w' non-empty has no successor.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { K_EPS = 0, K_BYTE, K_CLASS, K_CAT, K_ALT, K_STAR, K_PLUS, K_OPT, K_PLUSLOOP = 100 };

typedef struct {
    uint8_t kind, byte;
    uint16_t cls;
    int32_t c0, c1;
} rxo_ast;

typedef struct {
    int32_t m;        /* heap size (nodes incl. PLUS companions); null is index m */
    int32_t root;
    int32_t *kind, *c0, *c1, *cont;
    uint64_t (*label)[4]; /* per node: byte set of a leaf, zero otherwise */
} heap_t;

static void heap_free(heap_t* h) {
    free(h->kind); free(h->c0); free(h->c1); free(h->cont); free(h->label);
    memset(h, 0, sizeof(*h));
}

/* Returns 0 on success, -1 when the AST is not a tree rooted at `root`. */
static int heap_build(heap_t* h, const rxo_ast* ast, int n_ast, int root, const uint64_t* classes,
                      int n_classes, int search) {
    memset(h, 0, sizeof(*h));
    if (n_ast <= 0 || root < 0 || root >= n_ast) return -1;
    int n_tree = n_ast + (search ? 6 : 0);
    int n_plus = 0;
    for (int i = 0; i < n_ast; i++) n_plus += ast[i].kind == K_PLUS;
    int m = n_tree + n_plus;
    h->m = m;
    h->kind = calloc(m, sizeof(int32_t));
    h->c0 = calloc(m, sizeof(int32_t));
    h->c1 = calloc(m, sizeof(int32_t));
    h->cont = calloc(m, sizeof(int32_t));
    h->label = calloc(m, sizeof(*h->label));
    int* parents = calloc(n_tree, sizeof(int));
    int* companion = calloc(n_tree, sizeof(int));
    int* stack = calloc(m + 1, sizeof(int));
    int ok = h->kind && h->c0 && h->c1 && h->cont && h->label && parents && companion && stack;
    for (int i = 0; ok && i < n_ast; i++) {
        const rxo_ast* a = &ast[i];
        h->kind[i] = a->kind;
        h->c0[i] = a->c0;
        h->c1[i] = a->c1;
        switch (a->kind) {
        case K_EPS: break;
        case K_BYTE: h->label[i][a->byte >> 6] |= 1ull << (a->byte & 63); break;
        case K_CLASS:
            if (a->cls >= n_classes) { ok = 0; break; }
            memcpy(h->label[i], classes + 4 * (size_t)a->cls, 4 * sizeof(uint64_t));
            break;
        case K_CAT: case K_ALT:
            if (a->c0 < 0 || a->c0 >= n_ast || a->c1 < 0 || a->c1 >= n_ast) ok = 0;
            else { parents[a->c0]++; parents[a->c1]++; }
            break;
        case K_STAR: case K_PLUS: case K_OPT:
            if (a->c0 < 0 || a->c0 >= n_ast) ok = 0;
            else parents[a->c0]++;
            break;
        default: ok = 0;
        }
    }
    /* tree check: root has no parent, every other node exactly one, all reachable */
    for (int i = 0; ok && i < n_ast; i++)
        if (parents[i] != (i == root ? 0 : 1)) ok = 0;
    if (ok) {
        int sp = 0, seen = 0;
        stack[sp++] = root;
        while (sp) {
            int p = stack[--sp];
            seen++;
            if (seen > n_ast) { ok = 0; break; }
            int k = h->kind[p];
            if (k == K_CAT || k == K_ALT) { stack[sp++] = h->c0[p]; stack[sp++] = h->c1[p]; }
            else if (k == K_STAR || k == K_PLUS || k == K_OPT) stack[sp++] = h->c0[p];
        }
        if (seen != n_ast) ok = 0;
    }
    if (ok && search) {
        int b = n_ast;
        int kinds[6] = {K_CLASS, K_STAR, K_CAT, K_CLASS, K_STAR, K_CAT};
        int k0[6] = {-1, b + 0, b + 1, -1, b + 3, b + 2};
        int k1[6] = {-1, -1, root, -1, -1, b + 4};
        for (int j = 0; j < 6; j++) {
            h->kind[b + j] = kinds[j];
            h->c0[b + j] = k0[j];
            h->c1[b + j] = k1[j];
            if (kinds[j] == K_CLASS) for (int w = 0; w < 4; w++) h->label[b + j][w] = ~0ull;
        }
        root = b + 5;
    }
    if (ok) {
        int q = n_tree;
        for (int i = 0; i < n_ast; i++)
            if (h->kind[i] == K_PLUS) {
                companion[i] = q;
                h->kind[q] = K_PLUSLOOP;
                h->c0[q] = h->c0[i];
                h->c1[q] = -1;
                q++;
            }
        /* Def. 4.4 by a top-down walk with an explicit stack */
        h->root = root;
        h->cont[root] = -1;
        int sp = 0;
        stack[sp++] = root;
        while (sp) {
            int p = stack[--sp];
            int k = h->kind[p], a = h->c0[p], b = h->c1[p];
            if (k == K_ALT) { h->cont[a] = h->cont[p]; h->cont[b] = h->cont[p]; stack[sp++] = a; stack[sp++] = b; }
            else if (k == K_CAT) { h->cont[a] = b; h->cont[b] = h->cont[p]; stack[sp++] = a; stack[sp++] = b; }
            else if (k == K_STAR) { h->cont[a] = p; stack[sp++] = a; }
            else if (k == K_OPT) { h->cont[a] = h->cont[p]; stack[sp++] = a; }
            else if (k == K_PLUS) { int c = companion[p]; h->cont[c] = h->cont[p]; h->cont[a] = c; stack[sp++] = a; }
        }
        /* null is index m in the search below */
        for (int i = 0; i < m; i++) if (h->cont[i] < 0) h->cont[i] = m;
    }
    free(parents); free(companion); free(stack);
    if (!ok) { heap_free(h); return -1; }
    return 0;
}

typedef struct {
    uint64_t* visited;
    size_t visited_words;
    int64_t* stack; /* packed (p, i) */
    size_t stack_cap;
} scratch_t;

static int grow(scratch_t* s, size_t states) {
    size_t words = (states + 63) / 64;
    if (words > s->visited_words) {
        free(s->visited);
        s->visited = malloc(words * sizeof(uint64_t));
        if (!s->visited) return -1;
        s->visited_words = words;
    }
    if (states + 1 > s->stack_cap) {
        free(s->stack);
        s->stack = malloc((states + 1) * sizeof(int64_t));
        if (!s->stack) return -1;
        s->stack_cap = states + 1;
    }
    return 0;
}

/* Def. 4.5: search for <null; eps> from <root; w>.  Returns 1/0, or -1 on allocation failure. */
static int pwpi_run(const heap_t* h, const uint8_t* w, int64_t n, scratch_t* s) {
    const int64_t nodes = (int64_t)h->m + 1; /* including null = m */
    const size_t states = (size_t)nodes * (size_t)(n + 1);
    if (grow(s, states)) return -1;
    memset(s->visited, 0, ((states + 63) / 64) * sizeof(uint64_t));
    size_t sp = 0;
#define PUSH(P, I)                                                                    \
    do {                                                                              \
        size_t id_ = (size_t)(I) * (size_t)nodes + (size_t)(P);                       \
        if (!((s->visited[id_ >> 6] >> (id_ & 63)) & 1)) {                            \
            s->visited[id_ >> 6] |= 1ull << (id_ & 63);                               \
            s->stack[sp++] = (int64_t)id_;                                            \
        }                                                                             \
    } while (0)
    PUSH(h->root, 0);
    while (sp) {
        size_t id = (size_t)s->stack[--sp];
        int64_t i = (int64_t)(id / (size_t)nodes);
        int p = (int)(id % (size_t)nodes);
        if (p == h->m) {
            if (i == n) return 1; /* accepting configuration <null; eps> */
            continue;             /* a null thread with input left has no move */
        }
        switch (h->kind[p]) {
        case K_ALT: PUSH(h->c0[p], i); PUSH(h->c1[p], i); break;
        case K_CAT: PUSH(h->c0[p], i); break;
        case K_STAR: case K_OPT: case K_PLUSLOOP: PUSH(h->c0[p], i); PUSH(h->cont[p], i); break;
        case K_PLUS: PUSH(h->c0[p], i); break;
        case K_EPS: PUSH(h->cont[p], i); break;
        case K_BYTE: case K_CLASS:
            if (i < n) {
                uint8_t a = w[i];
                if ((h->label[p][a >> 6] >> (a & 63)) & 1) PUSH(h->cont[p], i + 1);
            }
            break;
        }
    }
#undef PUSH
    return 0;
}

typedef struct {
    const heap_t* h;
    const uint8_t* bytes;
    const int64_t* offsets;
    const int64_t* index; /* optional subset of string ids */
    int64_t n;
    uint8_t* out;
    int64_t next;          /* shared work counter */
    pthread_mutex_t mu;
    int failed;
} job_t;

static void* worker(void* arg) {
    job_t* j = (job_t*)arg;
    scratch_t s = {0};
    for (;;) {
        pthread_mutex_lock(&j->mu);
        int64_t b = j->next;
        j->next += 16;
        pthread_mutex_unlock(&j->mu);
        if (b >= j->n) break;
        int64_t e = b + 16 < j->n ? b + 16 : j->n;
        for (int64_t k = b; k < e; k++) {
            int64_t sid = j->index ? j->index[k] : k;
            int64_t lo = j->offsets[sid], hi = j->offsets[sid + 1];
            int r = pwpi_run(j->h, j->bytes + lo, hi - lo, &s);
            if (r < 0) { j->failed = 1; r = 0; }
            j->out[k] = (uint8_t)r;
        }
    }
    free(s.visited);
    free(s.stack);
    return NULL;
}

/*
 * Match strings (or the subset `index[0..n)` of them when index != NULL)
 * against one expression.  out[k] = 1 iff string k (resp. index[k]) is in the
 * language.  classes: n_classes x 4 little-endian u64 words (byte b is bit
 * b&63 of word b>>6).  threads <= 0 means 1.
 * Returns 0, -1 for a malformed AST, -2 for an allocation failure.
 */
int rxo_match(const rxo_ast* ast, int n_ast, int root, const uint64_t* classes, int n_classes,
              int search, const uint8_t* bytes, const int64_t* offsets, const int64_t* index,
              int64_t n, uint8_t* out, int threads) {
    heap_t h;
    if (heap_build(&h, ast, n_ast, root, classes, n_classes, search)) return -1;
    job_t j;
    j.h = &h; j.bytes = bytes; j.offsets = offsets; j.index = index; j.n = n; j.out = out;
    j.next = 0; j.failed = 0;
    pthread_mutex_init(&j.mu, NULL);
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    int started = 0;
    for (int t = 1; t < threads; t++)
        if (pthread_create(&tid[started], NULL, worker, &j) == 0) started++;
    worker(&j);
    for (int t = 0; t < started; t++) pthread_join(tid[t], NULL);
    pthread_mutex_destroy(&j.mu);
    heap_free(&h);
    return j.failed ? -2 : 0;
}

/* The continuation table of the oracle's heap (for pinning it to Fig. 4.1).
 * cont_out[p] for p < min(cap, m); null is reported as -1.  Returns m or -1. */
int rxo_heap_cont(const rxo_ast* ast, int n_ast, int root, const uint64_t* classes, int n_classes,
                  int search, int32_t* cont_out, int cap) {
    heap_t h;
    if (heap_build(&h, ast, n_ast, root, classes, n_classes, search)) return -1;
    for (int p = 0; p < h.m && p < cap; p++) cont_out[p] = h.cont[p] == h.m ? -1 : h.cont[p];
    int m = h.m;
    heap_free(&h);
    return m;
}
