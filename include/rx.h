/*
 * rx.h -- C interface of the MI355X lockstep regular expression matcher.
 *
 * The library implements the lockstep construction of Rathnayake & Thielecke,
 * "Regular Expression Matching and Operational Semantics" (SOS 2011): an
 * expression is laid out as a heap of nodes with continuation pointers
 * (Section 4, Def. 4.1 and Def. 4.4), and every input byte advances the whole
 * set of live threads at once (Section 5, Def. 5.2 / 5.3), duplicate threads
 * collapsing by pointer equality (the remark closing Section 3).  Thread sets
 * are bitsets over node indices; the per-byte macro step runs in hand-written
 * HIP kernels for gfx950.
 *
 * Conventions for every call:
 *   - Every function returns an int status: RX_OK (0) or a negative RX_E*
 *     code.  Nothing throws across this interface.  On failure a message is
 *     available from rx_last_error() on the same host thread.
 *   - Pointers named d_* are device pointers on the current HIP device (for
 *     example the data_ptr() of a torch tensor); everything else is host
 *     memory.  The caller owns every buffer it passes in.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued on it asynchronously; the library never
 *     synchronises the stream unless a call says so.
 */
#ifndef RX_H
#define RX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
    RX_OK = 0,
    RX_EINVAL = -1,        /* malformed AST or bad argument */
    RX_ETOOBIG = -2,       /* program above a kernel limit, or request above a budget */
    RX_ENOTUPLOADED = -3,  /* rx_match on a program without device tables */
    RX_EHIP = -4,          /* a HIP runtime call failed; message holds its error string */
    RX_EBUSY = -5,         /* server over its memory budget in non-blocking mode */
    RX_ENOMEM = -6,        /* host allocation failed */
    RX_EJIT = -7,          /* run-time kernel generation or compilation failed */
    RX_ETIMEOUT = -8       /* a wait reached its deadline */
};

/* Node kinds.  EPS, BYTE, CAT (concatenation), ALT and STAR are the grammar of
 * Section 2.  CLASS (a set of bytes), PLUS (one or more) and OPT (zero or one)
 * extend it: a CLASS leaf x moves x --a--> cont x for every byte a in its set;
 * OPT p moves to its child and to cont p, and its child's continuation is
 * cont p; PLUS p moves to its child, whose continuation is a companion loop
 * node q (RX_PLUSLOOP, created by rx_compile) that moves to the child and to
 * cont p. */
enum {
    RX_EPS = 0,
    RX_BYTE = 1,
    RX_CLASS = 2,
    RX_CAT = 3,
    RX_ALT = 4,
    RX_STAR = 5,
    RX_PLUS = 6,
    RX_OPT = 7,
    RX_PLUSLOOP = 8 /* only in compiled programs, never in an input AST */
};

/* rx_compile flags. */
enum {
    RX_SEARCH = 1u /* match .*(e).* (any substring) instead of the whole string */
};

/* One AST node.  Children are indices into the same array; an unused child is
 * -1.  BYTE uses `byte`, CLASS uses `cls` (an index into the class array). */
typedef struct {
    uint8_t kind;
    uint8_t byte;
    uint16_t cls;
    int32_t c0, c1;
} rx_ast_node;

/* A set of bytes: byte b is bit (b & 63) of bits[b >> 6]. */
typedef struct {
    uint64_t bits[4];
} rx_class;

/*
 * rx_parse -- regular-expression text into the AST rows rx_compile takes.
 *
 * The text form of the Section 2 grammar (bytes, concatenation, '|', '*',
 * the empty string, parentheses) and the extensions of the node kinds above:
 * '.' (every byte, newline included), bracket classes [abc] [a-z] [^...],
 * the escapes \d \w \s \D \W \S (ASCII digits, word bytes, white space),
 * \n \t \r \f \v \a \0 \xHH, any other non-alphanumeric byte after '\'
 * standing for itself, '+', '?', and bounded repetition {m} {m,} {m,n} {,n}
 * (n <= 1000), which expands into copies of the repeated expression (a node
 * has one parent, Def. 4.2).  A '{' that does not open a well-formed bound is
 * an ordinary byte.  Matching is of the whole string (or any substring with
 * RX_SEARCH), so '^' and '$' are refused.  The pattern is len bytes, not
 * NUL-terminated; bytes >= 0x80 are ordinary bytes.
 *
 * On success: ast[0 .. *n_ast) and classes[0 .. *n_classes) hold the tree,
 * *root its root.  If ast_cap or class_cap is too small the call returns
 * RX_ETOOBIG with *n_ast and *n_classes set to the sizes needed (ast and
 * classes may be NULL when their capacity is 0), so a caller can size its
 * buffers with a first call.  Errors: RX_EINVAL (syntax; the message gives
 * the byte position), RX_ETOOBIG (buffers, or more than 2^20 nodes after
 * expanding repetitions).
 */
int rx_parse(const char* pattern, size_t len, rx_ast_node* ast, int32_t ast_cap, int32_t* n_ast, int32_t* root,
             rx_class* classes, int32_t class_cap, int32_t* n_classes);

/* One node of a compiled program's node array d[] (the heap of Def. 4.1).
 * label: the byte of a BYTE leaf, the class index of a CLASS leaf (the search
 * wrapper's any-byte class is appended after the caller's classes), -1
 * otherwise.  cont: the continuation pointer of Def. 4.4, -1 for null. */
typedef struct {
    int32_t kind, c0, c1, label, cont;
} rx_node;

/* Facts about a compiled program. */
typedef struct {
    int32_t m;           /* nodes in d[], including search wrapper and PLUS companions */
    int32_t n_leaves;    /* L: leaves (BYTE and CLASS nodes); the accept bit has index L */
    int32_t words;       /* 32-bit words per thread set: ceil((L + 1) / 32) */
    int32_t nullable;    /* 1 if the empty string is accepted */
    int32_t suffix_any;  /* 1 if the root is (e)(any byte)*: acceptance is then absorbing */
    int32_t search;      /* 1 if compiled with RX_SEARCH */
    int64_t table_bytes; /* device bytes rx_program_upload needs */
    int32_t depth;       /* height of the node tree (root = 0) */
    int32_t n_classes;   /* classes including the wrapper's any-byte class */
} rx_info;

typedef struct rx_program rx_program; /* opaque; owned by the library */

/*
 * rx_compile -- validate an AST and build its program.
 *
 * Checks (Def. 4.3 with the disjoint union of Def. 4.2): kinds in range,
 * children in range, every node except `root` has exactly one parent, the
 * root none, every node reachable from the root (so there are no cycles),
 * class indices < n_classes.  The tree is packed into d[] in breadth-first
 * order with the root at d[0] (Section 8: the root node is the one scheduled
 * first); PLUS companions follow the tree nodes.  cont is wired by a second,
 * iterative pass (Def. 4.4).  Then the evolution tables of Def. 5.1 are
 * precomputed: First = the leaves (and accept bit) reachable from the root by
 * non-consuming moves, Follow[x] = those reachable from cont x, and for each
 * byte b the set of leaves whose label holds b.
 *
 * ast/n_ast/root: the tree; classes/n_classes: its byte classes (may be NULL
 * when n_classes is 0); flags: RX_SEARCH or 0.  On success *out owns a new
 * program (free it with rx_program_free).  Errors: RX_EINVAL (malformed),
 * RX_ETOOBIG (more than 4095 leaves or 2^20 nodes), RX_ENOMEM.
 */
int rx_compile(const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes,
               int32_t n_classes, uint32_t flags, rx_program** out);

/* Frees the program and its host tables.  Device memory handed to
 * rx_program_upload stays the caller's.  NULL is ignored. */
void rx_program_free(rx_program* prog);

/* Fills *out.  Errors: RX_EINVAL on NULL arguments. */
int rx_program_info(const rx_program* prog, rx_info* out);

/* Copies the node array d[] (with cont) into out[0 .. min(cap, m)) and sets
 * *m to the program's node count.  out may be NULL to query m only. */
int rx_program_nodes(const rx_program* prog, rx_node* out, int32_t cap, int32_t* m);

/*
 * Copies the evolution tables (Def. 5.1) to host memory, each optional (NULL
 * skips it).  Sets are `words` 32-bit words, leaf rank r is bit (r & 31) of
 * word r >> 5 and the accept bit is rank L.
 *   first[words]            -- the evolution of {root}
 *   follow[L * words]       -- row r: the evolution of {cont x} for the leaf x of rank r
 *   bytemask[256 * words]   -- row b: the leaves whose label holds byte b
 *   leaf_node[L]            -- the d[] index of the leaf of each rank
 */
int rx_program_sets(const rx_program* prog, uint32_t* first, uint32_t* follow, uint32_t* bytemask,
                    int32_t* leaf_node);

/*
 * Copies the program's device tables into d_buf (at least info.table_bytes
 * bytes, 256-byte aligned, on the current device) with an asynchronous copy
 * on `stream`, and records d_buf in the program.  The caller keeps d_buf
 * alive while the program is matched.  Errors: RX_EINVAL, RX_ETOOBIG (cap too
 * small), RX_EHIP.
 */
int rx_program_upload(rx_program* prog, void* d_buf, size_t cap, void* stream);

/*
 * rx_match -- one match bit per string (the lockstep machine of Def. 5.3).
 *
 * String i is d_bytes[d_offsets[i] .. d_offsets[i+1]); offsets are int64 and
 * must satisfy 0 <= offsets[i] <= offsets[i+1] (not checked on the device).
 * d_out[i] is set to 1 if string i is in the language (a substring of it, for
 * RX_SEARCH), else 0.  Runs asynchronously on `stream`; allocates nothing.
 * n == 0 is a no-op.  The kernel variant is chosen from the program's size
 * and the string count: wavefronts per string for sets above 16 words, and
 * for sets of 6-16 words when the strings number at most four per SIMD
 * (16 x compute units); otherwise one lane per string.  When the program's bit-sliced circuit is compiled
 * (rx_program_jit) and n >= 16384, a check on the device decides whether the
 * strings are equal-length and consecutive (offsets[i] = offsets[0] + i * len,
 * len a multiple of 16 up to 2^26, d_bytes + offsets[0] 16-byte aligned); if
 * so the bit-sliced kernel of rx_match_fixed matches them and the table-form
 * launch does nothing, else the reverse (both are queued; the bits are the
 * same either way).  The check keeps its verdict in a slot of a static array
 * per device (4096 slots, one per call in turn); a call whose slot is taken
 * by a later call before its kernels run falls back to the table form.
 * Errors: RX_EINVAL, RX_ENOTUPLOADED, RX_EHIP.
 */
int rx_match(const rx_program* prog, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t n,
             uint8_t* d_out, void* stream);

/* Kernel variants for rx_match_ex. */
enum {
    RX_VARIANT_AUTO = 0,
    RX_VARIANT_LANE = 1,   /* one lane owns one string and its set (sets of <= 16 words) */
    RX_VARIANT_WAVE = 2,   /* one wavefront owns one string; lane j owns word j of the set */
    RX_VARIANT_SLICED = 3, /* bit-sliced node circuit: one lane runs 32 strings at once
                              (needs rx_program_jit) */
    RX_VARIANT_CHUNKS = 4  /* rx_match_fixed_ex only: the bit-sliced circuit run chunk-parallel, for
                              circuits of at most two state words (rx_program_jit_stats): one
                              wavefront per string, the string cut into 2,048 chunks, each chunk run
                              from every one of the 2^words states (the step of Def. 5.1 depends on
                              the state and the byte alone, so a chunk is a map of states) and the
                              maps composed in order; any alignment and length */
};

/* Launch parameters; zero fields mean "default". */
typedef struct {
    int32_t variant;        /* RX_VARIANT_* */
    int32_t block;          /* threads per workgroup (multiple of 64, <= 1024) */
    int32_t grid;           /* workgroups (0 = enough for one pass over the strings) */
    int32_t unroll;         /* sliced: 1 = prefetch the next tile into registers while matching,
                               2 = load each tile, then match it, 3 = a loader wave fetches 64-byte bursts,
                               4 = as 3, and the second wave also transposes bytes into bit planes while the
                               first runs the circuit, 5 = as 4, with each wave fetching whole 64-byte bursts
                               for half of the strings, that half running 32 bytes behind the other so the two
                               waves' requests alternate (default).  A program whose staged kernels (1, 3, 4,
                               5) would spill registers runs 2 instead; 5 needs length <= 2^26 (else 4).
                               0 = 5 when its kernel was kept, else 3, else 2.
                               wave: wavefronts per string, 1, 2, 4, 8 or 16 (each takes every 2nd ...
                               16th survivor word and the partial next sets meet in LDS once per byte);
                               0 = the most that leave every wavefront at least three set words and
                               put at most four wavefronts on a SIMD (strings x wavefronts <= 4 x SIMDs),
                               else 1. */
} rx_launch;

/* Earliest accepting prefix (the accept bit's first appearance, Def. 5.3
 * applied to every prefix): d_first[i] = the smallest k in [0, len_i] such
 * that the first k bytes of string i are accepted, or -1 if no prefix is.
 * With RX_SEARCH this is the end offset of the match that ends first; without
 * it, the length of the shortest prefix in the language (k = len_i is a
 * whole-string match only when no shorter prefix matched).  Strings and
 * offsets as for rx_match; d_first is int64[n] on the device.  Runs the
 * table-form kernels (one lane per string up to 16 words, else one
 * wavefront per string), stopping each string at its first accept.  Errors
 * as rx_match. */
int rx_match_first(const rx_program* prog, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t n,
                   int64_t* d_first, void* stream);

/* rx_match_first for fixed-length strings (string i = d_bytes[i*length,
 * (i+1)*length)).  With a compiled circuit (rx_program_jit), 16-byte aligned
 * bytes and length % 16 == 0 (length <= 2^26), the skewed bit-sliced kernel
 * runs, recording each string's first accept as it appears; otherwise the
 * table-form kernels.  d_first: caller-owned device int64[n]; entry i = the
 * length of the shortest prefix of string i that the program accepts (with
 * RX_SEARCH: where the earliest-ending match ends), -1 if none.  A program
 * whose root is nullable answers 0 for every string without matching.
 * Asynchronous on stream; allocates nothing.  Errors as rx_match_fixed. */
int rx_match_first_fixed(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int64_t n,
                         int64_t* d_first, void* stream);

/* Chunk-parallel matching of one long string d_bytes[0, length): the result
 * bit (1 byte) goes to d_out[0].  The byte step of the lockstep machine maps a
 * union of thread sets to the union of their images (§5, Def. 5.1 / 5.2: a
 * set evolves pointer by pointer), so a chunk of the input acts on sets as a
 * relation: T[r] = the set reached from leaf r alone.  A first launch runs,
 * in parallel, chunk 0 from First and every later chunk from every single
 * leaf (and from the accept bit alone), one lane per run for sets of at most
 * 16 words, one wavefront above; a second launch applies the relations in
 * order.  Work grows by the number of leaves, time falls by the number of
 * chunks: for strings far longer than the expression.
 * chunks: 0 = about sqrt(length / 2) for sets of at most 16 words and
 * sqrt(length / 20) above, else the count wanted (at most 4096 and at most
 * length are used).  d_work: caller-owned device memory of at
 * least rx_match_long_workspace bytes (the rows: their sets as u32 words, then
 * one int64 each for rx_match_first_long), overwritten;
 * d_out: caller-owned device byte, 0 or 1.  Asynchronous on stream: d_bytes
 * and d_work stay in use until the stream passes the call; allocates
 * nothing.  Length 0 gives the nullable bit.
 * With chunks = 0 and a compiled circuit (rx_program_jit) of at most 31 state
 * words, the string runs as circuit chunks instead: every update of the
 * circuit's step (and its accept bit) is an OR of terms that read at most one
 * state word, so a chunk maps a state to the image of the empty state OR the
 * images of its words alone; one wavefront per segment of 2,048 chunks runs
 * each chunk from the empty state and from every word alone (bit j of a
 * circuit word = chunk j of a lane), composes the chunks' maps in order, and a
 * second launch composes the segments' maps and applies them to the start
 * state; the workspace holds every chunk's map (4 (words + 1) bytes per chunk,
 * chunks of at least 16 bytes, at most about 2,048 x 2,048 of them) and the
 * segments' maps.
 * rx_match_long_workspace(.., chunks = 0, ..) covers both forms.
 * Errors: RX_EINVAL (NULL buffers, negative sizes, short workspace),
 * RX_ENOTUPLOADED, RX_ETOOBIG (sets above 128 words), RX_EHIP. */
int rx_match_long_workspace(const rx_program* prog, int64_t length, int32_t chunks, size_t* bytes);
int rx_match_long(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int32_t chunks, void* d_work,
                  size_t work_bytes, uint8_t* d_out, void* stream);

/* rx_match_first for one long string, in chunks as rx_match_long: each row
 * also records how many bytes of its chunk it reads before its first accept;
 * the composition stops at the first chunk where a live row accepts.
 * d_first: caller-owned device int64, the length of the shortest accepted
 * prefix (with RX_SEARCH: where the earliest-ending match ends), or -1.  A
 * nullable program answers 0.  Workspace, chunks and errors as rx_match_long
 * (rx_match_long_workspace covers both). */
int rx_match_first_long(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int32_t chunks, void* d_work,
                        size_t work_bytes, int64_t* d_first, void* stream);

/* rx_match_long for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result, with the rows held in a static device array of 16 MiB that the
 * library owns (one per GPU it runs on, kept until the process ends) instead
 * of a caller workspace.  No hipMalloc, hipFree or allocating call is made.
 * chunks = 0 takes the default count, lowered if needed until the rows fit the
 * array; an explicit count whose rows (rx_match_long_workspace) exceed 16 MiB
 * fails with RX_ETOOBIG.  Calls that overlap on one GPU share the array and
 * race: serialise them (one stream, or events).  Other errors as rx_match_long. */
int rx_match_long_noalloc(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int32_t chunks,
                          uint8_t* d_out, void* stream);

/* The paper's own GPU machine (§8, on the process translation of §7): every
 * node of d[] is a process owned by one thread of a workgroup; stamp vectors
 * c and n (in LDS) hold which processes have a message in the current macro
 * step and which leaves moved on the byte; rounds of simulation run until
 * none sends a new message, then c and n swap.  One persistent launch, one
 * workgroup per string, barriers inside the kernel; the same results as
 * rx_match (the lockstep machine it realises), without the precomputed
 * evolution tables.  Kept for comparison: its rounds per byte grow with the
 * longest chain of messages, not with the input.
 *
 * rx_program_node_image writes the device image this machine reads: 16
 * bytes of header (m, number of classes), 16 bytes per node of d[] (kind |
 * label << 8, c0, c1, cont) and 32 bytes per class.  *len = its size; buf may
 * be NULL to query it; a buffer below *len gives RX_EINVAL.  The caller copies
 * it to device memory it owns and passes it as d_image, unchanged, for this
 * program only.
 * Errors: RX_EINVAL (NULL arguments, short buffer). */
int rx_program_node_image(const rx_program* prog, void* buf, size_t cap, size_t* len);

/* Strings as in rx_match (d_bytes, d_offsets[n + 1]); d_out: caller-owned
 * device uint8[n], 0 or 1 per string.  Reads only d_image, not the uploaded
 * tables, so rx_program_upload is not needed.  Asynchronous on stream;
 * allocates nothing.
 * Errors: RX_EINVAL (NULL buffers, n < 0), RX_ETOOBIG (more than 8191 nodes:
 * two 8-byte stamps per node in LDS), RX_EHIP. */
int rx_match_nodes(const rx_program* prog, const void* d_image, const uint8_t* d_bytes, const int64_t* d_offsets,
                   int64_t n, uint8_t* d_out, void* stream);

/* rx_match with an explicit kernel variant and launch shape (the autotuner's
 * entry point).  Every variant returns the same bits (Thm. 7.2: the parallel
 * schedule does not change the result). */
int rx_match_ex(const rx_program* prog, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t n,
                uint8_t* d_out, const rx_launch* launch, void* stream);

/*
 * Fixed-length strings: string i is d_bytes[i * length .. (i + 1) * length).
 * No offsets array is read.  With a run-time compiled bit-sliced circuit
 * (rx_program_jit), a 16-byte aligned d_bytes and length a multiple of 16,
 * the sliced kernel runs (one lane advances 32 strings per instruction);
 * otherwise the table-form kernels run.  Same results either way.
 * Errors: RX_EINVAL, RX_ENOTUPLOADED, RX_EHIP.
 */
int rx_match_fixed(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int64_t n, uint8_t* d_out,
                   void* stream);

/* rx_match_fixed with an explicit variant and launch shape (RX_VARIANT_SLICED
 * requires rx_program_jit, 16-byte alignment and length % 16 == 0;
 * RX_VARIANT_CHUNKS requires rx_program_jit and a circuit of at most two state
 * words, else RX_EINVAL).  With RX_VARIANT_AUTO such a circuit runs
 * chunk-parallel when length >= 32768 or n <= 4096. */
int rx_match_fixed_ex(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int64_t n, uint8_t* d_out,
                      const rx_launch* launch, void* stream);

/*
 * Generates the bit-sliced node circuit of the program (the per-node
 * processes of Section 7 evaluated as boolean signals: one 32-bit word per
 * node carries 32 strings) and compiles it with hiprtc.  arch: a gfx target
 * such as "gfx950", or NULL for the current device (then the code object is
 * also loaded, ready for rx_match_fixed).  Compiling for an explicit arch
 * without a device only checks that the generated source builds.
 * Programs whose circuit keeps more than 160 leaf states are refused with
 * RX_ETOOBIG (they would not fit in registers); the table-form kernels run
 * them.  When the code object is loaded, every kernel kept is run once on a
 * seeded batch and checked against the table step (rx_program_jit_selfcheck):
 * the call then allocates about 1.1 MB of device memory for that batch, frees
 * it, and waits for the check to finish (synchronous; not for capture).
 * Errors: RX_EJIT (message holds the compiler log, or the LDS-staged kernel
 * disagreed with the table step), RX_ETOOBIG, RX_EHIP.
 */
int rx_program_jit(rx_program* prog, const char* arch);

/* Copies the generated circuit source (NUL-terminated) into buf[0 .. cap) and
 * sets *len to its length without the NUL; buf may be NULL to query *len. */
int rx_program_jit_source(const rx_program* prog, char* buf, size_t cap, size_t* len);

/* ready: 1 when a loaded sliced kernel exists; state_words: 32-bit words of
 * live thread state per lane; ops: bitwise operations per byte step before
 * the device compiler's own simplification. */
int rx_program_jit_stats(const rx_program* prog, int32_t* ready, int32_t* state_words, int32_t* ops);

/* Which staging modes of the sliced kernel (rx_launch.unroll) run as
 * themselves for this program: staged[u] = 1 for mode u in 1..5 when its
 * kernel was kept, 0 when it was dropped (the device compiler spilled its
 * registers) and mode 2 runs in its place; staged[2] = 1 whenever the program
 * is compiled; staged[0] = the mode that unroll = 0 selects.  All zero before
 * rx_program_jit, or where the program has no loaded kernel.  staged[5] = 2
 * when mode 5 runs its form with single-dword transposer reads (the
 * pair-read form spilled).  staged[6] describes the earliest-accept form of
 * the mode-5 kernel that rx_match_first_fixed runs: 1 pair reads, 2
 * single-dword reads, 0 dropped (the table-form kernels run instead).
 * Errors: RX_EINVAL (NULL arguments). */
int rx_program_jit_staging(const rx_program* prog, int32_t staged[7]);

/* The static check behind the register-staged sliced kernels (staging modes
 * 1, 3, 4, 5 and the earliest-accept form).  Those kernels keep loads in
 * flight in accumulation registers written by inline assembly, which the
 * device compiler takes as present at once; rx_program_jit disassembles the
 * generated code object and keeps such a kernel only if no instruction other
 * than its own 16-byte global loads and 16-byte LDS writes names an
 * accumulation register (so nothing copies, spills or moves one before its
 * load lands).  *ran = 1 when the check ran (0: the disassembler was not
 * available, and every staged kernel is dropped); violations[k] = the number
 * of offending instructions in staged kernel k (-1: not checked) for k = 0..6
 * in the order mode 1, mode 3, mode 4, mode 5 (pair reads), mode 5
 * (single-dword reads), earliest accept (pair reads), earliest accept
 * (single-dword reads); violations[7] is unused; *dropped has bit k set when
 * kernel k was dropped by the check (it never runs; the staging report above
 * shows what runs instead).  Errors: RX_EINVAL (NULL arguments). */
int rx_program_jit_guard(const rx_program* prog, int32_t* ran, int32_t violations[8], int32_t* dropped);

/* The run-time check rx_program_jit makes on a device (after the static
 * check): every kept bit-sliced kernel matches a seeded batch (4,096 strings
 * of 256 bytes that walk the automaton, mostly through bytes a live leaf's
 * label holds) and its bits are compared with the table step of Def. 5.1
 * computed on the host (accept bits; first accepting prefixes for the
 * earliest-accept kernels of non-nullable programs).  *ran = 1 when the check
 * ran (0 before rx_program_jit or when the circuit was only compiled);
 * *dropped has bit k set when staged kernel k (the order of
 * rx_program_jit_guard) gave other bits and was dropped (the staging report
 * shows what runs instead).  The LDS-staged kernel is checked too; if it
 * disagrees, rx_program_jit fails with RX_EJIT.  Errors: RX_EINVAL (NULL
 * arguments). */
int rx_program_jit_selfcheck(const rx_program* prog, int32_t* ran, int32_t* dropped);

/* Generates and compiles the plane-form circuits of a list of programs, for
 * rx_match_multi with RX_FORM_PLANES on that list (same programs, same
 * order): one module holding every program's circuit (the per-node processes
 * of §7 as boolean signals over 32 strings per word, fed precomputed bit
 * planes), loaded on the current device and kept until the process ends.
 * Repeated calls for a list already loaded return at once.  arch as for
 * rx_program_jit (without a device the source is only compiled).  Programs
 * keep their leaf states in registers where they fit; the device compiler
 * spills the rest (*spill_bytes, may be NULL: private bytes per lane, 0 when
 * everything fits).  Errors: RX_EINVAL, RX_EJIT, RX_ETOOBIG (a program above
 * 1024 state words or more than 64 programs), RX_EHIP. */
int rx_match_multi_prepare(const rx_program* const* progs, int32_t n_progs, const char* arch,
                           int32_t* spill_bytes);

/* The plane-form source generated for the one-program list {prog}, as
 * rx_program_jit_source. */
int rx_program_jit_planes_source(const rx_program* prog, char* buf, size_t cap, size_t* len);

/* The same check on any code object (an AMDGPU ELF of len bytes, owned by the
 * caller) for the function `kernel` compiled for `arch` (e.g. "gfx950"):
 * *violations = instructions that name an accumulation register other than
 * 16-byte global loads and 16-byte LDS writes.  Returns RX_OK when the check
 * ran (the message of rx_last_error then names the first offending
 * instruction, if any); RX_EINVAL when it could not (no disassembler, no such
 * function, or no staging instruction recognised). */
int rx_isa_check_staging(const void* code, size_t len, const char* arch, const char* kernel, int32_t* violations);

/* Length bucketing and launch shape of rx_match_multi; zero fields mean default. */
typedef struct {
    int32_t n_edges;    /* bucket edges in use (0 = default ladder 8, 16, 32, ..., 4096) */
    int32_t edges[15];  /* ascending; bucket b holds lengths in (edges[b-1], edges[b]], the last one the rest */
    int32_t block;      /* strings per work item = threads per workgroup: 64, 128 or 256 (default 256) */
    int32_t grid;       /* persistent workgroups (default 4 per compute unit) */
    int32_t form;       /* RX_FORM_TABLE (0, default) or RX_FORM_PLANES (see rx_match_multi) */
    int32_t graph;      /* 1: replay the call's launches from a captured HIP graph (see rx_match_multi) */
    int64_t max_bytes;  /* RX_FORM_PLANES: at least the total bytes of all strings (e.g. the size of the
                           bytes buffer); sizes the workspace */
} rx_multi_config;

enum { RX_FORM_TABLE = 0, RX_FORM_PLANES = 1 };

/* Device workspace rx_match_multi needs for n strings and n_progs programs
 * (bytes), or a negative RX_E* code.  For RX_FORM_PLANES it grows with
 * cfg->max_bytes: about 9/8 of it for the bit planes plus 4 bytes per string. */
int64_t rx_match_multi_workspace(int64_t n, int32_t n_progs, const rx_multi_config* cfg);

/*
 * Batched matching: every string against every program in one persistent
 * launch (the generic lockstep machine of Def. 5.3 per (program, string)).
 * Strings are bucketed by length on the device; work items of up to `block`
 * strings of one bucket against one program are generated on the device,
 * longest bucket first, and pulled by a persistent kernel from an atomic
 * queue.  d_out is n_progs x n bytes, row p for program p.  d_work is caller
 * memory of at least rx_match_multi_workspace(...) bytes, 256-byte aligned; its
 * contents are scratch (cleared by the call's own kernels, never by a memset).
 * Programs must be uploaded, hold sets of at most 16 words, and number at
 * most 64.  Allocates nothing; asynchronous on `stream`.  Results do not
 * depend on the bucketing or launch shape.
 * Errors: RX_EINVAL, RX_ETOOBIG, RX_ENOTUPLOADED, RX_EHIP.
 */
/*
 * RX_FORM_PLANES (the bit-sliced circuit for strings of any length, §7):
 * strings are counting-sorted by length on the device (lengths below 8191
 * exactly; longer strings run in table form), cut into slabs of 2048
 * consecutive sorted strings, and every slab's bytes are gathered and
 * transposed once into bit planes (32 strings per word, plus one word per
 * position marking the strings that still have bytes).  Each program's
 * plane-form circuit then runs over all slabs -- one launch, one wavefront per
 * (program, slab), longest slabs first -- and keeps each string's accept bit
 * as of its last byte.  The list must have been prepared on the current
 * device (rx_match_multi_prepare);
 * cfg->max_bytes must be at least the total length of the strings (with a
 * smaller bound the slabs are skipped and their results are unspecified; no
 * memory outside the workspace is touched).
 *
 * cfg->graph = 1 (either form): the call's launch sequence is recorded once
 * by stream capture on a library stream of the current device, instantiated
 * as a HIP graph and replayed on `stream`; a later call with the same programs
 * and launch shape replays it, or updates it in place when only pointers and
 * sizes changed (waiting on the host for that graph's previous replay first),
 * else instantiates a new one.  Up to 8 graphs are kept per device, least
 * recently used dropped first.  Instantiation allocates host memory; results
 * equal those of the direct launches.  `stream` must not itself be capturing
 * (under the caller's own capture use graph = 0: the direct launches are then
 * what is captured).  Graph calls on one device are serialised by a lock on
 * the host; calls sharing a workspace race on the device as direct calls do.
 */
int rx_match_multi(const rx_program* const* progs, int32_t n_progs, const uint8_t* d_bytes,
                   const int64_t* d_offsets, int64_t n, uint8_t* d_out, void* d_work, size_t work_bytes,
                   const rx_multi_config* cfg, void* stream);

/* Graph use of rx_match_multi since the process started (all devices):
 * counts[0] replays as recorded, counts[1] in-place updates, counts[2]
 * instantiations.  Errors: RX_EINVAL (NULL). */
int rx_multi_graph_counts(int64_t counts[3]);

/*
 * Autotuner for rx_match / rx_match_fixed: successive halving over the kernel
 * variants (bit-sliced circuit when compiled, one lane per string, one
 * wavefront per string) and their workgroup and grid sizes, timed with HIP
 * events on `stream`.  d_offsets NULL means fixed-length strings of `length`
 * bytes (rx_match_fixed), otherwise offsets (rx_match; length ignored).
 * d_out receives the results (n bytes).  Every candidate must return the same
 * bits as the first (the parallel schedule does not change the result,
 * Thm. 7.2); a disagreement fails with RX_EINVAL.  budget_runs bounds the
 * timed launches.  Synchronises `stream`.  *best is the fastest launch shape,
 * *best_ms its mean device time, *n_candidates the candidates tried.
 */
int rx_autotune(const rx_program* prog, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t length, int64_t n,
                uint8_t* d_out, int32_t budget_runs, rx_launch* best, double* best_ms, int32_t* n_candidates,
                void* stream);

/* Autotuner for rx_match_multi: bucket ladders (powers of two, a finer
 * geometric ladder, a coarse one) x workgroup size x grid, same rules as
 * rx_autotune.  d_work must hold rx_match_multi_workspace(n, n_progs, cfg)
 * bytes for cfg = {15 edges, block 64} (the largest candidate). */
int rx_autotune_multi(const rx_program* const* progs, int32_t n_progs, const uint8_t* d_bytes,
                      const int64_t* d_offsets, int64_t n, uint8_t* d_out, void* d_work, size_t work_bytes,
                      int32_t budget_runs, rx_multi_config* best, double* best_ms, int32_t* n_candidates,
                      void* stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of match requests.
 *
 * A server owns a fixed device footprint, allocated once by rx_server_create:
 * `slots` step buffers (strings, offsets, work items, results) plus an arena of
 * `program_slots` resident program tables (64 KiB each).  That footprint must
 * fit `hbm_budget`.  Clients submit requests from any thread; a scheduler
 * thread admits pending requests into the next free step while they fit its
 * capacity, so requests that arrive while steps run join the next step and
 * steps on different slots overlap on the device.  Each step is one launch of
 * the batched item kernel framed by host<->device copies, replayed as a
 * hipGraph when use_graph is set.  Programs are cached by their AST bytes,
 * classes and flags.  A request's bits do not depend on what it was batched
 * with.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t hbm_budget;     /* device bytes the server may hold (default 2 GiB) */
    int64_t step_bytes;     /* string bytes per step (default 64 MiB); larger requests are refused */
    int64_t step_strings;   /* strings per step (default 262144); larger requests are refused */
    int32_t step_requests;  /* requests per step (default 512) */
    int32_t slots;          /* steps in flight (default 2, at most 8) */
    int32_t use_graph;      /* 1: replay each slot's step as a hipGraph with updated node parameters */
    int32_t block;          /* strings per work item: 64, 128 or 256 (default 256) */
    int32_t grid;           /* persistent workgroups per step (default 4 per compute unit) */
    int32_t program_slots;  /* resident programs (default 1024; at least `slots`).  One step uses at most
                               min(64, program_slots / slots) distinct programs, so the steps in flight
                               never hold every resident slot */
} rx_server_config;

typedef struct {
    int64_t submitted, completed, rejected, queued, max_queue;
    int64_t steps, graph_steps, strings, bytes;
    int64_t cache_hits, cache_misses, cache_evictions;
    double p50_us, p99_us, mean_us, max_us; /* latency: submit -> results on the host */
    double wall_s;                          /* first submit -> last completion */
    double pack_ms;                         /* scheduler time assembling and launching steps */
    double device_ms;                       /* device time of steps (copies in, kernel, copy out) */
} rx_server_counters;

typedef struct rx_server rx_server;

/* Creates a server and its scheduler thread on the current device.  cfg may
 * be NULL (defaults).  Errors: RX_EINVAL, RX_ETOOBIG (footprint above the
 * budget), RX_EHIP. */
int rx_server_create(const rx_server_config* cfg, rx_server** out);

/* Drains pending requests, stops the scheduler and frees everything.  After a
 * failed step no further step runs: requests still waiting fail with that
 * step's status, so every rx_server_wait returns. */
void rx_server_destroy(rx_server* srv);

/* Submits one request: the expression (as for rx_compile) and n host strings
 * (host_bytes[host_offsets[i] .. host_offsets[i+1])), copied before the call
 * returns.  *req_id identifies it for rx_server_wait.  Never blocks on the
 * device.  Errors: RX_EINVAL (malformed AST or batch), RX_ETOOBIG (above one
 * step's capacity or more than 511 leaves), RX_EHIP (the server failed). */
int rx_server_submit(rx_server* srv, const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes,
                     int32_t n_classes, uint32_t flags, const uint8_t* host_bytes, const int64_t* host_offsets,
                     int64_t n, int64_t* req_id);

/* Waits for a request (timeout_us < 0: forever), copies its n result bytes
 * into host_out (may be NULL) and forgets it.  Errors: RX_EINVAL (unknown id),
 * RX_ETIMEOUT (still running; the request stays waitable), RX_EHIP. */
int rx_server_wait(rx_server* srv, int64_t req_id, uint8_t* host_out, int64_t timeout_us);

/* Counters and latency percentiles since creation or the last reset. */
int rx_server_stats(rx_server* srv, rx_server_counters* out);
int rx_server_reset_stats(rx_server* srv);

/* The plain per-request path the server is measured against: compile, upload,
 * copy the strings in, one rx_match launch, copy the bits out, synchronise,
 * free -- all inside the call.  Same arguments as rx_server_submit. */
int rx_plain_match(const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes, int32_t n_classes,
                   uint32_t flags, const uint8_t* host_bytes, const int64_t* host_offsets, int64_t n,
                   uint8_t* host_out);

/* The same plain path with its resources made once: rx_plain_create makes one
 * stream and device buffers for requests of at most max_bytes string bytes and
 * max_strings strings (plus a 1 MiB table buffer); rx_plain_run then does, per
 * request, exactly compile, upload, copy in, one rx_match launch, copy out,
 * synchronise -- no allocation on the device and no stream creation.  Same
 * request arguments as rx_server_submit.  Errors: RX_EINVAL, RX_ETOOBIG (above
 * the context's capacity), RX_EHIP.  A context is used by one thread at a time. */
typedef struct rx_plain rx_plain;
int rx_plain_create(int64_t max_bytes, int64_t max_strings, rx_plain** out);
int rx_plain_run(rx_plain* ctx, const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes,
                 int32_t n_classes, uint32_t flags, const uint8_t* host_bytes, const int64_t* host_offsets, int64_t n,
                 uint8_t* host_out);
void rx_plain_destroy(rx_plain* ctx);

/* Thread-local message of the last failed call on this host thread. */
const char* rx_last_error(void);

/* 1 when entry points and server steps are wrapped in roctx ranges: the
 * environment variable RX_ROCTX is set (not "0") when the library first
 * looks, and a roctx library (librocprofiler-sdk-roctx or libroctx64) could
 * be opened; then `rocprofv3 --marker-trace` shows each range ("rx_match",
 * "rx_server.step", ...) around its kernels.  0 otherwise (ranges cost one
 * branch).  Never fails. */
int rx_trace_enabled(void);

/* Measurement only: a plain coalesced device-to-device copy of `bytes`
 * (a multiple of 16; both buffers 16-byte aligned) on `stream`.  It gives the
 * practical streaming ceiling of the memory system and calibrates hardware
 * byte counters against a kernel whose traffic is known exactly. */
int rx_stream_copy(void* d_dst, const void* d_src, int64_t bytes, void* stream);

/* Library version string. */
const char* rx_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RX_H */
