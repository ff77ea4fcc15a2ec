// Internal declarations shared by the host compiler, the C interface and the
// kernel launchers of the lockstep matcher.
#pragma once

#include <array>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "rx.h"

namespace rx {

constexpr int kMaxLeaves = 4095;        // accept bit is rank L, so sets hold <= 4096 bits
constexpr int kMaxNodes = 1 << 20;
constexpr int kLaneMaxWords = 16;       // one-lane-per-string kernel limit (L <= 511)
constexpr int kWaveMaxWords = 128;      // wavefront kernel limit: lane j owns words j and j+64
constexpr int kJitMaxState = 160;       // sliced circuit: leaf state words kept in registers
constexpr int kJitPlanesMaxState = 1024; // plane-form circuit: the device compiler spills what registers cannot hold
constexpr int kNodesMaxNodes = 8191;    // node-per-thread machine: two stamp vectors of m + 1 in LDS

// Device table layout (all offsets in bytes from the start of the uploaded
// buffer, each section 256-byte aligned).
struct DevLayout {
    int64_t first = 0;      // words u32
    int64_t follow = 0;     // L * words u32
    int64_t bytemask = 0;   // 256 * words u32
    int64_t chunks = 0;     // n_chunks * 256 * words u32 (large programs only)
    int32_t n_chunks = 0;
    int64_t total = 0;
};

struct Program {
    // node array d[] (the heap), breadth-first from the root at index 0
    std::vector<int32_t> kind, c0, c1, label, cont, depth;
    std::vector<std::array<uint64_t, 4>> classes;  // caller's classes + wrapper's any-byte class
    int32_t m = 0, n_tree = 0;
    uint32_t flags = 0;
    int32_t L = 0, W = 0, height = 0;
    bool nullable = false, suffix_any = false;
    std::vector<int32_t> leaf_node;  // rank -> node
    std::vector<int32_t> leaf_rank;  // node -> rank, -1 for internal nodes
    // evolution tables (Def. 5.1), 32-bit words
    std::vector<uint32_t> first, follow, bytemask;
    DevLayout layout;
    std::vector<uint8_t> blob;       // host image of the device tables
    // device state
    void* dev = nullptr;
    int dev_id = -1;
    // run-time generated kernel for the bit-sliced circuit (may be null)
    void* jit = nullptr;
    // identity for module caches: unique per compiled program in this process
    uint64_t uid = 0;
};

// batched matching (rx_multi.hip)
constexpr int kMaxItemProgs = 64;   // programs per batched launch (descriptors travel as kernel arguments)
constexpr int kMaxBuckets = 16;     // length bucket edges

struct ProgDesc {                   // device tables of one program
    const uint32_t* first;
    const uint32_t* follow;
    const uint32_t* bytemask;
    int32_t L, W, suffix_any, pad;
};

struct WorkItem {                   // up to `block` strings against one program
    int32_t prog;                   // index into the launch's program descriptors
    int32_t count;                  // strings in the item
    int64_t line0;                  // first string (or first entry of the id list)
    int64_t out0;                   // result of string s goes to out[out0 + s]
};

struct MultiArgs {
    ProgDesc progs[kMaxItemProgs];
    int32_t n_progs;
    int32_t edges[kMaxBuckets];
    int32_t n_edges;
    int32_t block_lines;
    int32_t grid;
    const uint8_t* bytes;
    const int64_t* offsets;
    int64_t n;
    uint8_t* out;
    void* work;
    void* stream;
};

struct ItemsArgs {
    ProgDesc progs[kMaxItemProgs];
    int32_t n_progs;
    int32_t block, grid;
    const uint8_t* bytes;
    const int64_t* offsets;
    const WorkItem* items;
    const int32_t* n_items;
    int32_t* head;
    uint8_t* out;
    void* stream;
};

struct Copy {
    void* dst;
    const void* src;
    size_t bytes;
};
struct StepDesc {          // one serving step
    Copy h2d[3];           // strings, offsets, work items (with the queue header)
    ItemsArgs items;       // item kernel arguments
    Copy d2h;              // results
};
struct StepGraph;
int step_launch_direct(const StepDesc& d, void* stream);
int step_graph_launch(StepGraph** g, const StepDesc& d, void* stream);
void step_graph_destroy(StepGraph* g);

int64_t multi_workspace_bytes(int64_t n, int32_t n_progs, int32_t n_buckets, int32_t block_lines);

// plane form of batched matching (rx_multi.hip): exact-length sort, slabs of
// 2048 strings, bit planes gathered once, every program's circuit over them
constexpr int kSortBins = 8192;      // lengths 0 .. 8190 sort exactly; longer strings run in table form
struct PlaneMultiArgs {
    const Program* progs[kMaxItemProgs];   // each with a loaded plane-form circuit
    ProgDesc descs[kMaxItemProgs];         // device tables (strings too long for a slab)
    int32_t n_progs;
    int32_t block_lines;                   // table-form item size
    int32_t item_grid;
    const uint8_t* bytes;
    const int64_t* offsets;
    int64_t n;
    int64_t max_bytes;                     // upper bound of the total string bytes
    uint8_t* out;
    void* work;
    void* stream;
};
int64_t plane_max_slabs(int64_t n);
int64_t plane_tick_cap(int64_t n, int64_t max_bytes);
int64_t plane_workspace_bytes(int64_t n, int64_t max_bytes, int32_t n_progs, int32_t block_lines);
int launch_planes_multi(const PlaneMultiArgs& m);
int launch_multi(const MultiArgs& m);
int launch_items(const ItemsArgs& m);

// graph replay of a launch sequence (rx_graph.cpp): `record` issues the
// sequence on the stream it is given (a capture stream); calls with equal
// `full` keys replay the instantiated graph, calls with another `full` but the
// same `topo` update it in place.  *how (may be NULL): 0 replayed, 1 updated,
// 2 instantiated.  Returns a HIP error code or the recorder's own.
int graph_replay(const std::string& topo, const std::string& full, const std::function<int(void*)>& record,
                 void* stream, int* how);
void graph_counts(int64_t out[3]);
void graph_key_add(std::string& key, const void* p, size_t n);
template <class T>
void graph_key(std::string& key, const T& v) { graph_key_add(key, &v, sizeof(v)); }

// autotuner (rx_autotune.cpp)
int autotune_single(const Program* P, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t length, int64_t n,
                    uint8_t* d_out, int budget_runs, rx_launch* best, double* best_ms, int* n_cands, void* stream);
int autotune_multi(const rx_program* const* progs, int32_t n_progs, const uint8_t* d_bytes, const int64_t* d_offsets,
                   int64_t n, uint8_t* d_out, void* d_work, size_t work_bytes, int budget_runs, rx_multi_config* best,
                   double* best_ms, int* n_cands, void* stream);

// profiler ranges (rx_trace.cpp): a roctx range for the scope, when RX_ROCTX is set
class TraceRange {
public:
    explicit TraceRange(const char* name);
    ~TraceRange();
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
private:
    bool on_;
};
bool trace_enabled();

// error reporting (thread-local message)
int fail(int code, const std::string& msg);
void clear_error();
const char* last_error_cstr();

// host compiler (rx_compile.cpp)
int compile(const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes,
            int32_t n_classes, uint32_t flags, Program** out);

// device launchers (rx_kernels.hip); return a hipError_t as int
struct LaunchArgs {
    const uint32_t* first;
    const uint32_t* follow;
    const uint32_t* bytemask;
    const uint32_t* chunks;  // chunk unions, or NULL
    int32_t L, W;
    int32_t suffix_any;
    const uint8_t* bytes;
    const int64_t* offsets;  // NULL: fixed-length strings, string i at bytes + i * stride
    int64_t stride;
    int64_t n;
    uint8_t* out;
    int32_t block, grid, unroll;
    void* stream;
    int64_t* first_pos = nullptr;   // rx_match_first: earliest accepting prefix per string (out unused)
    // rx_match_long, first pass: n rows of a chunk-parallel run (see KArgs in rx_kernels.hip)
    uint32_t* rows_out = nullptr;
    int64_t rows_len = 0, rows_cl = 0;
    int32_t rows_per_chunk = 0;
    // rx_match's layout slot (see launch_layout_check): nothing runs when the
    // bit-sliced kernel took the strings
    const int64_t* skip = nullptr;
    int64_t skip_id = 0;
};
int launch_lane(const LaunchArgs& a);
// Equal-length consecutive strings for rx_match (rx_kernels.hip): the slot of
// call `id` in a static per-device array of kLayoutSlots slots of four int64
// {id, length, first offset, flaw}; launch_layout_check fills it on `stream`
// (flaw 0: string i is bytes[first + i * length, + length), length a multiple
// of 16 up to kLayoutMaxLength and the first byte 16-byte aligned).
constexpr int64_t kLayoutSlots = 4096;
constexpr int64_t kLayoutMaxLength = (int64_t)1 << 26;
constexpr int64_t kLayoutMinStrings = 16384;   // fewer strings: the table form alone
int layout_slot(int64_t id, int64_t** slot);
int launch_layout_check(const int64_t* offsets, int64_t n, const uint8_t* bytes, int64_t* slot, int64_t id,
                        void* stream);
// bit-sliced node circuit (rx_jit.cpp)
// The chunk-parallel kernel of a compiled circuit of at most two state words
// (one wavefront per string, 2,048 chunks, each run from every state; the
// chunks' maps compose in order).
bool jit_chunks_ready(const Program* P);
// One long string as circuit chunks (circuits of at most kLongChunkMaxState
// words: the chunk maps are affine, NS + 1 runs each): the workspace it needs
// (-1: no such kernel for this program) and the launch (segments, then their
// composition, on `stream`).
constexpr int kLongChunkMaxState = 31;   // a state as bits 0 .. NS - 1 of a word, the accept bit 31
int64_t long_chunk_work_bytes(const Program* P, int64_t length);
int launch_long_chunks(const Program* P, const uint8_t* bytes, int64_t length, void* work, uint8_t* out,
                       void* stream);
int launch_sliced_chunks(const Program* P, const uint8_t* bytes, int64_t length, int64_t n, uint8_t* out,
                         void* stream);
// (suffix_slot: the state word of a searched program's suffix leaf, or -1)
std::string jit_step_source(const Program& P, int* n_state, int* n_ops, int* suffix_slot = nullptr);
std::string jit_full_source(const Program& P, int* n_state, int* n_ops);
int jit_compile(Program* P, const char* arch);
void jit_free(Program* P);
bool jit_ready(const Program* P, int* n_state, int* n_ops);
// rx_match's equal-length strings through the skewed kernel (the layout slot
// of call id decides whether it runs)
bool jit_offsets_ready(const Program* P);
int launch_sliced_offsets(const Program* P, const uint8_t* bytes, const int64_t* slot, int64_t id, int64_t n,
                          uint8_t* out, void* stream);
// staged[u] for staging modes u = 0..5 (see rx_program_jit_staging).
void jit_staging(const Program* P, int32_t staged[7]);
// Plane-form circuits (rx_jit.cpp): one module per list of programs.
// spec_lds (may be NULL): LDS bytes of the kernel that splits long slabs
std::string jit_multi_planes_source(const Program* const* progs, int n, int* max_state, int* spec_lds);
constexpr int kSpecWaves = 8;                    // wavefronts per long slab of a searched program
constexpr int64_t kSpecLdsBudget = 140 * 1024;   // the copies of a split slab's states
constexpr int kSpecCheckpoints = 4;              // after 4, 8, 16, 32 ticks of a segment
std::string jit_planes_source(const Program& P, int* n_state);   // the list of one program
// Compiles and loads (once per device and list) the module of `progs`.
int jit_prepare_planes(const Program* const* progs, int n, const char* arch, int* spill_bytes);
bool jit_planes_prepared(const Program* const* progs, int n);
// One wavefront per (program, slab) for the slabs of rank r_lo <= r < r_hi
// (rank 0 = the longest), or with split two per (program, slab), the second
// starting a searched program's slab of 16 ticks or more in the middle (see
// rx_run_slab_spec); returns -1 when the list was not prepared.
int launch_planes_circuits(const Program* const* progs, int n, const uint32_t* planes, const int64_t* slab_tick,
                           const int64_t* info, uint32_t* res, int64_t max_slabs, int64_t r_lo, int64_t r_hi,
                           bool split, void* stream);
// Static check of a register-staged kernel in a code object (rx_isa_guard.cpp):
// *violations = instructions not written by the kernel itself that name an
// accumulation register.  Returns 0 when the check ran, < 0 when it could not.
int isa_check_agpr_staging(const std::vector<char>& code, const std::string& arch, const char* kernel,
                           int* violations, std::string* example);
// The check's outcome for a program's kernels (see rx_program_jit_guard).
void jit_guard(const Program* P, int32_t* ran, int32_t violations[8], int32_t* dropped);
void jit_selfcheck_report(const Program* P, int32_t* ran, int32_t* dropped);
// The staging mode that unroll = 0 selects.
int jit_default_staging(const Program* P);
// The skewed kernel's earliest-accept form (kept unless it spills) and its launch.
bool jit_first_ready(const Program* P);
int launch_sliced_first(const Program* P, const uint8_t* bytes, int64_t length, int64_t n, int64_t* first,
                        void* stream);
// The node-per-thread machine (rx_nodes.hip): host image of d[] and its launch.
void node_image(const Program* P, std::vector<uint8_t>& img);
int launch_nodes(const void* image, int32_t m, const uint8_t* bytes, const int64_t* offsets, int64_t stride, int64_t n,
                 uint8_t* out, void* stream);
// The allocation-free chunk-parallel entry point's workspace: a static device
// array in rx_kernels.hip (one per GPU, held until the process ends).
constexpr size_t kLongScratchBytes = (size_t)16 << 20;
// Its device address on the current device (looked up once per device).
int long_scratch(void** ptr);
// first[i] = value for i < n (a fill kernel, no memset)
int launch_fill_i64(int64_t* first, int64_t n, int64_t value, void* stream);
int launch_sliced_fixed(const Program* P, const uint8_t* bytes, int64_t length, int64_t n, uint8_t* out,
                        int burst, void* stream);
int launch_wave(const LaunchArgs& a);
// rx_match_long, second pass: one workgroup applies the chunks' relations in order
int launch_compose(const uint32_t* rows, int64_t chunks, int32_t rpc, int32_t W, int32_t L, int32_t suffix_any,
                   uint8_t* out, void* stream);
int launch_compose_first(const uint32_t* rows, const int64_t* fp, int64_t chunks, int64_t cl, int32_t rpc,
                         int32_t W, int64_t* out, void* stream);
const char* hip_error_string(int err);
int launch_stream_copy(void* dst, const void* src, int64_t bytes, void* stream);
int hip_current_device(int* dev);
int hip_memcpy_h2d_async(void* dst, const void* src, size_t n, void* stream);
int hip_cu_count(int* cus);

}  // namespace rx
