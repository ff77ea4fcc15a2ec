// C interface of the lockstep matcher: program lifetime, upload and launch
// selection.  Every entry point catches everything and reports through a
// thread-local message.
#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <string>

#include "rx_internal.h"

namespace rx {

namespace {
thread_local std::string g_error;
}

const char* last_error_cstr() { return g_error.c_str(); }

int fail(int code, const std::string& msg) {
    g_error = msg;
    return code;
}

void clear_error() { g_error.clear(); }

static int hip_fail(int err, const char* what) {
    return fail(RX_EHIP, std::string(what) + ": " + hip_error_string(err));
}

int make_launch_args(const Program* P, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t n,
                     uint8_t* d_out, void* stream, LaunchArgs* a) {
    if (!P) return fail(RX_EINVAL, "program is NULL");
    if (n < 0) return fail(RX_EINVAL, "negative string count");
    if (n > 0 && (!d_bytes || !d_offsets || !d_out)) return fail(RX_EINVAL, "NULL device buffer");
    if (!P->dev) return fail(RX_ENOTUPLOADED, "program has not been uploaded (rx_program_upload)");
    const uint8_t* base = static_cast<const uint8_t*>(P->dev);
    a->first = reinterpret_cast<const uint32_t*>(base + P->layout.first);
    a->follow = reinterpret_cast<const uint32_t*>(base + P->layout.follow);
    a->bytemask = reinterpret_cast<const uint32_t*>(base + P->layout.bytemask);
    a->chunks = P->layout.n_chunks ? reinterpret_cast<const uint32_t*>(base + P->layout.chunks) : nullptr;
    a->L = P->L;
    a->W = P->W;
    a->suffix_any = P->suffix_any ? 1 : 0;
    a->bytes = d_bytes;
    a->offsets = d_offsets;
    a->stride = 0;
    a->n = n;
    a->out = d_out;
    a->block = 0;
    a->grid = 0;
    a->unroll = 0;
    a->stream = stream;
    return RX_OK;
}

}  // namespace rx

using namespace rx;

#define RX_GUARD_BEGIN try {
#define RX_GUARD_END                                                          \
    }                                                                         \
    catch (const std::bad_alloc&) {                                           \
        return fail(RX_ENOMEM, "out of host memory");                         \
    }                                                                         \
    catch (const std::exception& e) {                                         \
        return fail(RX_EINVAL, std::string("internal error: ") + e.what());   \
    }                                                                         \
    catch (...) {                                                             \
        return fail(RX_EINVAL, "internal error");                             \
    }

extern "C" {

int rx_compile(const rx_ast_node* ast, int32_t n_ast, int32_t root, const rx_class* classes,
               int32_t n_classes, uint32_t flags, rx_program** out) {
    TraceRange trace_range_("rx_compile");
    RX_GUARD_BEGIN
    if (!out) return fail(RX_EINVAL, "out is NULL");
    *out = nullptr;
    Program* P = nullptr;
    int rc = compile(ast, n_ast, root, classes, n_classes, flags, &P);
    if (rc) return rc;
    // the C handle is an opaque pointer to the library's Program
    *out = reinterpret_cast<rx_program*>(P);
    clear_error();
    return RX_OK;
    RX_GUARD_END
}

void rx_program_free(rx_program* prog) {
    try {
        Program* P = reinterpret_cast<Program*>(prog);
        if (P) jit_free(P);
        delete P;
    } catch (...) {
    }
}

int rx_program_info(const rx_program* prog, rx_info* out) {
    if (!prog || !out) return fail(RX_EINVAL, "NULL argument");
    const Program* P = reinterpret_cast<const Program*>(prog);
    std::memset(out, 0, sizeof(*out));
    out->m = P->m;
    out->n_leaves = P->L;
    out->words = P->W;
    out->nullable = P->nullable;
    out->suffix_any = P->suffix_any;
    out->search = (P->flags & RX_SEARCH) ? 1 : 0;
    out->table_bytes = P->layout.total;
    out->depth = P->height;
    out->n_classes = (int32_t)P->classes.size();
    return RX_OK;
}

int rx_program_nodes(const rx_program* prog, rx_node* out, int32_t cap, int32_t* m) {
    if (!prog) return fail(RX_EINVAL, "program is NULL");
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (m) *m = P->m;
    if (out) {
        const int32_t k = cap < P->m ? cap : P->m;
        for (int32_t i = 0; i < k; ++i) {
            out[i].kind = P->kind[i];
            out[i].c0 = P->c0[i];
            out[i].c1 = P->c1[i];
            out[i].label = P->label[i];
            out[i].cont = P->cont[i];
        }
    }
    return RX_OK;
}

int rx_program_sets(const rx_program* prog, uint32_t* first, uint32_t* follow, uint32_t* bytemask,
                    int32_t* leaf_node) {
    if (!prog) return fail(RX_EINVAL, "program is NULL");
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (first) std::memcpy(first, P->first.data(), 4 * P->first.size());
    if (follow && !P->follow.empty()) std::memcpy(follow, P->follow.data(), 4 * P->follow.size());
    if (bytemask) std::memcpy(bytemask, P->bytemask.data(), 4 * P->bytemask.size());
    if (leaf_node && !P->leaf_node.empty()) std::memcpy(leaf_node, P->leaf_node.data(), 4 * P->leaf_node.size());
    return RX_OK;
}

int rx_program_upload(rx_program* prog, void* d_buf, size_t cap, void* stream) {
    TraceRange trace_range_("rx_program_upload");
    RX_GUARD_BEGIN
    if (!prog || !d_buf) return fail(RX_EINVAL, "NULL argument");
    Program* P = reinterpret_cast<Program*>(prog);
    if ((reinterpret_cast<uintptr_t>(d_buf) & 255) != 0) return fail(RX_EINVAL, "device buffer must be 256-byte aligned");
    if (cap < (size_t)P->layout.total)
        return fail(RX_ETOOBIG, "device buffer holds " + std::to_string(cap) + " bytes; the program needs " +
                                    std::to_string(P->layout.total));
    int dev = -1;
    if (int e = hip_current_device(&dev)) return hip_fail(e, "hipGetDevice");
    if (int e = hip_memcpy_h2d_async(d_buf, P->blob.data(), P->blob.size(), stream)) return hip_fail(e, "hipMemcpyAsync");
    P->dev = d_buf;
    P->dev_id = dev;
    clear_error();
    return RX_OK;
    RX_GUARD_END
}

namespace {
// The table form for a batch: one lane per string while the strings fill the
// machine or the set is small; for few strings and sets of six words or more,
// wavefronts per string (two or more, at least three words each), so the
// set's words are worked in parallel rather than the strings (256 strings in
// one-lane form are four wavefronts).  Measured on 256 strings of 10^4 bytes:
// 7 words 84 -> 68 ms; 3 words 19 ms one lane per string, 46 ms one
// wavefront per string.
int auto_table_variant(const Program* P, int64_t n) {
    if (P->W > kLaneMaxWords) return RX_VARIANT_WAVE;
    if (P->W < 6) return RX_VARIANT_LANE;
    int cus = 0;
    if (hip_cu_count(&cus) || cus <= 0) cus = 256;
    return n <= 16 * (int64_t)cus ? RX_VARIANT_WAVE : RX_VARIANT_LANE;   // at most four wavefronts per SIMD
}
}  // namespace

int rx_match_ex(const rx_program* prog, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t n,
                uint8_t* d_out, const rx_launch* launch, void* stream) {
    TraceRange trace_range_("rx_match_ex");
    RX_GUARD_BEGIN
    LaunchArgs a;
    if (int rc = make_launch_args(reinterpret_cast<const Program*>(prog), d_bytes, d_offsets, n, d_out, stream, &a)) return rc;
    if (n == 0) return RX_OK;
    const Program* P = reinterpret_cast<const Program*>(prog);
    int variant = launch ? launch->variant : RX_VARIANT_AUTO;
    if (launch) {
        if (launch->block < 0 || launch->block > 1024 || (launch->block % 64) != 0)
            return fail(RX_EINVAL, "block must be a multiple of 64 in [64, 1024]");
        if (launch->grid < 0) return fail(RX_EINVAL, "negative grid");
        a.block = launch->block;
        a.grid = launch->grid;
        a.unroll = launch->unroll;
    }
    if (variant == RX_VARIANT_AUTO && n >= kLayoutMinStrings && jit_offsets_ready(P)) {
        // Equal-length consecutive strings go to the bit-sliced kernel: a
        // check on the device fills this call's layout slot, the sliced kernel
        // runs if the slot says so, and the table-form launch below does
        // nothing in that case (and everything otherwise).
        static std::atomic<int64_t> next_id{0};
        const int64_t id = ++next_id;
        int64_t* slot = nullptr;
        if (int e = layout_slot(id, &slot)) return hip_fail(e, "layout slot");
        if (int e = launch_layout_check(d_offsets, n, d_bytes, slot, id, stream)) return hip_fail(e, "layout check");
        if (int e = launch_sliced_offsets(P, d_bytes, slot, id, n, d_out, stream))
            return hip_fail(e, "kernel launch (sliced)");
        a.skip = slot;
        a.skip_id = id;
    }
    if (variant == RX_VARIANT_AUTO) variant = auto_table_variant(P, n);
    int e;
    switch (variant) {
    case RX_VARIANT_LANE:
        if (P->W > kLaneMaxWords) return fail(RX_ETOOBIG, "the lane kernel holds sets of at most 16 words");
        if (a.block > 256) return fail(RX_EINVAL, "the lane kernel runs at most 256 threads per workgroup");
        e = launch_lane(a);
        break;
    case RX_VARIANT_WAVE:
        if (P->W > kWaveMaxWords) return fail(RX_ETOOBIG, "the wavefront kernel holds sets of at most 128 words");
        if (a.unroll != 0 && a.unroll != 1 && a.unroll != 2 && a.unroll != 4 && a.unroll != 8 && a.unroll != 16)
            return fail(RX_EINVAL, "wavefronts per string (unroll) must be 0 (by string count), 1, 2, 4, 8 or 16");
        e = launch_wave(a);
        break;
    default: return fail(RX_EINVAL, "unknown or unavailable kernel variant");
    }
    if (e) return hip_fail(e, "kernel launch");
    return RX_OK;
    RX_GUARD_END
}

int rx_match(const rx_program* prog, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t n,
             uint8_t* d_out, void* stream) {
    TraceRange trace_range_("rx_match");
    return rx_match_ex(prog, d_bytes, d_offsets, n, d_out, nullptr, stream);
}

namespace {
// Chunks of a chunk-parallel run: the requested count, at most 4096 and at most
// one per byte; every chunk holds at least one byte.  By default the count
// balances the rows' time against the composition's (about 1 us per chunk):
// lane rows all run at once, about 0.5 us per byte each, so C ~ sqrt(length / 2);
// wavefront rows share the chip, so fewer chunks: C ~ sqrt(length / 20).
void long_chunks(const Program* P, int64_t length, int32_t chunks, int64_t* C, int64_t* cl) {
    const double per = P->W <= kLaneMaxWords ? 2.0 : 20.0;
    int64_t c = chunks > 0 ? chunks : (int64_t)std::llround(std::sqrt((double)length / per));
    if (c > 4096) c = 4096;
    if (c > length) c = length;
    if (c < 1) c = 1;
    *cl = length > 0 ? (length + c - 1) / c : 0;
    *C = length > 0 ? (length + *cl - 1) / *cl : 1;
}

int64_t long_rows(const Program* P, int64_t C) { return 1 + (C - 1) * (int64_t)(P->L + 1); }

// The rows' sets (u32 words), then, 8-byte aligned, one int64 per row for the
// earliest-accept form.
size_t long_sets_bytes(const Program* P, int64_t C) {
    return ((size_t)long_rows(P, C) * (size_t)P->W * 4 + 7) & ~(size_t)7;
}
size_t long_rows_bytes(const Program* P, int64_t C) { return long_sets_bytes(P, C) + 8 * (size_t)long_rows(P, C); }
}  // namespace

int rx_match_long_workspace(const rx_program* prog, int64_t length, int32_t chunks, size_t* bytes) {
    RX_GUARD_BEGIN
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (!P || !bytes) return fail(RX_EINVAL, "NULL argument");
    if (length < 0 || chunks < 0) return fail(RX_EINVAL, "negative length or chunk count");
    int64_t C, cl;
    long_chunks(P, length, chunks, &C, &cl);
    *bytes = long_rows_bytes(P, C);
    // rx_match_long's circuit form (chunks = 0 with a compiled circuit) needs its segment maps
    const int64_t circuit = chunks == 0 ? long_chunk_work_bytes(P, length) : -1;
    if (circuit > 0 && (size_t)circuit > *bytes) *bytes = (size_t)circuit;
    return RX_OK;
    RX_GUARD_END
}

namespace {
// The two launches of a chunk-parallel run over C chunks of cl bytes, with the
// rows in d_work (long_rows_bytes(P, C) bytes; every row is written before it
// is read, so the workspace needs no clearing).
int match_long_run(const Program* P, const uint8_t* d_bytes, int64_t length, int64_t C, int64_t cl, void* d_work,
                   uint8_t* d_out, void* stream) {
    LaunchArgs a;
    const int64_t rows = long_rows(P, C);
    if (int rc = make_launch_args(P, d_bytes ? d_bytes : static_cast<const uint8_t*>(d_work),
                                  static_cast<const int64_t*>(d_work), rows, d_out, stream, &a))
        return rc;
    a.offsets = nullptr;
    a.out = nullptr;
    a.rows_out = static_cast<uint32_t*>(d_work);
    a.rows_len = length;
    a.rows_cl = cl;
    a.rows_per_chunk = P->L + 1;
    int e = P->W <= kLaneMaxWords ? launch_lane(a) : launch_wave(a);
    if (e) return hip_fail(e, "kernel launch (rows)");
    e = launch_compose(a.rows_out, C, P->L + 1, P->W, P->L, P->suffix_any ? 1 : 0, d_out, stream);
    if (e) return hip_fail(e, "kernel launch (composition)");
    return RX_OK;
}

int check_long_args(const Program* P, const uint8_t* d_bytes, int64_t length, int32_t chunks, const void* d_out) {
    if (!P) return fail(RX_EINVAL, "program is NULL");
    if (length < 0 || chunks < 0) return fail(RX_EINVAL, "negative length or chunk count");
    if (!d_out || (length > 0 && !d_bytes)) return fail(RX_EINVAL, "NULL device buffer");
    if (!P->dev) return fail(RX_ENOTUPLOADED, "program has not been uploaded (rx_program_upload)");
    if (P->W > kWaveMaxWords) return fail(RX_ETOOBIG, "the wavefront kernel holds sets of at most 128 words");
    return RX_OK;
}
}  // namespace

int rx_match_long(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int32_t chunks, void* d_work,
                  size_t work_bytes, uint8_t* d_out, void* stream) {
    TraceRange trace_range_("rx_match_long");
    RX_GUARD_BEGIN
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (int rc = check_long_args(P, d_bytes, length, chunks, d_out)) return rc;
    if (!d_work) return fail(RX_EINVAL, "NULL device buffer");
    // a compiled circuit of at most kLongChunkMaxState words, default chunking:
    // the string as circuit chunks (each an affine map of the state words)
    const int64_t circuit_need = chunks == 0 && length <= (int64_t(1) << 40) ? long_chunk_work_bytes(P, length) : -1;
    if (circuit_need >= 0 && (size_t)circuit_need <= work_bytes) {
        if (int e = launch_long_chunks(P, d_bytes, length, d_work, d_out, stream)) return hip_fail(e, "kernel launch");
        return RX_OK;
    }
    int64_t C, cl;
    long_chunks(P, length, chunks, &C, &cl);
    const size_t need = long_rows_bytes(P, C);
    if (work_bytes < need)
        return fail(RX_EINVAL, "workspace holds " + std::to_string(work_bytes) + " bytes; this run needs " +
                                   std::to_string(need) + " (rx_match_long_workspace)");
    return match_long_run(P, d_bytes, length, C, cl, d_work, d_out, stream);
    RX_GUARD_END
}

int rx_match_long_noalloc(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int32_t chunks,
                          uint8_t* d_out, void* stream) {
    TraceRange trace_range_("rx_match_long_noalloc");
    RX_GUARD_BEGIN
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (int rc = check_long_args(P, d_bytes, length, chunks, d_out)) return rc;
    int64_t C, cl;
    long_chunks(P, length, chunks, &C, &cl);
    if (long_rows_bytes(P, C) > kLongScratchBytes) {
        if (chunks > 0)
            return fail(RX_ETOOBIG, std::to_string(chunks) + " chunks need " + std::to_string(long_rows_bytes(P, C)) +
                                        " bytes of rows; the static workspace holds " +
                                        std::to_string(kLongScratchBytes));
        // the default count, lowered until the rows fit the static workspace
        while (C > 1 && long_rows_bytes(P, C) > kLongScratchBytes) long_chunks(P, length, (int32_t)(C - 1), &C, &cl);
        if (long_rows_bytes(P, C) > kLongScratchBytes)
            return fail(RX_ETOOBIG, "one chunk's rows exceed the static workspace");
    }
    void* work = nullptr;
    if (int e = long_scratch(&work)) return hip_fail(e, "device address of the static workspace");
    return match_long_run(P, d_bytes, length, C, cl, work, d_out, stream);
    RX_GUARD_END
}

int rx_match_first_long(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int32_t chunks, void* d_work,
                        size_t work_bytes, int64_t* d_first, void* stream) {
    TraceRange trace_range_("rx_match_first_long");
    RX_GUARD_BEGIN
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (!P) return fail(RX_EINVAL, "program is NULL");
    if (length < 0 || chunks < 0) return fail(RX_EINVAL, "negative length or chunk count");
    if (!d_first || !d_work || (length > 0 && !d_bytes)) return fail(RX_EINVAL, "NULL device buffer");
    if (!P->dev) return fail(RX_ENOTUPLOADED, "program has not been uploaded (rx_program_upload)");
    if (P->W > kWaveMaxWords) return fail(RX_ETOOBIG, "the wavefront kernel holds sets of at most 128 words");
    int64_t C, cl;
    long_chunks(P, length, chunks, &C, &cl);
    const size_t need = long_rows_bytes(P, C);
    if (work_bytes < need)
        return fail(RX_EINVAL, "workspace holds " + std::to_string(work_bytes) + " bytes; this run needs " +
                                   std::to_string(need) + " (rx_match_long_workspace)");
    int e;
    if (P->nullable) {
        e = launch_fill_i64(d_first, 1, 0, stream);   // the empty prefix is accepted
        if (e) return hip_fail(e, "kernel launch");
        return RX_OK;
    }
    LaunchArgs a;
    if (int rc = make_launch_args(P, d_bytes ? d_bytes : static_cast<const uint8_t*>(d_work),
                                  static_cast<const int64_t*>(d_work), long_rows(P, C),
                                  static_cast<uint8_t*>(d_work), stream, &a))
        return rc;
    a.offsets = nullptr;
    a.out = nullptr;
    a.rows_out = static_cast<uint32_t*>(d_work);
    a.first_pos = reinterpret_cast<int64_t*>(static_cast<uint8_t*>(d_work) + long_sets_bytes(P, C));
    a.rows_len = length;
    a.rows_cl = cl;
    a.rows_per_chunk = P->L + 1;
    e = P->W <= kLaneMaxWords ? launch_lane(a) : launch_wave(a);
    if (e) return hip_fail(e, "kernel launch (rows)");
    e = launch_compose_first(a.rows_out, a.first_pos, C, cl, P->L + 1, P->W, d_first, stream);
    if (e) return hip_fail(e, "kernel launch (composition)");
    return RX_OK;
    RX_GUARD_END
}

int rx_program_node_image(const rx_program* prog, void* buf, size_t cap, size_t* len) {
    RX_GUARD_BEGIN
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (!P || !len) return fail(RX_EINVAL, "NULL argument");
    std::vector<uint8_t> img;
    node_image(P, img);
    *len = img.size();
    if (buf) {
        if (cap < img.size())
            return fail(RX_EINVAL, "node image needs " + std::to_string(img.size()) + " bytes, buffer holds " +
                                       std::to_string(cap));
        std::memcpy(buf, img.data(), img.size());
    }
    return RX_OK;
    RX_GUARD_END
}

int rx_match_nodes(const rx_program* prog, const void* d_image, const uint8_t* d_bytes, const int64_t* d_offsets,
                   int64_t n, uint8_t* d_out, void* stream) {
    TraceRange trace_range_("rx_match_nodes");
    RX_GUARD_BEGIN
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (!P) return fail(RX_EINVAL, "program is NULL");
    if (n < 0) return fail(RX_EINVAL, "negative string count");
    if (n == 0) return RX_OK;
    if (!d_image || !d_bytes || !d_offsets || !d_out) return fail(RX_EINVAL, "NULL device buffer");
    if (P->m > kNodesMaxNodes)
        return fail(RX_ETOOBIG, "the node-per-thread machine keeps stamps for at most " +
                                    std::to_string(kNodesMaxNodes) + " nodes; this program has " + std::to_string(P->m));
    if (int e = launch_nodes(d_image, P->m, d_bytes, d_offsets, 0, n, d_out, stream)) return hip_fail(e, "kernel launch");
    return RX_OK;
    RX_GUARD_END
}

int rx_match_first_fixed(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int64_t n,
                         int64_t* d_first, void* stream) {
    TraceRange trace_range_("rx_match_first_fixed");
    RX_GUARD_BEGIN
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (!P) return fail(RX_EINVAL, "program is NULL");
    if (length < 0) return fail(RX_EINVAL, "negative length");
    if (n < 0) return fail(RX_EINVAL, "negative string count");
    if (n > 0 && (!d_first || (length > 0 && !d_bytes))) return fail(RX_EINVAL, "NULL device buffer");
    if (!P->dev) return fail(RX_ENOTUPLOADED, "program has not been uploaded (rx_program_upload)");
    if (n == 0) return RX_OK;
    int e;
    if (P->nullable) {
        e = launch_fill_i64(d_first, n, 0, stream);   // the empty prefix is accepted
    } else if (jit_first_ready(P) && length > 0 && (length % 16) == 0 && length <= (1 << 26) &&
               (reinterpret_cast<uintptr_t>(d_bytes) & 15) == 0) {
        e = launch_sliced_first(P, d_bytes, length, n, d_first, stream);
    } else {
        LaunchArgs a;
        if (int rc = make_launch_args(P, d_bytes ? d_bytes : reinterpret_cast<const uint8_t*>(d_first),
                                      reinterpret_cast<const int64_t*>(d_first), n,
                                      reinterpret_cast<uint8_t*>(d_first), stream, &a))
            return rc;
        a.offsets = nullptr;
        a.stride = length;
        a.out = nullptr;
        a.first_pos = d_first;
        if (P->W <= kLaneMaxWords) {
            e = launch_lane(a);
        } else {
            if (P->W > kWaveMaxWords) return fail(RX_ETOOBIG, "the wavefront kernel holds sets of at most 128 words");
            e = launch_wave(a);
        }
    }
    if (e) return hip_fail(e, "kernel launch");
    return RX_OK;
    RX_GUARD_END
}

int rx_match_first(const rx_program* prog, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t n,
                   int64_t* d_first, void* stream) {
    TraceRange trace_range_("rx_match_first");
    RX_GUARD_BEGIN
    LaunchArgs a;
    // the result bytes are not written: pass the position buffer through the checks
    if (int rc = make_launch_args(reinterpret_cast<const Program*>(prog), d_bytes, d_offsets, n,
                                  reinterpret_cast<uint8_t*>(d_first), stream, &a))
        return rc;
    if (n == 0) return RX_OK;
    const Program* P = reinterpret_cast<const Program*>(prog);
    a.out = nullptr;
    a.first_pos = d_first;
    int e;
    if (P->W <= kLaneMaxWords) {
        e = launch_lane(a);
    } else {
        if (P->W > kWaveMaxWords) return fail(RX_ETOOBIG, "the wavefront kernel holds sets of at most 128 words");
        e = launch_wave(a);
    }
    if (e) return hip_fail(e, "kernel launch");
    return RX_OK;
    RX_GUARD_END
}

int rx_match_fixed_ex(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int64_t n, uint8_t* d_out,
                      const rx_launch* launch, void* stream) {
    TraceRange trace_range_("rx_match_fixed_ex");
    RX_GUARD_BEGIN
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (length < 0) return fail(RX_EINVAL, "negative length");
    if (n > 0 && length > 0 && !d_bytes) return fail(RX_EINVAL, "NULL device buffer");
    LaunchArgs a;
    // offsets are not read: pass a non-null placeholder through the checks
    if (int rc = make_launch_args(P, d_bytes ? d_bytes : d_out, reinterpret_cast<const int64_t*>(d_out), n, d_out,
                                  stream, &a))
        return rc;
    if (n == 0) return RX_OK;
    a.offsets = nullptr;
    a.stride = length;
    int variant = launch ? launch->variant : RX_VARIANT_AUTO;
    if (launch) {
        if (launch->block < 0 || launch->block > 1024 || (launch->block % 64) != 0)
            return fail(RX_EINVAL, "block must be a multiple of 64 in [64, 1024]");
        if (launch->grid < 0) return fail(RX_EINVAL, "negative grid");
        a.block = launch->block;
        a.grid = launch->grid;
        a.unroll = launch->unroll;
    }
    const bool sliced_ok = jit_ready(P, nullptr, nullptr) && length > 0 && (length % 16) == 0 &&
                           (reinterpret_cast<uintptr_t>(d_bytes) & 15) == 0;
    // A circuit of at most two words runs few or long strings chunk-parallel;
    // many short ones fill the chip better 32 strings to a lane.
    const bool chunks_ok = jit_chunks_ready(P) && length > 0;
    if (variant == RX_VARIANT_AUTO)
        variant = chunks_ok && (length >= 32768 || n <= 4096) ? RX_VARIANT_CHUNKS
                  : sliced_ok                                 ? RX_VARIANT_SLICED
                                                              : auto_table_variant(P, n);
    int e;
    switch (variant) {
    case RX_VARIANT_CHUNKS:
        if (!chunks_ok) return fail(RX_EINVAL, "the chunk-parallel kernel needs rx_program_jit and a circuit of at "
                                               "most two state words");
        if (n > 0x7fffffffll) return fail(RX_EINVAL, "the chunk-parallel kernel runs at most 2^31 - 1 strings");
        if (length > (int64_t(1) << 40)) return fail(RX_EINVAL, "the chunk-parallel kernel runs strings of at most 2^40 bytes");
        e = launch_sliced_chunks(P, d_bytes, length, n, d_out, stream);
        break;
    case RX_VARIANT_SLICED:
        if (!jit_ready(P, nullptr, nullptr)) return fail(RX_EINVAL, "sliced kernel needs rx_program_jit first");
        if (!sliced_ok) return fail(RX_EINVAL, "sliced kernel needs 16-byte aligned bytes and length % 16 == 0");
        {
            int dev = -1;
            hip_current_device(&dev);
            if (a.unroll < 0 || a.unroll > 5)
                return fail(RX_EINVAL, "sliced kernel staging (unroll) must be 1 (prefetch), 2 (load then match), "
                                       "3 (loader wave), 4 (transposing wave) or 5 (skewed sets)");
            e = launch_sliced_fixed(P, d_bytes, length, n, d_out, a.unroll ? a.unroll : jit_default_staging(P), stream);
        }
        break;
    case RX_VARIANT_LANE:
        if (P->W > kLaneMaxWords) return fail(RX_ETOOBIG, "the lane kernel holds sets of at most 16 words");
        if (a.block > 256) return fail(RX_EINVAL, "the lane kernel runs at most 256 threads per workgroup");
        e = launch_lane(a);
        break;
    case RX_VARIANT_WAVE:
        if (P->W > kWaveMaxWords) return fail(RX_ETOOBIG, "the wavefront kernel holds sets of at most 128 words");
        if (a.unroll != 0 && a.unroll != 1 && a.unroll != 2 && a.unroll != 4 && a.unroll != 8 && a.unroll != 16)
            return fail(RX_EINVAL, "wavefronts per string (unroll) must be 0 (by string count), 1, 2, 4, 8 or 16");
        e = launch_wave(a);
        break;
    default: return fail(RX_EINVAL, "unknown kernel variant");
    }
    if (e) return hip_fail(e, "kernel launch");
    return RX_OK;
    RX_GUARD_END
}

int rx_match_fixed(const rx_program* prog, const uint8_t* d_bytes, int64_t length, int64_t n, uint8_t* d_out,
                   void* stream) {
    TraceRange trace_range_("rx_match_fixed");
    return rx_match_fixed_ex(prog, d_bytes, length, n, d_out, nullptr, stream);
}

static int multi_shape(const rx_multi_config* cfg, int32_t* edges, int32_t* n_edges, int32_t* block, int32_t* grid) {
    *n_edges = 0;
    if (cfg && cfg->n_edges > 0) {
        if (cfg->n_edges > 15) return fail(RX_EINVAL, "at most 15 bucket edges");
        for (int i = 0; i < cfg->n_edges; ++i) {
            if (cfg->edges[i] < 0 || (i > 0 && cfg->edges[i] <= cfg->edges[i - 1]))
                return fail(RX_EINVAL, "bucket edges must be non-negative and ascending");
            edges[i] = cfg->edges[i];
        }
        *n_edges = cfg->n_edges;
    } else {
        for (int e = 8; e <= 4096; e *= 2) edges[(*n_edges)++] = e;
    }
    *block = cfg && cfg->block ? cfg->block : 256;
    if (*block != 64 && *block != 128 && *block != 256) return fail(RX_EINVAL, "block must be 64, 128 or 256");
    *grid = cfg && cfg->grid > 0 ? cfg->grid : 0;
    if (cfg && cfg->grid < 0) return fail(RX_EINVAL, "negative grid");
    if (*grid == 0) {
        int cus = 0;
        if (hip_cu_count(&cus) || cus <= 0) cus = 256;
        *grid = 4 * cus;
    }
    return RX_OK;
}

int64_t rx_match_multi_workspace(int64_t n, int32_t n_progs, const rx_multi_config* cfg) {
    RX_GUARD_BEGIN
    if (n < 0 || n_progs < 0) return fail(RX_EINVAL, "negative size");
    int32_t edges[16], ne, block, grid;
    if (cfg && cfg->n_edges > 15) return fail(RX_EINVAL, "at most 15 bucket edges");
    ne = cfg && cfg->n_edges > 0 ? cfg->n_edges : 10;
    block = cfg && cfg->block ? cfg->block : 256;
    (void)edges;
    (void)grid;
    if (cfg && cfg->form == RX_FORM_PLANES) {
        if (cfg->max_bytes < 0) return fail(RX_EINVAL, "negative max_bytes");
        return plane_workspace_bytes(n, cfg->max_bytes, n_progs > 0 ? n_progs : 1, block);
    }
    return multi_workspace_bytes(n, n_progs > 0 ? n_progs : 1, ne + 1, block);
    RX_GUARD_END
}

namespace {
// rx_match_multi in plane form: every program's plane-form circuit over slabs
// of length-sorted strings; strings of kSortBins - 1 bytes or more in table form.
int match_multi_planes(const rx_program* const* progs, int32_t n_progs, const uint8_t* d_bytes,
                       const int64_t* d_offsets, int64_t n, uint8_t* d_out, void* d_work, size_t work_bytes,
                       const rx_multi_config& cfg, const MultiArgs& shape, void* stream) {
    if (cfg.max_bytes < 0) return fail(RX_EINVAL, "negative max_bytes");
    const int64_t need = plane_workspace_bytes(n, cfg.max_bytes, n_progs, shape.block_lines);
    if ((int64_t)work_bytes < need)
        return fail(RX_ETOOBIG, "workspace holds " + std::to_string(work_bytes) + " bytes; need " + std::to_string(need));
    PlaneMultiArgs m;
    for (int i = 0; i < n_progs; ++i) {
        const Program* P = reinterpret_cast<const Program*>(progs[i]);
        if (!P) return fail(RX_EINVAL, "program " + std::to_string(i) + " is NULL");
        if (!P->dev) return fail(RX_ENOTUPLOADED, "program " + std::to_string(i) + " has not been uploaded");
        if (P->W > kLaneMaxWords) return fail(RX_ETOOBIG, "program " + std::to_string(i) + " holds more than 16 words");
        const uint8_t* base = static_cast<const uint8_t*>(P->dev);
        m.progs[i] = P;
        m.descs[i].first = reinterpret_cast<const uint32_t*>(base + P->layout.first);
        m.descs[i].follow = reinterpret_cast<const uint32_t*>(base + P->layout.follow);
        m.descs[i].bytemask = reinterpret_cast<const uint32_t*>(base + P->layout.bytemask);
        m.descs[i].L = P->L;
        m.descs[i].W = P->W;
        m.descs[i].suffix_any = P->suffix_any ? 1 : 0;
        m.descs[i].pad = 0;
    }
    if (!jit_planes_prepared(m.progs, n_progs))
        return fail(RX_EINVAL, "this program list has no plane-form module on the device (rx_match_multi_prepare)");
    m.n_progs = n_progs;
    m.block_lines = shape.block_lines;
    m.item_grid = shape.grid;
    m.bytes = d_bytes;
    m.offsets = d_offsets;
    m.n = n;
    m.max_bytes = cfg.max_bytes;
    m.out = d_out;
    m.work = d_work;
    m.stream = stream;
    if (n == 0) return RX_OK;
    if (cfg.graph) {
        std::string topo = "planes", full;
        graph_key(topo, n_progs);
        for (int i = 0; i < n_progs; ++i) graph_key(topo, m.progs[i]->uid);
        graph_key(topo, m.block_lines);
        graph_key(topo, m.item_grid);
        full = topo;
        for (int i = 0; i < n_progs; ++i) graph_key(full, m.descs[i]);
        graph_key(full, m.bytes);
        graph_key(full, m.offsets);
        graph_key(full, m.n);
        graph_key(full, m.max_bytes);
        graph_key(full, m.out);
        graph_key(full, m.work);
        const auto record = [&m](void* cs) {
            PlaneMultiArgs r = m;
            r.stream = cs;
            return launch_planes_multi(r);
        };
        if (int e = graph_replay(topo, full, record, stream, nullptr)) return hip_fail(e, "plane-form graph");
        return RX_OK;
    }
    if (int e = launch_planes_multi(m)) return hip_fail(e, "plane-form launch");
    return RX_OK;
}
}  // namespace

int rx_match_multi(const rx_program* const* progs, int32_t n_progs, const uint8_t* d_bytes,
                   const int64_t* d_offsets, int64_t n, uint8_t* d_out, void* d_work, size_t work_bytes,
                   const rx_multi_config* cfg, void* stream) {
    TraceRange trace_range_("rx_match_multi");
    RX_GUARD_BEGIN
    if (n_progs <= 0 || !progs) return fail(RX_EINVAL, "no programs");
    if (n_progs > kMaxItemProgs) return fail(RX_ETOOBIG, "at most 64 programs per call");
    if (n < 0) return fail(RX_EINVAL, "negative string count");
    if (n > ((int64_t)1 << 31) - 1) return fail(RX_ETOOBIG, "at most 2^31 - 1 strings per call");
    if (n > 0 && (!d_bytes || !d_offsets || !d_out)) return fail(RX_EINVAL, "NULL device buffer");
    if (!d_work || (reinterpret_cast<uintptr_t>(d_work) & 255)) return fail(RX_EINVAL, "workspace must be 256-byte aligned");
    MultiArgs m;
    if (int rc = multi_shape(cfg, m.edges, &m.n_edges, &m.block_lines, &m.grid)) return rc;
    if (cfg && cfg->form != RX_FORM_TABLE && cfg->form != RX_FORM_PLANES) return fail(RX_EINVAL, "unknown form");
    if (cfg && cfg->graph != 0 && cfg->graph != 1) return fail(RX_EINVAL, "graph must be 0 or 1");
    if (cfg && cfg->form == RX_FORM_PLANES) return match_multi_planes(progs, n_progs, d_bytes, d_offsets, n, d_out,
                                                                     d_work, work_bytes, *cfg, m, stream);
    const int64_t need = multi_workspace_bytes(n, n_progs, m.n_edges + 1, m.block_lines);
    if ((int64_t)work_bytes < need)
        return fail(RX_ETOOBIG, "workspace holds " + std::to_string(work_bytes) + " bytes; need " + std::to_string(need));
    for (int i = 0; i < n_progs; ++i) {
        const Program* P = reinterpret_cast<const Program*>(progs[i]);
        if (!P) return fail(RX_EINVAL, "program " + std::to_string(i) + " is NULL");
        if (!P->dev) return fail(RX_ENOTUPLOADED, "program " + std::to_string(i) + " has not been uploaded");
        if (P->W > kLaneMaxWords) return fail(RX_ETOOBIG, "program " + std::to_string(i) + " holds more than 16 words");
        const uint8_t* base = static_cast<const uint8_t*>(P->dev);
        m.progs[i].first = reinterpret_cast<const uint32_t*>(base + P->layout.first);
        m.progs[i].follow = reinterpret_cast<const uint32_t*>(base + P->layout.follow);
        m.progs[i].bytemask = reinterpret_cast<const uint32_t*>(base + P->layout.bytemask);
        m.progs[i].L = P->L;
        m.progs[i].W = P->W;
        m.progs[i].suffix_any = P->suffix_any ? 1 : 0;
        m.progs[i].pad = 0;
    }
    m.n_progs = n_progs;
    m.bytes = d_bytes;
    m.offsets = d_offsets;
    m.n = n;
    m.out = d_out;
    m.work = d_work;
    m.stream = stream;
    if (n == 0) return RX_OK;
    if (cfg && cfg->graph) {
        std::string topo = "table", full;
        graph_key(topo, n_progs);
        graph_key(topo, m.n_edges);
        graph_key(topo, m.edges);
        graph_key(topo, m.block_lines);
        graph_key(topo, m.grid);
        full = topo;
        for (int i = 0; i < n_progs; ++i) graph_key(full, m.progs[i]);
        graph_key(full, m.bytes);
        graph_key(full, m.offsets);
        graph_key(full, m.n);
        graph_key(full, m.out);
        graph_key(full, m.work);
        const auto record = [&m](void* cs) {
            MultiArgs r = m;
            r.stream = cs;
            return launch_multi(r);
        };
        if (int e = graph_replay(topo, full, record, stream, nullptr)) return hip_fail(e, "batched graph");
        return RX_OK;
    }
    if (int e = launch_multi(m)) return hip_fail(e, "batched launch");
    return RX_OK;
    RX_GUARD_END
}

int rx_multi_graph_counts(int64_t counts[3]) {
    RX_GUARD_BEGIN
    if (!counts) return fail(RX_EINVAL, "NULL counts");
    graph_counts(counts);
    return RX_OK;
    RX_GUARD_END
}

int rx_autotune(const rx_program* prog, const uint8_t* d_bytes, const int64_t* d_offsets, int64_t length, int64_t n,
                uint8_t* d_out, int32_t budget_runs, rx_launch* best, double* best_ms, int32_t* n_candidates,
                void* stream) {
    RX_GUARD_BEGIN
    if (!prog || !best) return fail(RX_EINVAL, "NULL argument");
    if (n <= 0) return fail(RX_EINVAL, "autotune needs at least one string");
    const Program* P = reinterpret_cast<const Program*>(prog);
    if (!P->dev) return fail(RX_ENOTUPLOADED, "program has not been uploaded");
    int nc = 0;
    int rc = autotune_single(P, d_bytes, d_offsets, length, n, d_out, budget_runs > 0 ? budget_runs : 64, best, best_ms,
                             &nc, stream);
    if (n_candidates) *n_candidates = nc;
    if (rc == RX_OK) clear_error();
    return rc;
    RX_GUARD_END
}

int rx_autotune_multi(const rx_program* const* progs, int32_t n_progs, const uint8_t* d_bytes,
                      const int64_t* d_offsets, int64_t n, uint8_t* d_out, void* d_work, size_t work_bytes,
                      int32_t budget_runs, rx_multi_config* best, double* best_ms, int32_t* n_candidates,
                      void* stream) {
    RX_GUARD_BEGIN
    if (!progs || !best) return fail(RX_EINVAL, "NULL argument");
    if (n <= 0) return fail(RX_EINVAL, "autotune needs at least one string");
    int nc = 0;
    int rc = autotune_multi(progs, n_progs, d_bytes, d_offsets, n, d_out, d_work, work_bytes,
                            budget_runs > 0 ? budget_runs : 96, best, best_ms, &nc, stream);
    if (n_candidates) *n_candidates = nc;
    if (rc == RX_OK) clear_error();
    return rc;
    RX_GUARD_END
}

int rx_program_jit(rx_program* prog, const char* arch) {
    TraceRange trace_range_("rx_program_jit");
    RX_GUARD_BEGIN
    if (!prog) return fail(RX_EINVAL, "program is NULL");
    int rc = jit_compile(reinterpret_cast<Program*>(prog), arch);
    if (rc == RX_OK) clear_error();
    return rc;
    RX_GUARD_END
}

int rx_program_jit_source(const rx_program* prog, char* buf, size_t cap, size_t* len) {
    RX_GUARD_BEGIN
    if (!prog) return fail(RX_EINVAL, "program is NULL");
    const std::string s = jit_full_source(*reinterpret_cast<const Program*>(prog), nullptr, nullptr);
    if (len) *len = s.size();
    if (buf && cap) {
        const size_t k = s.size() < cap - 1 ? s.size() : cap - 1;
        std::memcpy(buf, s.data(), k);
        buf[k] = 0;
    }
    return RX_OK;
    RX_GUARD_END
}

int rx_program_jit_planes_source(const rx_program* prog, char* buf, size_t cap, size_t* len) {
    RX_GUARD_BEGIN
    if (!prog) return fail(RX_EINVAL, "program is NULL");
    const std::string s = jit_planes_source(*reinterpret_cast<const Program*>(prog), nullptr);
    if (len) *len = s.size();
    if (buf && cap) {
        const size_t k = s.size() < cap - 1 ? s.size() : cap - 1;
        std::memcpy(buf, s.data(), k);
        buf[k] = 0;
    }
    return RX_OK;
    RX_GUARD_END
}

int rx_program_jit_stats(const rx_program* prog, int32_t* ready, int32_t* state_words, int32_t* ops) {
    if (!prog) return fail(RX_EINVAL, "program is NULL");
    int ns = 0, no = 0;
    const bool r = jit_ready(reinterpret_cast<const Program*>(prog), &ns, &no);
    if (ready) *ready = r ? 1 : 0;
    if (state_words) *state_words = ns;
    if (ops) *ops = no;
    return RX_OK;
}

int rx_program_jit_staging(const rx_program* prog, int32_t staged[7]) {
    if (!prog || !staged) return fail(RX_EINVAL, "NULL argument");
    jit_staging(reinterpret_cast<const Program*>(prog), staged);
    return RX_OK;
}

int rx_match_multi_prepare(const rx_program* const* progs, int32_t n_progs, const char* arch,
                           int32_t* spill_bytes) {
    TraceRange trace_range_("rx_match_multi_prepare");
    RX_GUARD_BEGIN
    if (n_progs <= 0 || !progs) return fail(RX_EINVAL, "no programs");
    if (n_progs > kMaxItemProgs) return fail(RX_ETOOBIG, "at most 64 programs per call");
    std::vector<const Program*> ps(n_progs);
    for (int i = 0; i < n_progs; ++i) {
        ps[i] = reinterpret_cast<const Program*>(progs[i]);
        if (!ps[i]) return fail(RX_EINVAL, "program " + std::to_string(i) + " is NULL");
    }
    int sp = 0;
    int rc = jit_prepare_planes(ps.data(), n_progs, arch, &sp);
    if (spill_bytes) *spill_bytes = sp;
    if (rc == RX_OK) clear_error();
    return rc;
    RX_GUARD_END
}

int rx_program_jit_guard(const rx_program* prog, int32_t* ran, int32_t violations[8], int32_t* dropped) {
    if (!prog || !ran || !violations || !dropped) return fail(RX_EINVAL, "NULL argument");
    jit_guard(reinterpret_cast<const Program*>(prog), ran, violations, dropped);
    return RX_OK;
}

int rx_program_jit_selfcheck(const rx_program* prog, int32_t* ran, int32_t* dropped) {
    if (!prog || !ran || !dropped) return fail(RX_EINVAL, "NULL argument");
    jit_selfcheck_report(reinterpret_cast<const Program*>(prog), ran, dropped);
    return RX_OK;
}

int rx_isa_check_staging(const void* code, size_t len, const char* arch, const char* kernel, int32_t* violations) {
    RX_GUARD_BEGIN
    if (!code || !arch || !kernel || !violations) return fail(RX_EINVAL, "NULL argument");
    std::vector<char> co(static_cast<const char*>(code), static_cast<const char*>(code) + len);
    int v = 0;
    std::string example;
    const int rc = isa_check_agpr_staging(co, arch, kernel, &v, &example);
    *violations = v;
    if (rc != 0) return fail(RX_EINVAL, "the check could not run on this code object (code " + std::to_string(rc) + ")");
    if (v) return fail(RX_OK, "first offending instruction:" + example);
    return RX_OK;
    RX_GUARD_END
}

const char* rx_last_error(void) { return last_error_cstr(); }

int rx_trace_enabled(void) { return trace_enabled() ? 1 : 0; }

int rx_stream_copy(void* d_dst, const void* d_src, int64_t bytes, void* stream) {
    if (bytes < 0 || (bytes % 16) != 0) return fail(RX_EINVAL, "bytes must be a non-negative multiple of 16");
    if (bytes && (!d_dst || !d_src)) return fail(RX_EINVAL, "NULL device buffer");
    if ((reinterpret_cast<uintptr_t>(d_dst) | reinterpret_cast<uintptr_t>(d_src)) & 15)
        return fail(RX_EINVAL, "buffers must be 16-byte aligned");
    if (!bytes) return RX_OK;
    if (int e = launch_stream_copy(d_dst, d_src, bytes, stream)) return hip_fail(e, "copy launch");
    return RX_OK;
}

const char* rx_version(void) { return "rx-mi355x 0.1 (gfx950)"; }

}  // extern "C"
