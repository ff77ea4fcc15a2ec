// Batched matching: many programs and strings of uneven length in one
// persistent launch.
//
// Strings are bucketed by length on the device (a histogram, a scan over the
// buckets, a scatter of string ids), so a work item -- up to `block` strings of
// one bucket against one program -- keeps the lanes of a workgroup busy for a
// similar number of bytes.  Work items are generated on the device, longest
// bucket first, and a persistent kernel pulls them from an atomic queue; each
// workgroup stages the item's program tables in LDS (Def. 5.1 evolutions and
// byte masks) and runs the table-form macro step of Def. 5.2 with one lane
// per string.  The same item kernel serves the request batches of the server,
// whose items name a program and a contiguous range of strings.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>

#include "rx_internal.h"
#include "rx_planes.h"

namespace rx {

namespace {

constexpr int kWMax = kLaneMaxWords;

struct ItemKArgs {
    ProgDesc progs[kMaxItemProgs];
    int32_t n_progs;
    int32_t block_lines;
    const uint8_t* bytes;
    const int64_t* offsets;
    const int32_t* ids;     // optional: item lines index this array
    const WorkItem* items;
    const int32_t* n_items; // device count
    int32_t* head;          // device queue head
    uint8_t* out;
};

// One macro step on a W-word set: survivors X = S & M[c]; S' = OR of their
// Follow rows.  Up to four survivors are taken per round so their rows are
// fetched from LDS together (a repeated row is harmless under OR).
template <int W>
__device__ __forceinline__ void step_w(uint32_t (&S)[W], uint32_t c, const uint32_t* __restrict__ M,
                                       const uint32_t* __restrict__ F) {
    uint32_t X[W];
#pragma unroll
    for (int w = 0; w < W; ++w) X[w] = S[w] & M[c * W + w];
#pragma unroll
    for (int w = 0; w < W; ++w) S[w] = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint32_t x = X[w];
        while (x) {
            const int b0 = __builtin_ctz(x);
            x &= x - 1;
            const int b1 = x ? __builtin_ctz(x) : b0;
            x &= x - 1;
            const int b2 = x ? __builtin_ctz(x) : b0;
            x &= x - 1;
            const int b3 = x ? __builtin_ctz(x) : b0;
            x &= x - 1;
            const uint32_t* r0 = F + (w * 32 + b0) * W;
            const uint32_t* r1 = F + (w * 32 + b1) * W;
            const uint32_t* r2 = F + (w * 32 + b2) * W;
            const uint32_t* r3 = F + (w * 32 + b3) * W;
#pragma unroll
            for (int v = 0; v < W; ++v) S[v] |= (r0[v] | r1[v]) | (r2[v] | r3[v]);
        }
    }
}

template <int W>
__device__ int match_w(const uint32_t* __restrict__ first, const uint32_t* M, const uint32_t* F, int L,
                       int suffix_any, const uint8_t* __restrict__ bytes, int64_t lo, int64_t hi) {
    uint32_t S[W];
#pragma unroll
    for (int w = 0; w < W; ++w) S[w] = first[w];
    const int aw = L >> 5;
    const uint32_t abit = 1u << (L & 31);
    const int64_t skew = (int64_t)(reinterpret_cast<uintptr_t>(bytes) & 15);
    for (int64_t base = ((lo + skew) & ~int64_t(15)) - skew; base < hi; base += 16) {
        const uint4 v = *reinterpret_cast<const uint4*>(bytes + base);
        const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
        const int b0 = lo > base ? (int)(lo - base) : 0;
        const int b1 = hi - base < 16 ? (int)(hi - base) : 16;
#pragma unroll
        for (int b = 0; b < 16; ++b)
            if (b >= b0 && b < b1) step_w<W>(S, (wv[b >> 2] >> (8 * (b & 3))) & 255u, M, F);
        uint32_t any = 0, acc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            any |= S[w];
            acc |= (w == aw) ? S[w] : 0u;
        }
        if (any == 0) return 0;
        if (suffix_any && (acc & abit)) return 1;
    }
    uint32_t acc = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) acc |= (w == aw) ? S[w] : 0u;
    return (acc & abit) ? 1 : 0;
}

__device__ int match_one(const uint32_t* __restrict__ first, const uint32_t* M, const uint32_t* F, int L, int W,
                         int suffix_any, const uint8_t* __restrict__ bytes, int64_t lo, int64_t hi) {
    switch (W) {
#define RX_MW(w) \
    case w: return match_w<w>(first, M, F, L, suffix_any, bytes, lo, hi);
        RX_MW(1) RX_MW(2) RX_MW(3) RX_MW(4) RX_MW(5) RX_MW(6) RX_MW(7) RX_MW(8)
        RX_MW(9) RX_MW(10) RX_MW(11) RX_MW(12) RX_MW(13) RX_MW(14) RX_MW(15) RX_MW(16)
#undef RX_MW
    default: return 0;  // not reached: the host refuses programs above 16 words
    }
}

__global__ __launch_bounds__(256) void k_items(ItemKArgs a) {
    extern __shared__ uint32_t lds[];
    __shared__ int s_item;
    int loaded = -1;
    const int total = *a.n_items;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.head, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= total) break;  // every wave of the workgroup sees the same value and exits
        const WorkItem item = a.items[it];
        const ProgDesc& P = a.progs[item.prog];
        if (item.prog != loaded) {
            for (int i = threadIdx.x; i < 256 * P.W; i += blockDim.x) lds[i] = P.bytemask[i];
            for (int i = threadIdx.x; i < P.L * P.W; i += blockDim.x) lds[256 * P.W + i] = P.follow[i];
            loaded = item.prog;
            __syncthreads();
        }
        for (int k = threadIdx.x; k < item.count; k += blockDim.x) {
            const int64_t line = a.ids ? (int64_t)a.ids[item.line0 + k] : item.line0 + k;
            const int64_t lo = a.offsets[line], hi = a.offsets[line + 1];
            const int r = match_one(P.first, lds, lds + 256 * P.W, P.L, P.W, P.suffix_any, a.bytes, lo, hi);
            a.out[item.out0 + line] = (uint8_t)r;
        }
        __syncthreads();  // the tables and s_item are reused by the next item
    }
}

// -- bucketing -------------------------------------------------------------
__device__ __forceinline__ int bucket_of(int64_t len, const int32_t* edges, int n_edges) {
    int b = 0;
    while (b < n_edges && len > edges[b]) ++b;
    return b;  // bucket b holds lengths in (edges[b-1], edges[b]]; the last one everything longer
}

struct BucketArgs {
    int32_t edges[kMaxBuckets];
    int32_t n_edges;
    const int64_t* offsets;
    int64_t n;
    int32_t* counts;   // [n_buckets]
    int32_t* cursor;   // [n_buckets]
    int32_t* start;    // [n_buckets + 1]
    int32_t* item_start;  // [n_buckets]
    int32_t* ids;      // [n]
    WorkItem* items;
    int32_t* n_items;
    int32_t* head;
    int32_t n_progs;
    int32_t block_lines;
    int64_t out_stride;
};

__global__ void k_bucket_clear(BucketArgs a) {
    const int nb = a.n_edges + 1;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        a.counts[i] = 0;
        a.cursor[i] = 0;
    }
    if (threadIdx.x == 0) {
        *a.n_items = 0;
        *a.head = 0;
    }
}

// Each workgroup histograms a contiguous range of strings in LDS and adds
// its totals to the global counts once per bucket (a global atomic per
// string on ~16 counters serialises at the L2).
__device__ __forceinline__ void wg_range(int64_t n, int64_t& r0, int64_t& r1) {
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    r0 = (int64_t)blockIdx.x * per;
    r1 = r0 + per < n ? r0 + per : n;
}

__global__ __launch_bounds__(256) void k_bucket_count(BucketArgs a) {
    __shared__ int32_t h[kMaxBuckets];
    const int nb = a.n_edges + 1;
    if (threadIdx.x < kMaxBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    int64_t r0, r1;
    wg_range(a.n, r0, r1);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x)
        atomicAdd(&h[bucket_of(a.offsets[i + 1] - a.offsets[i], a.edges, a.n_edges)], 1);
    __syncthreads();
    if (threadIdx.x < nb && h[threadIdx.x]) atomicAdd(&a.counts[threadIdx.x], h[threadIdx.x]);
}

// one thread: bucket starts, and where each bucket's items begin in the
// queue (longest bucket first; within a bucket, program-major so that a
// workgroup's successive items tend to share the staged tables)
__global__ void k_bucket_scan(BucketArgs a) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int nb = a.n_edges + 1;
    int32_t s = 0;
    for (int b = 0; b < nb; ++b) {
        a.start[b] = s;
        s += a.counts[b];
    }
    a.start[nb] = s;
    int32_t k = 0;
    for (int b = nb - 1; b >= 0; --b) {
        a.item_start[b] = k;
        k += (a.counts[b] + a.block_lines - 1) / a.block_lines * a.n_progs;
    }
    *a.n_items = k;
}

__global__ void k_bucket_fill(BucketArgs a) {
    const int nb = a.n_edges + 1;
    const int32_t total = *a.n_items;
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < total; k += gridDim.x * blockDim.x) {
        int b = -1;
        for (int c = 0; c < nb; ++c) {
            const int32_t tiles = (a.counts[c] + a.block_lines - 1) / a.block_lines;
            if (tiles > 0 && k >= a.item_start[c] && k < a.item_start[c] + tiles * a.n_progs) b = c;
        }
        if (b < 0) continue;  // not reached: every k < total lies in one bucket's range
        const int32_t tiles = (a.counts[b] + a.block_lines - 1) / a.block_lines;
        const int32_t local = k - a.item_start[b];
        const int32_t p = local / tiles, t = local % tiles;
        WorkItem w;
        w.prog = p;
        w.count = a.counts[b] - t * a.block_lines < a.block_lines ? a.counts[b] - t * a.block_lines : a.block_lines;
        w.line0 = a.start[b] + (int64_t)t * a.block_lines;
        w.out0 = (int64_t)p * a.out_stride;
        a.items[k] = w;
    }
}

// The same ranges as k_bucket_count: a workgroup reserves its share of each
// bucket with one global atomic, then places its strings through LDS
// cursors.  The order of ids inside a bucket varies from run to run; every
// string's bit is written at its own index, so results do not.
__global__ __launch_bounds__(256) void k_bucket_scatter(BucketArgs a) {
    __shared__ int32_t h[kMaxBuckets];
    __shared__ int32_t g[kMaxBuckets];
    const int nb = a.n_edges + 1;
    if (threadIdx.x < kMaxBuckets) h[threadIdx.x] = 0;
    __syncthreads();
    int64_t r0, r1;
    wg_range(a.n, r0, r1);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x)
        atomicAdd(&h[bucket_of(a.offsets[i + 1] - a.offsets[i], a.edges, a.n_edges)], 1);
    __syncthreads();
    if (threadIdx.x < nb) {
        g[threadIdx.x] = h[threadIdx.x] ? atomicAdd(&a.cursor[threadIdx.x], h[threadIdx.x]) : 0;
        h[threadIdx.x] = 0;
    }
    __syncthreads();
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const int b = bucket_of(a.offsets[i + 1] - a.offsets[i], a.edges, a.n_edges);
        const int32_t pos = atomicAdd(&h[b], 1);
        a.ids[a.start[b] + g[b] + pos] = (int32_t)i;
    }
}

// -- plane form: exact-length sort, slabs, bit planes ------------------------
//
// Strings shorter than kSortBins - 1 bytes are counting-sorted by length, so
// a slab of 2048 consecutive sorted strings spans lengths close together;
// longer strings (rare) are left to the table-form item kernel.  A slab runs
// ceil(max length / 4) ticks; the planes of all slabs are gathered and
// transposed once per call, then every program's circuit reads them.

struct SortArgs {
    const int64_t* offsets;
    int64_t n;
    int32_t* counts;   // [kSortBins]
    int32_t* cursor;   // [kSortBins]
    int32_t* start;    // [kSortBins + 1]
    int64_t* info;     // [0] strings in slabs, [1] longer strings, [2] plane-kernel groups, [3] capacity exceeded
    int32_t* sorted;   // [n]: slab strings by length, then the longer ones
    int32_t* rank;     // [n]: where each string went in `sorted`
    int64_t* slab_tick;   // [max_slabs + 1]
    int64_t* slab_chunk;  // [max_slabs + 1]
    int64_t max_slabs;
    int64_t tick_cap;     // ticks the plane buffer holds
};

constexpr int kGroupTicks = 64;   // plane-kernel work unit: 256 positions of one slab
constexpr int64_t kLongSlabs = 16;   // slabs whose circuits start first, on their own stream

__device__ __forceinline__ int sort_bin(int64_t len) { return len < kSortBins - 1 ? (int)len : kSortBins - 1; }

__global__ void k_sort_clear(SortArgs a) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kSortBins; i += gridDim.x * blockDim.x) {
        a.counts[i] = 0;
        a.cursor[i] = 0;
    }
}

__global__ __launch_bounds__(256) void k_sort_count(SortArgs a) {
    __shared__ int32_t h[kSortBins];
    for (int i = threadIdx.x; i < kSortBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    int64_t r0, r1;
    wg_range(a.n, r0, r1);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) atomicAdd(&h[sort_bin(a.offsets[i + 1] - a.offsets[i])], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < kSortBins; i += blockDim.x)
        if (h[i]) atomicAdd(&a.counts[i], h[i]);
}

// One workgroup of 1024 threads: bin starts (exclusive scan), the split
// between slab strings and longer ones.
__global__ __launch_bounds__(1024) void k_sort_scan(SortArgs a) {
    __shared__ int32_t part[1024];
    constexpr int per = (kSortBins + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    int32_t sum = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < kSortBins) sum += a.counts[b0 + k];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {   // inclusive scan of the parts
        const int32_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - sum;
    for (int k = 0; k < per; ++k)
        if (b0 + k < kSortBins) {
            a.start[b0 + k] = run;
            run += a.counts[b0 + k];
        }
    if (threadIdx.x == 1023) {
        a.start[kSortBins] = part[1023];
        a.info[0] = part[1023] - a.counts[kSortBins - 1];
        a.info[1] = a.counts[kSortBins - 1];
    }
}

__global__ __launch_bounds__(256) void k_sort_scatter(SortArgs a) {
    __shared__ int32_t h[kSortBins];
    __shared__ int32_t g[kSortBins];
    for (int i = threadIdx.x; i < kSortBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    int64_t r0, r1;
    wg_range(a.n, r0, r1);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) atomicAdd(&h[sort_bin(a.offsets[i + 1] - a.offsets[i])], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < kSortBins; i += blockDim.x) {
        g[i] = h[i] ? atomicAdd(&a.cursor[i], h[i]) : 0;
        h[i] = 0;
    }
    __syncthreads();
    for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const int b = sort_bin(a.offsets[i + 1] - a.offsets[i]);
        const int32_t pos = atomicAdd(&h[b], 1);
        a.sorted[a.start[b] + g[b] + pos] = (int32_t)i;
        a.rank[i] = a.start[b] + g[b] + pos;
    }
}

// One workgroup of 1024 threads: ticks of every slab (its longest string is
// its last), their prefix sums, and the groups of kGroupTicks ticks the plane
// kernel works in (slab_chunk: prefix sums of groups).  If the total would pass the plane buffer's capacity (only when
// the caller's byte bound is below the real total), every slab gets no ticks:
// nothing is read or written past the buffer, and info[3] is set.
__global__ __launch_bounds__(1024) void k_slab_scan(SortArgs a) {
    __shared__ int64_t part[1024], cpart[1024];
    const int64_t n_sliced = a.info[0];
    const int64_t S = (n_sliced + kSlabStrings - 1) / kSlabStrings;
    const int64_t per = (S + 1023) / 1024;
    const int64_t s0 = (int64_t)threadIdx.x * per;
    auto ticks_of = [&](int64_t s) -> int64_t {
        const int64_t last = s * kSlabStrings + kSlabStrings - 1 < n_sliced ? s * kSlabStrings + kSlabStrings - 1
                                                                              : n_sliced - 1;
        const int32_t id = a.sorted[last];
        return (a.offsets[id + 1] - a.offsets[id] + 3) / 4;
    };
    int64_t sum = 0, csum = 0;
    for (int64_t k = 0; k < per; ++k)
        if (s0 + k < S) {
            const int64_t t = ticks_of(s0 + k);
            sum += t;
            csum += (t + kGroupTicks - 1) / kGroupTicks;
        }
    part[threadIdx.x] = sum;
    cpart[threadIdx.x] = csum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = threadIdx.x >= d ? part[threadIdx.x - d] : 0;
        const int64_t cv = threadIdx.x >= d ? cpart[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        cpart[threadIdx.x] += cv;
        __syncthreads();
    }
    const bool over = part[1023] > a.tick_cap;
    int64_t run = part[threadIdx.x] - sum, crun = cpart[threadIdx.x] - csum;
    for (int64_t k = 0; k < per; ++k)
        if (s0 + k < S) {
            a.slab_tick[s0 + k] = over ? 0 : run;
            a.slab_chunk[s0 + k] = over ? 0 : crun;
            const int64_t t = ticks_of(s0 + k);
            run += t;
            crun += (t + kGroupTicks - 1) / kGroupTicks;
        }
    if (threadIdx.x == 1023) {
        a.slab_tick[S] = over ? 0 : part[1023];
        a.slab_chunk[S] = over ? 0 : cpart[1023];
        a.info[2] = over ? 0 : cpart[1023];
        a.info[3] = over ? 1 : 0;
    }
}

struct PlanesArgs {
    const uint8_t* bytes;
    const int64_t* offsets;
    const int32_t* sorted;
    const int64_t* info;
    const int64_t* slab_tick;
    const int64_t* slab_chunk;
    uint32_t* planes;
    int64_t r_lo, r_hi;   // the slabs of rank r_lo <= r < r_hi (rank 0 = the longest)
};

// Gathers and transposes: one workgroup per group of kGroupTicks ticks of a
// slab (longest slabs first), its four wavefronts on 16-position chunks c =
// wave, wave + 4, ... of the group, so the four read the same cache lines of
// the slab's strings at about the same time.  Lane l reads a 16-byte window
// of each of its 32 strings and writes four ticks of plane words (1 KiB per
// group of four words, coalesced).  A slab of n ticks takes n / kGroupTicks
// workgroups, so the longest slabs do not serialise the kernel; with SPLIT,
// the four rounds of a group (chunks 4 i .. 4 i + 3) go to four workgroups,
// for the few longest slabs whose planes are wanted first.  Only the slabs of
// rank r_lo .. r_hi - 1 (rank 0 = the longest, slab S - 1).
template <bool SPLIT>
__global__ __launch_bounds__(256, 2) void k_planes(PlanesArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t n_sliced = a.info[0];
    const int64_t S = (n_sliced + kSlabStrings - 1) / kSlabStrings;
    const int64_t s_first = S - a.r_hi > 0 ? S - a.r_hi : 0, s_end = S - a.r_lo > 0 ? S - a.r_lo : 0;
    if (s_first >= s_end) return;
    const int64_t unit = SPLIT ? (int64_t)(blockIdx.x >> 2) : (int64_t)blockIdx.x;
    const int64_t u = a.slab_chunk[s_end] - 1 - unit;   // the last groups belong to the longest slabs
    if (u < a.slab_chunk[s_first]) return;
    // the slab holding group u: the last s with slab_chunk[s] <= u
    int64_t lo = s_first, hi = s_end - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (a.slab_chunk[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    const int64_t s = lo;
    const int64_t g = u - a.slab_chunk[s];
    const int64_t t_base = a.slab_tick[s], T = a.slab_tick[s + 1] - t_base;
    const int64_t c_end = (g + 1) * (kGroupTicks / 4) < (T + 3) / 4 ? (g + 1) * (kGroupTicks / 4) : (T + 3) / 4;
    const int64_t c_begin = g * (kGroupTicks / 4) + (SPLIT ? 4 * (int64_t)(blockIdx.x & 3) : 0);
    const int64_t c_stop = SPLIT ? (c_begin + 4 < c_end ? c_begin + 4 : c_end) : c_end;
    if (c_begin >= c_stop) return;
    const int64_t first = a.sorted[s * kSlabStrings];
    const int64_t minlen = a.offsets[first + 1] - a.offsets[first];
    // where the slab's strings are, once per workgroup (the four wavefronts share them)
    __shared__ int64_t s_lo[kSlabStrings];
    __shared__ int32_t s_len[kSlabStrings];
    for (int k = threadIdx.x; k < kSlabStrings; k += blockDim.x) {
        const int64_t e = s * kSlabStrings + k;
        int64_t o = 0, n = 0;
        if (e < n_sliced) {
            const int32_t id = a.sorted[e];
            o = a.offsets[id];
            n = a.offsets[id + 1] - o;
        }
        s_lo[k] = o;
        s_len[k] = (int32_t)n;   // slab strings are shorter than kSortBins
    }
    __syncthreads();
    for (int64_t c = c_begin + wave; c < c_stop; c += 4) {
        uint32_t win[32][4];
        int32_t len[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            len[j] = s_len[j * 64 + lane];
            planes_window16(a.bytes + s_lo[j * 64 + lane], len[j], 16 * c, win[j]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t t = 4 * c + k;
            if (t >= T) break;
            uint32_t w[kPlaneTickWords];
            planes_tick(win, len, k, 4 * t, minlen, w);
            uint4* dst = reinterpret_cast<uint4*>(a.planes) + (t_base + t) * (9 * 64) + lane;
#pragma unroll
            for (int q = 0; q < 9; ++q) dst[q * 64] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
        }
    }
}

// Results back in the strings' own order: string i went to sorted position
// rank[i] (slab r / 2048, entry r % 2048 = 64 j + l: bit j of lane l's word).
// One thread per string and program, consecutive threads on consecutive
// strings, so the result bytes are written in order.  The strings of the
// long_slabs longest slabs are left to k_gather_long (their circuits run on
// the other stream and may still be running), those too long for a slab to
// the table-form kernel.
struct GatherArgs {
    const int32_t* rank;
    const int32_t* sorted;
    const int64_t* info;
    const uint32_t* res;   // slab s, lane l, program p at (s * 64 + l) * n_progs + p
    int64_t n, long_slabs;
    int32_t n_progs;
    uint8_t* out;
};

// the first sorted position of the long slabs
__device__ __forceinline__ int64_t long_cut(const GatherArgs& a, int64_t n_sliced) {
    const int64_t S = (n_sliced + kSlabStrings - 1) / kSlabStrings;
    return S > a.long_slabs ? (S - a.long_slabs) * kSlabStrings : 0;
}

// The bit of sorted position r for every program, written to string i: the
// programs' words of r's (slab, lane) are side by side, so one string reads
// them as a few 16-byte loads, and each program's bytes go out in string
// order.
__device__ __forceinline__ void gather_one(const GatherArgs& a, int64_t r, int64_t i) {
    const int P = a.n_progs;
    const uint32_t* w = a.res + ((r >> 11) * 64 + (r & 63)) * P;
    const int bit = (int)((r & (kSlabStrings - 1)) >> 6);
    uint8_t* out = a.out + i;
    int p = 0;
    if ((P & 3) == 0) {
        for (; p < P; p += 4) {
            const uint4 v = *reinterpret_cast<const uint4*>(w + p);
            out[(p + 0) * a.n] = (uint8_t)((v.x >> bit) & 1u);
            out[(p + 1) * a.n] = (uint8_t)((v.y >> bit) & 1u);
            out[(p + 2) * a.n] = (uint8_t)((v.z >> bit) & 1u);
            out[(p + 3) * a.n] = (uint8_t)((v.w >> bit) & 1u);
        }
    }
    for (; p < P; ++p) out[p * a.n] = (uint8_t)((w[p] >> bit) & 1u);
}

__global__ __launch_bounds__(256) void k_gather_out(GatherArgs a) {
    const int64_t n_sliced = a.info[0];
    const int64_t cut = long_cut(a, n_sliced);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = a.rank[i];
        if (r < cut) gather_one(a, r, i);
    }
}

// The long slabs' results: one thread per sorted position e of those slabs,
// written to string sorted[e].
__global__ __launch_bounds__(256) void k_gather_long(GatherArgs a) {
    const int64_t n_sliced = a.info[0];
    const int64_t cut = long_cut(a, n_sliced);
    for (int64_t e = cut + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_sliced;
         e += (int64_t)gridDim.x * blockDim.x)
        gather_one(a, e, a.sorted[e]);
}

// Work items for the strings too long for slabs: every program, 256 of them
// per item, indices into `sorted` after the slab strings.
struct OverArgs {
    const int64_t* info;
    WorkItem* items;
    int32_t* n_items;
    int32_t* head;
    int32_t n_progs, block_lines;
    int64_t out_stride;
};

__global__ void k_over_fill(OverArgs a) {
    const int64_t n_sliced = a.info[0], n_over = a.info[1];
    const int64_t tiles = (n_over + a.block_lines - 1) / a.block_lines;
    const int64_t total = tiles * a.n_progs;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *a.n_items = (int32_t)total;
        *a.head = 0;
    }
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = k / tiles, t = k % tiles;
        WorkItem w;
        w.prog = (int32_t)p;
        w.count = (int32_t)(n_over - t * a.block_lines < a.block_lines ? n_over - t * a.block_lines : a.block_lines);
        w.line0 = n_sliced + t * a.block_lines;
        w.out0 = p * a.out_stride;
        a.items[k] = w;
    }
}

}  // namespace

namespace {
// A second stream per device for the longest slabs' circuits, with the
// events that fork it from and join it to the caller's stream; the lock keeps
// each call's record/wait pairs together.  A stream under capture gets a
// side stream of its own (it stays in the capture until the capture ends).
struct SideStream {
    std::mutex mu;
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

int side_stream(hipStream_t st, SideStream** out) {
    static std::mutex g_mu;
    static std::map<std::pair<int, int>, SideStream*> g_side;
    int dev = -1;
    if (hipError_t e = hipGetDevice(&dev)) return (int)e;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipError_t e = hipStreamIsCapturing(st, &cap)) return (int)e;
    std::lock_guard<std::mutex> lk(g_mu);
    SideStream*& S = g_side[{dev, cap == hipStreamCaptureStatusNone ? 0 : 1}];
    if (!S) {
        SideStream* x = new SideStream;
        hipError_t e = hipStreamCreateWithFlags(&x->stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x->fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x->join, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (x->fork) (void)hipEventDestroy(x->fork);
            if (x->stream) (void)hipStreamDestroy(x->stream);
            delete x;
            return (int)e;
        }
        S = x;
    }
    *out = S;
    return 0;
}
}  // namespace

int64_t plane_max_slabs(int64_t n) { return (n + kSlabStrings - 1) / kSlabStrings; }

int64_t plane_tick_cap(int64_t n, int64_t max_bytes) {
    // sorted by exact length, every slab but the last two is no longer than the
    // shortest string of the next one: sum of slab lengths <= bytes / 2048 +
    // 2 (kSortBins - 2); a slab's ticks are its length / 4 rounded up
    return max_bytes / (4 * kSlabStrings) + (kSortBins - 2) / 2 + plane_max_slabs(n) + 2;
}

int64_t plane_workspace_bytes(int64_t n, int64_t max_bytes, int32_t n_progs, int32_t block_lines) {
    auto al = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    if (block_lines <= 0) block_lines = 256;
    const int64_t S = plane_max_slabs(n);
    return al(4 * (3 * (int64_t)kSortBins + 1)) + al(8 * 8) + 2 * al(4 * n) + 2 * al(8 * (S + 1)) + al(8 * 4) +
           al((int64_t)sizeof(WorkItem) * (int64_t)n_progs * (n / block_lines + 1)) +
           al(4 * 64 * S * (int64_t)n_progs) + al(plane_tick_cap(n, max_bytes) * kPlaneTickWords * 64 * 4);
}

int launch_planes_multi(const PlaneMultiArgs& m) {
    const hipStream_t st = (hipStream_t)m.stream;
    auto al = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    uint8_t* w = static_cast<uint8_t*>(m.work);
    const int64_t S = plane_max_slabs(m.n);
    SortArgs a;
    a.offsets = m.offsets;
    a.n = m.n;
    a.counts = reinterpret_cast<int32_t*>(w);
    a.cursor = a.counts + kSortBins;
    a.start = a.cursor + kSortBins;
    w += al(4 * (3 * (int64_t)kSortBins + 1));
    a.info = reinterpret_cast<int64_t*>(w);
    w += al(8 * 8);
    a.sorted = reinterpret_cast<int32_t*>(w);
    w += al(4 * m.n);
    a.rank = reinterpret_cast<int32_t*>(w);
    w += al(4 * m.n);
    a.slab_tick = reinterpret_cast<int64_t*>(w);
    w += al(8 * (S + 1));
    a.slab_chunk = reinterpret_cast<int64_t*>(w);
    w += al(8 * (S + 1));
    int32_t* q = reinterpret_cast<int32_t*>(w);   // item count, queue head
    w += al(8 * 4);
    WorkItem* items = reinterpret_cast<WorkItem*>(w);
    w += al((int64_t)sizeof(WorkItem) * (int64_t)m.n_progs * (m.n / m.block_lines + 1));
    uint32_t* res = reinterpret_cast<uint32_t*>(w);
    w += al(4 * 64 * S * (int64_t)m.n_progs);
    uint32_t* planes = reinterpret_cast<uint32_t*>(w);
    a.max_slabs = S;
    a.tick_cap = plane_tick_cap(m.n, m.max_bytes);
    SideStream* side = nullptr;
    if (int e = side_stream(st, &side)) return e;
    std::lock_guard<std::mutex> lk(side->mu);
    const int gs = (int)((m.n + 255) / 256 < 1024 ? (m.n + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_sort_clear, dim3((kSortBins + 255) / 256), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_sort_count, dim3(gs > 0 ? gs : 1), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, st, a);
    hipLaunchKernelGGL(k_sort_scatter, dim3(gs > 0 ? gs : 1), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_slab_scan, dim3(1), dim3(1024), 0, st, a);
    PlanesArgs pa;
    pa.bytes = m.bytes;
    pa.offsets = m.offsets;
    pa.sorted = a.sorted;
    pa.info = a.info;
    pa.slab_tick = a.slab_tick;
    pa.slab_chunk = a.slab_chunk;
    pa.planes = planes;
    // The longest slabs first, their circuits on a second stream: a slab's
    // circuit runs one position after another, so the few longest set the
    // length of the call; the planes and circuits of every other slab run
    // beside them.
    const int64_t R = kLongSlabs < S ? kLongSlabs : S;
    pa.r_lo = 0;
    pa.r_hi = R;
    hipLaunchKernelGGL(k_planes<true>, dim3((unsigned)(4 * R * (kSortBins / (4 * kGroupTicks) + 1))), dim3(256), 0, st,
                       pa);
    if (hipError_t e = hipGetLastError()) return (int)e;
    if (hipError_t e = hipEventRecord(side->fork, st)) return (int)e;
    if (hipError_t e = hipStreamWaitEvent(side->stream, side->fork, 0)) return (int)e;
    if (int e = launch_planes_circuits(m.progs, m.n_progs, planes, a.slab_tick, a.info, res, S, 0, R, true,
                                       side->stream))
        return e;
    if (hipError_t e = hipEventRecord(side->join, side->stream)) return (int)e;
    pa.r_lo = R;
    pa.r_hi = S;
    if (S > R)
        hipLaunchKernelGGL(k_planes<false>, dim3((unsigned)(a.tick_cap / kGroupTicks + S + 1)), dim3(256), 0, st, pa);
    if (hipError_t e = hipGetLastError()) return (int)e;
    if (int e = launch_planes_circuits(m.progs, m.n_progs, planes, a.slab_tick, a.info, res, S, R, S, false, m.stream))
        return e;
    GatherArgs ga;
    ga.rank = a.rank;
    ga.sorted = a.sorted;
    ga.info = a.info;
    ga.res = res;
    ga.n = m.n;
    ga.long_slabs = R;
    ga.n_progs = m.n_progs;
    ga.out = m.out;
    const unsigned gx = (unsigned)((m.n + 255) / 256 < 8192 ? (m.n + 255) / 256 : 8192);
    hipLaunchKernelGGL(k_gather_out, dim3(gx), dim3(256), 0, st, ga);
    // then the long slabs, once their circuits are done
    if (hipError_t e = hipStreamWaitEvent(st, side->join, 0)) return (int)e;
    hipLaunchKernelGGL(k_gather_long, dim3((unsigned)((R * kSlabStrings + 255) / 256)), dim3(256), 0, st, ga);
    // strings too long for a slab: table form, every program
    OverArgs o;
    o.info = a.info;
    o.items = items;
    o.n_items = q;
    o.head = q + 1;
    o.n_progs = m.n_progs;
    o.block_lines = m.block_lines;
    o.out_stride = m.n;
    hipLaunchKernelGGL(k_over_fill, dim3(64), dim3(256), 0, st, o);
    ItemKArgs k;
    for (int i = 0; i < m.n_progs; ++i) k.progs[i] = m.descs[i];
    k.n_progs = m.n_progs;
    k.block_lines = m.block_lines;
    k.bytes = m.bytes;
    k.offsets = m.offsets;
    k.ids = a.sorted;
    k.items = items;
    k.n_items = q;
    k.head = q + 1;
    k.out = m.out;
    int max_lds_words = 0;
    for (int i = 0; i < m.n_progs; ++i) {
        const int words = (256 + m.descs[i].L) * m.descs[i].W;
        if (words > max_lds_words) max_lds_words = words;
    }
    hipLaunchKernelGGL(k_items, dim3(m.item_grid), dim3(m.block_lines), 4 * (size_t)max_lds_words, st, k);
    return (int)hipGetLastError();
}

int64_t multi_workspace_bytes(int64_t n, int32_t n_progs, int32_t n_buckets, int32_t block_lines) {
    auto al = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    if (block_lines <= 0) block_lines = 256;
    const int64_t max_items = (n / block_lines + n_buckets + 1) * (int64_t)n_progs;
    return al(4 * (int64_t)(4 * (n_buckets + 1) + 4)) + al(4 * n) + al((int64_t)sizeof(WorkItem) * max_items);
}

int launch_multi(const MultiArgs& m) {
    const hipStream_t st = (hipStream_t)m.stream;
    const int nb = m.n_edges + 1;
    uint8_t* w = static_cast<uint8_t*>(m.work);
    auto al = [](int64_t x) { return (x + 255) & ~int64_t(255); };
    BucketArgs b;
    for (int i = 0; i < kMaxBuckets; ++i) b.edges[i] = i < m.n_edges ? m.edges[i] : 0;
    b.n_edges = m.n_edges;
    b.offsets = m.offsets;
    b.n = m.n;
    int32_t* small = reinterpret_cast<int32_t*>(w);
    b.counts = small;
    b.cursor = small + (nb + 1);
    b.start = small + 2 * (nb + 1);
    b.item_start = small + 3 * (nb + 1);
    b.n_items = small + 4 * (nb + 1);
    b.head = small + 4 * (nb + 1) + 1;
    const int64_t o_ids = al(4 * (int64_t)(4 * (nb + 1) + 4));
    b.ids = reinterpret_cast<int32_t*>(w + o_ids);
    b.items = reinterpret_cast<WorkItem*>(w + o_ids + al(4 * m.n));
    b.n_progs = m.n_progs;
    b.block_lines = m.block_lines;
    b.out_stride = m.n;
    const int gs = (int)((m.n + 255) / 256 < 1024 ? (m.n + 255) / 256 : 1024);
    hipLaunchKernelGGL(k_bucket_clear, dim3(1), dim3(64), 0, st, b);
    if (m.n > 0) hipLaunchKernelGGL(k_bucket_count, dim3(gs > 0 ? gs : 1), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(64), 0, st, b);
    if (m.n > 0) hipLaunchKernelGGL(k_bucket_scatter, dim3(gs > 0 ? gs : 1), dim3(256), 0, st, b);
    hipLaunchKernelGGL(k_bucket_fill, dim3(1024), dim3(256), 0, st, b);
    if (hipError_t e = hipGetLastError()) return (int)e;
    ItemKArgs k;
    for (int i = 0; i < m.n_progs; ++i) k.progs[i] = m.progs[i];
    k.n_progs = m.n_progs;
    k.block_lines = m.block_lines;
    k.bytes = m.bytes;
    k.offsets = m.offsets;
    k.ids = b.ids;
    k.items = b.items;
    k.n_items = b.n_items;
    k.head = b.head;
    k.out = m.out;
    int max_lds_words = 0;
    for (int i = 0; i < m.n_progs; ++i) {
        const int words = (256 + m.progs[i].L) * m.progs[i].W;
        if (words > max_lds_words) max_lds_words = words;
    }
    const int grid = m.grid > 0 ? m.grid : 1024;
    hipLaunchKernelGGL(k_items, dim3(grid), dim3(m.block_lines), 4 * (size_t)max_lds_words, st, k);
    return (int)hipGetLastError();
}

int launch_items(const ItemsArgs& m) {
    ItemKArgs k;
    for (int i = 0; i < m.n_progs; ++i) k.progs[i] = m.progs[i];
    k.n_progs = m.n_progs;
    k.block_lines = m.block;
    k.bytes = m.bytes;
    k.offsets = m.offsets;
    k.ids = nullptr;
    k.items = m.items;
    k.n_items = m.n_items;
    k.head = m.head;
    k.out = m.out;
    int max_lds_words = 0;
    for (int i = 0; i < m.n_progs; ++i) {
        const int words = (256 + m.progs[i].L) * m.progs[i].W;
        if (words > max_lds_words) max_lds_words = words;
    }
    hipLaunchKernelGGL(k_items, dim3(m.grid > 0 ? m.grid : 1024), dim3(m.block > 0 ? m.block : 256),
                       4 * (size_t)max_lds_words, (hipStream_t)m.stream, k);
    return (int)hipGetLastError();
}

// -- one serving step: copies in, the item kernel, results out ----------------
namespace {

ItemKArgs item_kargs(const ItemsArgs& m) {
    ItemKArgs k;
    for (int i = 0; i < kMaxItemProgs; ++i) k.progs[i] = i < m.n_progs ? m.progs[i] : ProgDesc{};
    k.n_progs = m.n_progs;
    k.block_lines = m.block;
    k.bytes = m.bytes;
    k.offsets = m.offsets;
    k.ids = nullptr;
    k.items = m.items;
    k.n_items = m.n_items;
    k.head = m.head;
    k.out = m.out;
    return k;
}

constexpr unsigned kStepLds = 4u * (256u + 511u) * (unsigned)kLaneMaxWords;  // the largest program a step may hold

}  // namespace

int step_launch_direct(const StepDesc& d, void* stream) {
    const hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < 3; ++i)
        if (d.h2d[i].bytes)
            if (hipError_t e = hipMemcpyAsync(d.h2d[i].dst, d.h2d[i].src, d.h2d[i].bytes, hipMemcpyHostToDevice, st))
                return (int)e;
    ItemKArgs k = item_kargs(d.items);
    hipLaunchKernelGGL(k_items, dim3(d.items.grid), dim3(d.items.block), kStepLds, st, k);
    if (hipError_t e = hipGetLastError()) return (int)e;
    if (d.d2h.bytes)
        if (hipError_t e = hipMemcpyAsync(d.d2h.dst, d.d2h.src, d.d2h.bytes, hipMemcpyDeviceToHost, st)) return (int)e;
    return 0;
}

struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t copy[3] = {}, kernel = nullptr, back = nullptr;
    ItemKArgs args;
};

int step_graph_launch(StepGraph** pg, const StepDesc& d, void* stream) {
    const hipStream_t st = (hipStream_t)stream;
    auto sz = [](size_t b) { return b ? b : (size_t)1; };
    StepGraph* g = *pg;
    if (!g) {
        g = new StepGraph;
        hipError_t e = hipGraphCreate(&g->graph, 0);
        hipGraphNode_t prev = nullptr;
        for (int i = 0; i < 3 && e == hipSuccess; ++i) {
            e = hipGraphAddMemcpyNode1D(&g->copy[i], g->graph, prev ? &prev : nullptr, prev ? 1 : 0, d.h2d[i].dst,
                                        d.h2d[i].src, sz(d.h2d[i].bytes), hipMemcpyHostToDevice);
            prev = g->copy[i];
        }
        g->args = item_kargs(d.items);
        if (e == hipSuccess) {
            hipKernelNodeParams kp = {};
            void* params[] = {&g->args};
            kp.func = (void*)k_items;
            kp.gridDim = dim3(d.items.grid);
            kp.blockDim = dim3(d.items.block);
            kp.sharedMemBytes = kStepLds;
            kp.kernelParams = params;
            kp.extra = nullptr;
            e = hipGraphAddKernelNode(&g->kernel, g->graph, &prev, 1, &kp);
            prev = g->kernel;
        }
        if (e == hipSuccess)
            e = hipGraphAddMemcpyNode1D(&g->back, g->graph, &prev, 1, d.d2h.dst, d.d2h.src, sz(d.d2h.bytes),
                                        hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            step_graph_destroy(g);
            return (int)e;
        }
        *pg = g;
        return (int)hipGraphLaunch(g->exec, st);
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
        e = hipGraphExecMemcpyNodeSetParams1D(g->exec, g->copy[i], d.h2d[i].dst, d.h2d[i].src, sz(d.h2d[i].bytes),
                                              hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        g->args = item_kargs(d.items);
        hipKernelNodeParams kp = {};
        void* params[] = {&g->args};
        kp.func = (void*)k_items;
        kp.gridDim = dim3(d.items.grid);
        kp.blockDim = dim3(d.items.block);
        kp.sharedMemBytes = kStepLds;
        kp.kernelParams = params;
        kp.extra = nullptr;
        e = hipGraphExecKernelNodeSetParams(g->exec, g->kernel, &kp);
    }
    if (e == hipSuccess)
        e = hipGraphExecMemcpyNodeSetParams1D(g->exec, g->back, d.d2h.dst, d.d2h.src, sz(d.d2h.bytes),
                                              hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipGraphLaunch(g->exec, st);
    return (int)e;
}

void step_graph_destroy(StepGraph* g) {
    if (!g) return;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
}

}  // namespace rx
