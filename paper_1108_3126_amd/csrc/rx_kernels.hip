// Table-form lockstep kernels for gfx950.
//
// One macro step of the generic lockstep machine (Def. 5.2 / 5.3, Rathnayake &
// Thielecke, SOS 2011) on a bitset thread set S over leaf ranks:
//     X  = S & Mask[c]              -- the synchronised move on byte c: only
//                                      leaves whose label holds c survive
//     S' = OR_{x in X} Follow[x]    -- each survivor moves to its continuation
//                                      and is evolved (Def. 5.1); OR-ing the
//                                      precomputed evolutions is exactly the
//                                      removal of duplicate threads by pointer
//                                      equality.
// The accept bit (null) has rank L and is never in Mask[c], so a thread that
// reached null dies when input remains.  A string is accepted when the accept
// bit is in S after its last byte.
//
// Two layouts:
//   k_lane<W>  one lane owns one string and its W-word set in registers;
//              Mask and Follow are staged once per workgroup in LDS.
//   k_wave<>   one wavefront owns one string; lane j owns words j and j+64 of
//              the set; survivors are enumerated wave-uniformly with ballot.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <unordered_map>

#include "rx_internal.h"

namespace rx {

namespace {

struct KArgs {
    const uint32_t* first;
    const uint32_t* follow;
    const uint32_t* bytemask;
    const uint32_t* chunks;
    int32_t L, W, suffix_any, pad;
    const uint8_t* bytes;
    const int64_t* offsets;  // NULL: string i is bytes[i * stride, (i + 1) * stride)
    int64_t stride;
    int64_t n;
    uint8_t* out;
    int64_t* first_pos;   // FIRST kernels: the earliest accepting prefix length, -1 if none
    // ROWS kernels (chunk-parallel matching of one string bytes[0, rows_len)):
    // row 0 runs chunk 0 from First; row 1 + (c - 1) * rows_per_chunk + r
    // runs chunk c (bytes [c * rows_cl, (c + 1) * rows_cl)) from the set {r}
    // (r = L: the accept bit alone); each writes its final set to rows_out.
    uint32_t* rows_out;
    int64_t rows_len, rows_cl;
    int32_t rows_per_chunk, rows_pad;
    // rx_match's layout slot: the kernel does nothing when the slot holds
    // skip_id and no flaw (the bit-sliced kernel has matched the strings)
    const int64_t* skip;
    int64_t skip_id;
};

// true when the layout check of this call found equal lengths and the
// bit-sliced kernel took the strings
__device__ __forceinline__ bool taken_by_sliced(const KArgs& a) {
    return a.skip && a.skip[0] == a.skip_id && a.skip[3] == 0;
}

// Start and byte range of row j of the chunk-parallel run.
__device__ __forceinline__ void row_span(const KArgs& a, int64_t j, int* r, int64_t* lo, int64_t* hi) {
    int64_t c = 0;
    *r = -1;
    if (j > 0) {
        c = 1 + (j - 1) / a.rows_per_chunk;
        *r = (int)((j - 1) % a.rows_per_chunk);
    }
    *lo = c * a.rows_cl;
    *hi = *lo + a.rows_cl < a.rows_len ? *lo + a.rows_cl : a.rows_len;
}

template <int W>
__device__ __forceinline__ uint32_t pick(const uint32_t (&S)[W], int w) {
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) r |= (i == w) ? S[i] : 0u;
    return r;
}

template <int W>
__device__ __forceinline__ void lane_step(uint32_t (&S)[W], uint32_t c, const uint32_t* __restrict__ M,
                                          const uint32_t* __restrict__ F) {
    uint32_t X[W];
    const uint32_t* mrow = M + c * W;
#pragma unroll
    for (int w = 0; w < W; ++w) X[w] = S[w] & mrow[w];
#pragma unroll
    for (int w = 0; w < W; ++w) S[w] = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint32_t x = X[w];
        while (x) {
            // up to four survivors per round: their rows are fetched together
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

// FIRST: instead of the result bit, the smallest k such that the accept bit
// is in S after the first k bytes (k = 0: the root is nullable), or -1.
template <int W, bool FIRST, bool ROWS>
__global__ __launch_bounds__(256) void k_lane(KArgs a) {
    if (taken_by_sliced(a)) return;
    extern __shared__ uint32_t lds[];
    uint32_t* M = lds;
    uint32_t* F = lds + 256 * W;
    for (int i = threadIdx.x; i < 256 * W; i += blockDim.x) M[i] = a.bytemask[i];
    for (int i = threadIdx.x; i < a.L * W; i += blockDim.x) F[i] = a.follow[i];
    __syncthreads();
    const int aw = a.L >> 5;
    const uint32_t abit = 1u << (a.L & 31);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t sid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; sid < a.n; sid += stride) {
        uint32_t S[W];
        int64_t lo, hi;
        if (ROWS) {
            int r;
            row_span(a, sid, &r, &lo, &hi);
#pragma unroll
            for (int w = 0; w < W; ++w) S[w] = r < 0 ? a.first[w] : ((r >> 5) == w ? 1u << (r & 31) : 0u);
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) S[w] = a.first[w];
            lo = a.offsets ? a.offsets[sid] : sid * a.stride;
            hi = a.offsets ? a.offsets[sid + 1] : lo + a.stride;
        }
        int res = -1;
        // (rows look for accepts after at least one byte of their chunk)
        int64_t pos = (FIRST && !ROWS && (pick<W>(S, aw) & abit)) ? 0 : -1;
        // aligned 16-byte blocks of the absolute address range [bytes+lo, bytes+hi):
        // every block read holds at least one byte of the string
        const int64_t skew = (int64_t)(reinterpret_cast<uintptr_t>(a.bytes) & 15);
        for (int64_t base = ((lo + skew) & ~int64_t(15)) - skew; base < hi && pos < 0; base += 16) {
            const uint4 v = *reinterpret_cast<const uint4*>(a.bytes + base);
            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
            const int b0 = lo > base ? (int)(lo - base) : 0;
            const int b1 = hi - base < 16 ? (int)(hi - base) : 16;
#pragma unroll
            for (int b = 0; b < 16; ++b) {
                if (b >= b0 && b < b1 && (!FIRST || pos < 0)) {
                    lane_step<W>(S, (wv[b >> 2] >> (8 * (b & 3))) & 255u, M, F);
                    if (FIRST && (pick<W>(S, aw) & abit)) pos = base + b + 1 - lo;
                }
            }
            uint32_t any = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) any |= S[w];
            if (any == 0) { res = 0; break; }                          // no live thread: reject
            if (!FIRST && a.suffix_any && (pick<W>(S, aw) & abit)) { res = 1; break; }  // accept is absorbing
        }
        if (ROWS) {   // the set reached; an absorbed accept stands alone
            uint32_t* o = a.rows_out + sid * W;
#pragma unroll
            for (int w = 0; w < W; ++w) o[w] = res == 1 ? (w == aw ? abit : 0u) : S[w];
            if (FIRST) a.first_pos[sid] = pos;   // bytes of the chunk up to the row's first accept, or -1
            continue;
        }
        if (FIRST) {
            a.first_pos[sid] = pos;
            continue;
        }
        if (res < 0) res = (pick<W>(S, aw) & abit) ? 1 : 0;
        a.out[sid] = (uint8_t)res;
    }
}

// One wavefront per string.  Lane j owns words j and j + 64 of the set.
template <bool TABLES_IN_LDS, bool FIRST, bool ROWS>
__global__ __launch_bounds__(1024) void k_wave(KArgs a) {
    if (taken_by_sliced(a)) return;
    extern __shared__ uint32_t lds[];
    const int W = a.W, L = a.L;
    const uint32_t* M = a.bytemask;
    const uint32_t* F = a.follow;
    if (TABLES_IN_LDS) {
        uint32_t* Ml = lds;
        uint32_t* Fl = lds + 256 * W;
        for (int i = threadIdx.x; i < 256 * W; i += blockDim.x) Ml[i] = a.bytemask[i];
        for (int i = threadIdx.x; i < L * W; i += blockDim.x) Fl[i] = a.follow[i];
        __syncthreads();
        M = Ml;
        F = Fl;
    }
    const int lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool own0 = lane < W, own1 = lane + 64 < W;
    const int aw = L >> 5;
    const uint32_t abit = 1u << (L & 31);
    for (int64_t sid = (int64_t)blockIdx.x * waves + wave; sid < a.n; sid += (int64_t)gridDim.x * waves) {
        uint32_t S0 = own0 ? a.first[lane] : 0u;
        uint32_t S1 = own1 ? a.first[lane + 64] : 0u;
        int64_t lo, hi;
        if (ROWS) {
            int r;
            row_span(a, sid, &r, &lo, &hi);
            if (r >= 0) {
                S0 = (r >> 5) == lane ? 1u << (r & 31) : 0u;
                S1 = (r >> 5) == lane + 64 ? 1u << (r & 31) : 0u;
            }
        } else {
            lo = a.offsets ? a.offsets[sid] : sid * a.stride;
            hi = a.offsets ? a.offsets[sid + 1] : lo + a.stride;
        }
        int res = -1;
        int64_t pos = -1;
        if (FIRST && !ROWS) {
            const uint32_t sw = (uint32_t)__builtin_amdgcn_readlane((int)(aw < 64 ? S0 : S1), aw & 63);
            if (sw & abit) pos = 0;
        }
        const int64_t skew = (int64_t)(reinterpret_cast<uintptr_t>(a.bytes) & 3);
        for (int64_t base = ((lo + skew) & ~int64_t(3)) - skew; base < hi && res < 0 && pos < 0; base += 4) {
            const uint32_t word = *reinterpret_cast<const uint32_t*>(a.bytes + base);
            const int b0 = lo > base ? (int)(lo - base) : 0;
            const int b1 = hi - base < 4 ? (int)(hi - base) : 4;
            for (int b = b0; b < b1 && pos < 0; ++b) {
                const uint32_t c = (word >> (8 * b)) & 255u;
                const uint32_t X0 = own0 ? (S0 & M[c * W + lane]) : 0u;
                const uint32_t X1 = own1 ? (S1 & M[c * W + 64 + lane]) : 0u;
                uint32_t N0 = 0, N1 = 0;
                for (int half = 0; half < 2; ++half) {
                    uint64_t nz = __ballot((half ? X1 : X0) != 0);
                    while (nz) {
                        const int wl = __builtin_ctzll(nz);
                        nz &= nz - 1;
                        uint32_t xw = (uint32_t)__builtin_amdgcn_readlane((int)(half ? X1 : X0), wl);
                        const int wordidx = wl + 64 * half;
                        if (a.chunks) {
                            // one union row per survivor byte; the four rows are independent loads
                            const uint32_t* T = a.chunks + (size_t)wordidx * 4 * 256 * W;
                            const uint32_t* r0 = T + (size_t)(0 * 256 + ((xw >> 0) & 255u)) * W;
                            const uint32_t* r1 = T + (size_t)(1 * 256 + ((xw >> 8) & 255u)) * W;
                            const uint32_t* r2 = T + (size_t)(2 * 256 + ((xw >> 16) & 255u)) * W;
                            const uint32_t* r3 = T + (size_t)(3 * 256 + ((xw >> 24) & 255u)) * W;
                            if (own0) N0 |= (r0[lane] | r1[lane]) | (r2[lane] | r3[lane]);
                            if (own1) N1 |= (r0[lane + 64] | r1[lane + 64]) | (r2[lane + 64] | r3[lane + 64]);
                            continue;
                        }
                        while (xw) {
                            const int bit = __builtin_ctz(xw);
                            xw &= xw - 1;
                            const uint32_t* row = F + (size_t)(wordidx * 32 + bit) * W;
                            if (own0) N0 |= row[lane];
                            if (own1) N1 |= row[lane + 64];
                        }
                    }
                }
                S0 = N0;
                S1 = N1;
                if (FIRST) {
                    const uint32_t sw = (uint32_t)__builtin_amdgcn_readlane((int)(aw < 64 ? S0 : S1), aw & 63);
                    if (sw & abit) pos = base + b + 1 - lo;
                }
            }
            const bool live = __ballot((S0 | S1) != 0) != 0;
            if (!live) { res = 0; break; }
            if (!FIRST && a.suffix_any) {
                const uint32_t sw = (uint32_t)__builtin_amdgcn_readlane((int)(aw < 64 ? S0 : S1), aw & 63);
                if (sw & abit) { res = 1; break; }
            }
        }
        if (ROWS) {   // the set reached; an absorbed accept stands alone
            uint32_t* o = a.rows_out + sid * W;
            if (own0) o[lane] = res == 1 ? (lane == aw ? abit : 0u) : S0;
            if (own1) o[lane + 64] = res == 1 ? (lane + 64 == aw ? abit : 0u) : S1;
            if (FIRST && lane == 0) a.first_pos[sid] = pos;
            continue;
        }
        if (FIRST) {
            if (lane == 0) a.first_pos[sid] = pos;
            continue;
        }
        if (res < 0) {
            const uint32_t sw = (uint32_t)__builtin_amdgcn_readlane((int)(aw < 64 ? S0 : S1), aw & 63);
            res = (sw & abit) ? 1 : 0;
        }
        if (lane == 0) a.out[sid] = (uint8_t)res;
    }
}

// One workgroup of WS wavefronts per string, for large sets and few strings
// (otherwise most SIMDs would sit idle).  Every wavefront keeps the whole set
// (lane j: words j and j + 64); per byte each takes the survivor words whose
// index is its own modulo WS, ORs their Follow rows (or chunk-union rows)
// into a partial next set, and the partials meet in LDS: the union of the
// images of a set's pointers is the image of the set (Def. 5.1).  One barrier
// per byte (the partials alternate between two LDS buffers).
template <bool TABLES_IN_LDS, int WS>
__global__ __launch_bounds__(64 * WS) void k_wave_split(KArgs a) {
    if (taken_by_sliced(a)) return;
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t part[2][WS][kWaveMaxWords];
    const int W = a.W, L = a.L;
    const uint32_t* M = a.bytemask;
    const uint32_t* F = a.follow;
    if (TABLES_IN_LDS) {
        uint32_t* Ml = lds;
        uint32_t* Fl = lds + 256 * W;
        for (int i = threadIdx.x; i < 256 * W; i += blockDim.x) Ml[i] = a.bytemask[i];
        for (int i = threadIdx.x; i < L * W; i += blockDim.x) Fl[i] = a.follow[i];
        __syncthreads();
        M = Ml;
        F = Fl;
    }
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool own0 = lane < W, own1 = lane + 64 < W;
    const int aw = L >> 5;
    const uint32_t abit = 1u << (L & 31);
    // survivor words this wavefront takes: word index (lane + 64 half) % WS == wave
    uint64_t mine[2] = {0, 0};
    for (int l = 0; l < 64; ++l) {
        if ((l % WS) == wave) mine[0] |= 1ull << l;
        if (((l + 64) % WS) == wave) mine[1] |= 1ull << l;
    }
    int parity = 0;
    for (int64_t sid = blockIdx.x; sid < a.n; sid += gridDim.x) {
        uint32_t S0 = own0 ? a.first[lane] : 0u;
        uint32_t S1 = own1 ? a.first[lane + 64] : 0u;
        const int64_t lo = a.offsets ? a.offsets[sid] : sid * a.stride;
        const int64_t hi = a.offsets ? a.offsets[sid + 1] : lo + a.stride;
        int res = -1;
        const int64_t skew = (int64_t)(reinterpret_cast<uintptr_t>(a.bytes) & 3);
        for (int64_t base = ((lo + skew) & ~int64_t(3)) - skew; base < hi && res < 0; base += 4) {
            const uint32_t word = *reinterpret_cast<const uint32_t*>(a.bytes + base);
            const int b0 = lo > base ? (int)(lo - base) : 0;
            const int b1 = hi - base < 4 ? (int)(hi - base) : 4;
            for (int b = b0; b < b1; ++b) {
                const uint32_t c = (word >> (8 * b)) & 255u;
                const uint32_t X0 = own0 ? (S0 & M[c * W + lane]) : 0u;
                const uint32_t X1 = own1 ? (S1 & M[c * W + 64 + lane]) : 0u;
                uint32_t N0 = 0, N1 = 0;
                for (int half = 0; half < 2; ++half) {
                    uint64_t nz = __ballot((half ? X1 : X0) != 0) & mine[half];
                    while (nz) {
                        const int wl = __builtin_ctzll(nz);
                        nz &= nz - 1;
                        uint32_t xw = (uint32_t)__builtin_amdgcn_readlane((int)(half ? X1 : X0), wl);
                        const int wordidx = wl + 64 * half;
                        if (a.chunks) {
                            const uint32_t* T = a.chunks + (size_t)wordidx * 4 * 256 * W;
                            const uint32_t* r0 = T + (size_t)(0 * 256 + ((xw >> 0) & 255u)) * W;
                            const uint32_t* r1 = T + (size_t)(1 * 256 + ((xw >> 8) & 255u)) * W;
                            const uint32_t* r2 = T + (size_t)(2 * 256 + ((xw >> 16) & 255u)) * W;
                            const uint32_t* r3 = T + (size_t)(3 * 256 + ((xw >> 24) & 255u)) * W;
                            if (own0) N0 |= (r0[lane] | r1[lane]) | (r2[lane] | r3[lane]);
                            if (own1) N1 |= (r0[lane + 64] | r1[lane + 64]) | (r2[lane + 64] | r3[lane + 64]);
                            continue;
                        }
                        while (xw) {
                            const int bit = __builtin_ctz(xw);
                            xw &= xw - 1;
                            const uint32_t* row = F + (size_t)(wordidx * 32 + bit) * W;
                            if (own0) N0 |= row[lane];
                            if (own1) N1 |= row[lane + 64];
                        }
                    }
                }
                // the partial sets meet: every wavefront leaves with the same S
                part[parity][wave][lane] = N0;
                part[parity][wave][lane + 64] = N1;
                __syncthreads();
                S0 = 0;
                S1 = 0;
#pragma unroll
                for (int w = 0; w < WS; ++w) {
                    S0 |= part[parity][w][lane];
                    S1 |= part[parity][w][lane + 64];
                }
                parity ^= 1;
            }
            const bool live = __ballot((S0 | S1) != 0) != 0;
            if (!live) { res = 0; break; }
            if (a.suffix_any) {
                const uint32_t sw = (uint32_t)__builtin_amdgcn_readlane((int)(aw < 64 ? S0 : S1), aw & 63);
                if (sw & abit) { res = 1; break; }
            }
        }
        if (res < 0) {
            const uint32_t sw = (uint32_t)__builtin_amdgcn_readlane((int)(aw < 64 ? S0 : S1), aw & 63);
            res = (sw & abit) ? 1 : 0;
        }
        if (threadIdx.x == 0) a.out[sid] = (uint8_t)res;
        // the next string's first byte reuses the buffers: no wavefront may still read them
        __syncthreads();
    }
}

KArgs kargs(const LaunchArgs& a) {
    KArgs k;
    k.first = a.first;
    k.follow = a.follow;
    k.bytemask = a.bytemask;
    k.chunks = a.chunks;
    k.L = a.L;
    k.W = a.W;
    k.suffix_any = a.suffix_any;
    k.pad = 0;
    k.bytes = a.bytes;
    k.offsets = a.offsets;
    k.stride = a.stride;
    k.n = a.n;
    k.out = a.out;
    k.first_pos = a.first_pos;
    k.rows_out = a.rows_out;
    k.rows_len = a.rows_len;
    k.rows_cl = a.rows_cl;
    k.rows_per_chunk = a.rows_per_chunk;
    k.rows_pad = 0;
    k.skip = a.skip;
    k.skip_id = a.skip_id;
    return k;
}

template <int W>
int launch_lane_w(const LaunchArgs& a) {
    const int block = a.block > 0 ? a.block : 256;
    int64_t need = (a.n + block - 1) / block;
    int grid = a.grid > 0 ? a.grid : (int)(need < (1 << 30) ? need : (1 << 30));
    if (grid < 1) grid = 1;
    const size_t lds = 4 * (size_t)(256 + a.L) * W;
    if (a.rows_out)
        if (a.first_pos)
            hipLaunchKernelGGL((k_lane<W, true, true>), dim3(grid), dim3(block), lds, (hipStream_t)a.stream, kargs(a));
        else
            hipLaunchKernelGGL((k_lane<W, false, true>), dim3(grid), dim3(block), lds, (hipStream_t)a.stream, kargs(a));
    else if (a.first_pos)
        hipLaunchKernelGGL((k_lane<W, true, false>), dim3(grid), dim3(block), lds, (hipStream_t)a.stream, kargs(a));
    else
        hipLaunchKernelGGL((k_lane<W, false, false>), dim3(grid), dim3(block), lds, (hipStream_t)a.stream, kargs(a));
    return (int)hipGetLastError();
}

}  // namespace

int launch_lane(const LaunchArgs& a) {
    switch (a.W) {
#define RX_LANE_CASE(w) \
    case w: return launch_lane_w<w>(a);
        RX_LANE_CASE(1) RX_LANE_CASE(2) RX_LANE_CASE(3) RX_LANE_CASE(4) RX_LANE_CASE(5) RX_LANE_CASE(6)
        RX_LANE_CASE(7) RX_LANE_CASE(8) RX_LANE_CASE(9) RX_LANE_CASE(10) RX_LANE_CASE(11) RX_LANE_CASE(12)
        RX_LANE_CASE(13) RX_LANE_CASE(14) RX_LANE_CASE(15) RX_LANE_CASE(16)
#undef RX_LANE_CASE
    default: return (int)hipErrorInvalidValue;
    }
}

namespace {
template <int WS>
int launch_wave_split(const LaunchArgs& a, size_t lds) {
    const int grid = (int)(a.n < (1 << 30) ? a.n : (1 << 30));
    // the tables go to LDS when they fit beside the partial sets (2 x WS x 512 bytes)
    const size_t cap = (size_t)(158 * 1024) - 2 * WS * kWaveMaxWords * 4 < (size_t)(150 * 1024)
                           ? (size_t)(158 * 1024) - 2 * WS * kWaveMaxWords * 4
                           : (size_t)(150 * 1024);
    if (lds <= cap) {
        static bool attr_set = false;
        if (!attr_set) {
            hipFuncSetAttribute((const void*)k_wave_split<true, WS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)cap);
            attr_set = true;
        }
        hipLaunchKernelGGL((k_wave_split<true, WS>), dim3(grid), dim3(64 * WS), lds, (hipStream_t)a.stream, kargs(a));
    } else {
        hipLaunchKernelGGL((k_wave_split<false, WS>), dim3(grid), dim3(64 * WS), 0, (hipStream_t)a.stream, kargs(a));
    }
    return (int)hipGetLastError();
}
}  // namespace

int launch_wave(const LaunchArgs& a) {
    const size_t lds_tables = 4 * (size_t)(256 + a.L) * a.W;
    if (!a.rows_out && !a.first_pos && a.n > 0) {
        // Few strings: several wavefronts per string keep the SIMDs busy.
        // rx_launch.unroll picks wavefronts per string (1, 2, 4, 8 or 16; 0 =
        // the most that leave every wavefront at least three set words and
        // put at most four wavefronts on a SIMD: the per-byte barrier costs
        // more than a wavefront with fewer words saves).
        int ws = a.unroll;
        if (ws == 0) {
            int cus = 0;
            if (hip_cu_count(&cus) || cus <= 0) cus = 256;
            const int64_t simds = 4 * (int64_t)cus;
            ws = 1;
            for (int c : {16, 8, 4, 2})
                if (a.n * c <= 4 * simds && 3 * c <= a.W) {
                    ws = c;
                    break;
                }
        }
        if (ws == 16) return launch_wave_split<16>(a, lds_tables);
        if (ws == 8) return launch_wave_split<8>(a, lds_tables);
        if (ws == 4) return launch_wave_split<4>(a, lds_tables);
        if (ws == 2) return launch_wave_split<2>(a, lds_tables);
    }
    const int block = a.block > 0 ? a.block : 256;
    const int waves = block / 64;
    int64_t need = (a.n + waves - 1) / waves;
    int grid = a.grid > 0 ? a.grid : (int)(need < (1 << 30) ? need : (1 << 30));
    if (grid < 1) grid = 1;
    const size_t lds = 4 * (size_t)(256 + a.L) * a.W;
    if (a.rows_out) {
        // many independent rows: tables through the caches, so more waves fit per CU
        if (a.first_pos)
            hipLaunchKernelGGL((k_wave<false, true, true>), dim3(grid), dim3(block), 0, (hipStream_t)a.stream, kargs(a));
        else
            hipLaunchKernelGGL((k_wave<false, false, true>), dim3(grid), dim3(block), 0, (hipStream_t)a.stream, kargs(a));
    } else if (lds <= 150 * 1024) {
        static bool attr_set = false;
        if (!attr_set) {
            hipFuncSetAttribute((const void*)k_wave<true, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024);
            hipFuncSetAttribute((const void*)k_wave<true, true, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                160 * 1024);
            attr_set = true;
        }
        if (a.first_pos)
            hipLaunchKernelGGL((k_wave<true, true, false>), dim3(grid), dim3(block), lds, (hipStream_t)a.stream, kargs(a));
        else
            hipLaunchKernelGGL((k_wave<true, false, false>), dim3(grid), dim3(block), lds, (hipStream_t)a.stream, kargs(a));
    } else if (a.first_pos) {
        hipLaunchKernelGGL((k_wave<false, true, false>), dim3(grid), dim3(block), 0, (hipStream_t)a.stream, kargs(a));
    } else {
        hipLaunchKernelGGL((k_wave<false, false, false>), dim3(grid), dim3(block), 0, (hipStream_t)a.stream, kargs(a));
    }
    return (int)hipGetLastError();
}

// Chunk-parallel matching, second pass: apply the chunks' relations in order.
// S starts as row 0 (chunk 0 run from First); for chunk c the new set is the
// union of the rows T_c[r] over the leaves r in S, because the byte step maps
// a union of thread sets to the union of their images (Def. 5.1 / 5.2: the
// evolution of a set is the union of the evolutions of its pointers).  One
// workgroup; exits early when S is empty or holds an absorbing accept.
__global__ __launch_bounds__(1024) void k_compose(const uint32_t* __restrict__ T, int64_t chunks, int32_t rpc,
                                                  int32_t W, int32_t L, int32_t suffix_any,
                                                  uint8_t* __restrict__ out) {
    __shared__ uint32_t S[kWaveMaxWords], N[kWaveMaxWords];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int aw = L >> 5;
    const uint32_t abit = 1u << (L & 31);
    for (int w = tid; w < W; w += nt) S[w] = T[w];
    __syncthreads();
    for (int64_t c = 1; c < chunks; ++c) {
        uint32_t any = 0;
        for (int w = 0; w < W; ++w) any |= S[w];
        if (any == 0) break;                          // no live thread: reject
        if (suffix_any && (S[aw] & abit)) break;      // accept is absorbing
        for (int w = tid; w < W; w += nt) N[w] = 0;
        __syncthreads();
        const uint32_t* rows = T + (1 + (c - 1) * (int64_t)rpc) * W;
        for (int r = tid; r < rpc; r += nt) {
            if (!((S[r >> 5] >> (r & 31)) & 1u)) continue;
            const uint32_t* row = rows + (int64_t)r * W;
            for (int w = 0; w < W; ++w) {
                const uint32_t v = row[w];
                if (v) atomicOr(&N[w], v);
            }
        }
        __syncthreads();
        for (int w = tid; w < W; w += nt) S[w] = N[w];
        __syncthreads();
    }
    if (tid == 0) out[0] = (S[aw] & abit) ? 1 : 0;
}

// The same for sets of at most 16 words (at most 512 rows per chunk): one row
// per thread, and each thread loads its row of the next chunk while the
// current chunk is applied, so the loads' latency is off the chain.
template <int W>
__global__ __launch_bounds__(512) void k_compose_lane(const uint32_t* __restrict__ T, int64_t chunks, int32_t rpc,
                                                      int32_t L, int32_t suffix_any, uint8_t* __restrict__ out) {
    __shared__ uint32_t S[W], N[W];
    const int tid = threadIdx.x;
    const bool own = tid < rpc;
    const int aw = L >> 5;
    const uint32_t abit = 1u << (L & 31);
    if (tid < W) S[tid] = T[tid];
    uint32_t cur[W];
#pragma unroll
    for (int w = 0; w < W; ++w) cur[w] = (own && chunks > 1) ? T[(1 + (int64_t)tid) * W + w] : 0u;
    __syncthreads();
    for (int64_t c = 1; c < chunks; ++c) {
        uint32_t nxt[W];
        const bool more = own && c + 1 < chunks;
        const uint32_t* nrow = T + (1 + c * (int64_t)rpc + tid) * W;
#pragma unroll
        for (int w = 0; w < W; ++w) nxt[w] = more ? nrow[w] : 0u;
        uint32_t any = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) any |= S[w];
        if (any == 0) break;                          // no live thread: reject
        if (suffix_any && (S[aw] & abit)) break;      // accept is absorbing
        if (tid < W) N[tid] = 0;
        __syncthreads();
        if (own && ((S[tid >> 5] >> (tid & 31)) & 1u)) {
#pragma unroll
            for (int w = 0; w < W; ++w)
                if (cur[w]) atomicOr(&N[w], cur[w]);
        }
        __syncthreads();
        if (tid < W) S[tid] = N[tid];
        __syncthreads();
#pragma unroll
        for (int w = 0; w < W; ++w) cur[w] = nxt[w];
    }
    if (tid == 0) out[0] = (S[aw] & abit) ? 1 : 0;
}

// The earliest accepting prefix of the whole string: chunk by chunk, the
// first chunk in which a live row meets an accept ends the search; the answer
// is the chunk's start plus the smallest such row offset (FP holds each row's
// bytes up to its first accept, -1 if none).
__global__ __launch_bounds__(1024) void k_compose_first(const uint32_t* __restrict__ T, const int64_t* __restrict__ FP,
                                                        int64_t chunks, int64_t cl, int32_t rpc, int32_t W,
                                                        int64_t* __restrict__ out) {
    __shared__ uint32_t S[kWaveMaxWords], N[kWaveMaxWords];
    __shared__ unsigned long long best;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int w = tid; w < W; w += nt) S[w] = T[w];
    if (tid == 0) best = ~0ull;
    __syncthreads();
    if (FP[0] >= 0) {                                 // inside chunk 0
        if (tid == 0) out[0] = FP[0];
        return;
    }
    for (int64_t c = 1; c < chunks; ++c) {
        uint32_t any = 0;
        for (int w = 0; w < W; ++w) any |= S[w];
        if (any == 0) break;                          // no live thread: no accept
        for (int w = tid; w < W; w += nt) N[w] = 0;
        __syncthreads();
        const uint32_t* rows = T + (1 + (c - 1) * (int64_t)rpc) * W;
        const int64_t* fps = FP + 1 + (c - 1) * (int64_t)rpc;
        for (int r = tid; r < rpc; r += nt) {
            if (!((S[r >> 5] >> (r & 31)) & 1u)) continue;
            const int64_t p = fps[r];
            if (p >= 0) atomicMin(&best, (unsigned long long)p);
            const uint32_t* row = rows + (int64_t)r * W;
            for (int w = 0; w < W; ++w) {
                const uint32_t v = row[w];
                if (v) atomicOr(&N[w], v);
            }
        }
        __syncthreads();
        const unsigned long long b = best;
        if (b != ~0ull) {                             // every thread reads the same value
            if (tid == 0) out[0] = c * cl + (int64_t)b;
            return;
        }
        for (int w = tid; w < W; w += nt) S[w] = N[w];
        __syncthreads();
    }
    if (tid == 0) out[0] = -1;
}

// Streaming copy (measurement only): the practical HBM ceiling and the
// calibration of byte counters against a kernel of known traffic.
__global__ __launch_bounds__(256) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

int launch_compose_first(const uint32_t* rows, const int64_t* fp, int64_t chunks, int64_t cl, int32_t rpc,
                         int32_t W, int64_t* out, void* stream) {
    int threads = ((rpc + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    hipLaunchKernelGGL(k_compose_first, dim3(1), dim3(threads), 0, (hipStream_t)stream, rows, fp, chunks, cl, rpc, W,
                       out);
    return (int)hipGetLastError();
}

int launch_compose(const uint32_t* rows, int64_t chunks, int32_t rpc, int32_t W, int32_t L, int32_t suffix_any,
                   uint8_t* out, void* stream) {
    int threads = ((rpc + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    if (W <= kLaneMaxWords && rpc <= 512) {
        switch (W) {
#define RX_COMPOSE_CASE(w)                                                                                        \
    case w:                                                                                                       \
        hipLaunchKernelGGL((k_compose_lane<w>), dim3(1), dim3(threads), 0, (hipStream_t)stream, rows, chunks, rpc, L, \
                           suffix_any, out);                                                                      \
        return (int)hipGetLastError();
            RX_COMPOSE_CASE(1) RX_COMPOSE_CASE(2) RX_COMPOSE_CASE(3) RX_COMPOSE_CASE(4) RX_COMPOSE_CASE(5)
            RX_COMPOSE_CASE(6) RX_COMPOSE_CASE(7) RX_COMPOSE_CASE(8) RX_COMPOSE_CASE(9) RX_COMPOSE_CASE(10)
            RX_COMPOSE_CASE(11) RX_COMPOSE_CASE(12) RX_COMPOSE_CASE(13) RX_COMPOSE_CASE(14) RX_COMPOSE_CASE(15)
            RX_COMPOSE_CASE(16)
#undef RX_COMPOSE_CASE
        default: break;
        }
    }
    hipLaunchKernelGGL(k_compose, dim3(1), dim3(threads), 0, (hipStream_t)stream, rows, chunks, rpc, W, L, suffix_any,
                       out);
    return (int)hipGetLastError();
}

int launch_stream_copy(void* dst, const void* src, int64_t bytes, void* stream) {
    const int64_t n16 = bytes / 16;
    int cus = 256;
    hip_cu_count(&cus);
    int64_t grid = (n16 + 255) / 256;
    if (grid > (int64_t)cus * 16) grid = (int64_t)cus * 16;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
    return (int)hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

int launch_fill_i64(int64_t* p, int64_t n, int64_t v, void* stream) {
    int64_t grid = (n + 255) / 256;
    if (grid > 4096) grid = 4096;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, p, n, v);
    return (int)hipGetLastError();
}

const char* hip_error_string(int err) { return hipGetErrorString((hipError_t)err); }

// Workspace of rx_match_long_noalloc: a file-scope device array, so the entry
// point allocates nothing.  In host code `scratch` only stands in for the
// symbol; its device address on each GPU comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address reaches a
// kernel.  Every call on a GPU shares the GPU's copy: calls that overlap on
// one GPU race.
static __device__ __align__(256) unsigned char scratch[kLongScratchBytes];

int long_scratch(void** ptr) {
    static std::mutex mu;
    static std::unordered_map<int, void*> by_device;
    int dev = -1;
    if (hipError_t e = hipGetDevice(&dev)) return (int)e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = by_device.find(dev);
    if (it == by_device.end()) {
        void* p = nullptr;
        if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        it = by_device.emplace(dev, p).first;
    }
    *ptr = it->second;
    return 0;
}

// Layout check of rx_match's strings, so that equal-length consecutive
// strings can go to the bit-sliced kernel without the host reading the
// offsets.  Each call takes the slot of its id (id modulo the slot count) in
// a static array per device: {id, length, first offset, flaw}.  The readers
// of a slot act only while it holds their id, so a later call that takes the
// same slot sends the earlier call's strings to the table form, which gives
// the same bits; ids only grow, so once a reader has seen another id every
// later reader of that call sees one too.
static __device__ __align__(256) int64_t layout_slots[kLayoutSlots * 4];

namespace {
__global__ void k_layout_begin(const int64_t* __restrict__ offsets, int64_t n, const uint8_t* bytes, int64_t* slot,
                               int64_t id) {
    const int64_t o0 = offsets[0], len = offsets[1] - o0;
    const bool ok = len > 0 && (len & 15) == 0 && len <= kLayoutMaxLength && offsets[n] - o0 == n * len &&
                    (reinterpret_cast<uintptr_t>(bytes + o0) & 15) == 0;
    slot[1] = len;
    slot[2] = o0;
    slot[3] = ok ? 0 : 1;
    slot[0] = id;
}

__global__ __launch_bounds__(256) void k_layout_check(const int64_t* __restrict__ offsets, int64_t n,
                                                      int64_t* slot, int64_t id) {
    if (slot[0] != id || slot[3] != 0) return;
    const int64_t len = slot[1], o0 = slot[2];
    bool flaw = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x)
        flaw |= offsets[i] != o0 + i * len;
    if (__any(flaw) && (threadIdx.x & 63) == 0)
        atomicOr(reinterpret_cast<unsigned long long*>(slot + 3), 1ull);
}
}  // namespace

int layout_slot(int64_t id, int64_t** slot) {
    static std::mutex mu;
    static std::unordered_map<int, int64_t*> by_device;
    int dev = -1;
    if (hipError_t e = hipGetDevice(&dev)) return (int)e;
    std::lock_guard<std::mutex> lk(mu);
    auto it = by_device.find(dev);
    if (it == by_device.end()) {
        void* p = nullptr;
        if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(layout_slots))) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        it = by_device.emplace(dev, static_cast<int64_t*>(p)).first;
    }
    *slot = it->second + (id % kLayoutSlots) * 4;
    return 0;
}

int launch_layout_check(const int64_t* offsets, int64_t n, const uint8_t* bytes, int64_t* slot, int64_t id,
                        void* stream) {
    hipLaunchKernelGGL(k_layout_begin, dim3(1), dim3(1), 0, (hipStream_t)stream, offsets, n, bytes, slot, id);
    const int64_t blocks = (n + 1 + 255) / 256;
    hipLaunchKernelGGL(k_layout_check, dim3((unsigned)(blocks < 2048 ? blocks : 2048)), dim3(256), 0,
                       (hipStream_t)stream, offsets, n, slot, id);
    return (int)hipGetLastError();
}

int hip_current_device(int* dev) { return (int)hipGetDevice(dev); }

int hip_memcpy_h2d_async(void* dst, const void* src, size_t n, void* stream) {
    return (int)hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, (hipStream_t)stream);
}

int hip_cu_count(int* cus) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    return (int)hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
}

}  // namespace rx
