// The node-per-thread machine: the paper's own GPU realisation of lockstep
// matching (Rathnayake & Thielecke, SOS 2011, §8, with the process
// translation of §7), run as one persistent launch.
//
// Every node d[i] of the heap is a small process owned by one thread.  Two
// stamp vectors c and n (one entry per node, plus one for null) carry the
// messages of a macro step:
//   * c[i] holds the stamp of the current step: node i has been sent a
//     message and is to be simulated now;
//   * a simulated node is marked consumed, so a process takes one message
//     per macro step (receivers are not replicated);
//   * simulating a node sends its messages on c: alt -> both children,
//     cat / plus -> the first child, star / opt / plus-loop -> the child and
//     cont, eps -> cont (the translation of §7, with the companion rules
//     for plus and opt);
//   * a leaf whose label holds the next input byte sends to its cont on n,
//     which is the synchronised move on that byte;
//   * a message to null is kept as the null entry's stamp; the string is
//     accepted when null has been sent a message once the input is spent.
// A macro step repeats rounds of simulation until a round sends no new
// message on c (the shared activity flag), then swaps c and n and advances
// the step count.  The step stamps replace the paper's t / -t encoding:
// step t schedules with 2t+2 and marks consumed with 2t+3, and messages are
// LDS atomic maxima, so a message can never revive a receiver that has
// already run in this step, and old stamps never need clearing.  Every
// thread of the workgroup takes the same decisions (another round, another
// step), so the barriers always match: round g reports activity in slot
// g & 1, which is next written two rounds later, after every thread has read
// it; the move flag n only grows, and a later step writes it only when every
// thread has seen it set.
//
// Layout: one workgroup per string (persistent, grid-stride), one thread per
// node up to 1024 nodes and several nodes per thread beyond; both stamp
// vectors in LDS (16 bytes per node); node records and classes read from the
// image through the caches.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

#include "rx_internal.h"

namespace rx {

namespace {

struct NodeRec {
    int32_t kl;     // kind | label << 8 (byte value or class index)
    int32_t c0, c1, cont;
};

typedef unsigned long long u64;

__device__ __forceinline__ void send(u64* c, int q, int m, u64 S, u64 g, u64* act) {   // act: the activity slot of this pass
    if (q == -2) return;                               // no message
    const int idx = q < 0 ? m : q;                     // -1: null
    if (atomicMax(&c[idx], S) < S) *act = g;           // a fresh receiver: another pass is needed
}

__global__ __launch_bounds__(1024) void k_nodes(const int32_t* __restrict__ image, const uint8_t* __restrict__ bytes,
                                                const int64_t* __restrict__ offsets, int64_t stride, int64_t n,
                                                uint8_t* __restrict__ out) {
    extern __shared__ u64 stamps[];   // vectors A and B, m + 1 entries each; entry m is null
    __shared__ u64 act[2];            // round g writes g into act[g & 1] when it schedules a node on c
    __shared__ u64 nact;              // stamp of the last move sent on n
    const int m = image[0];
    const NodeRec* __restrict__ nodes = reinterpret_cast<const NodeRec*>(image + 4);
    const uint32_t* __restrict__ classes = reinterpret_cast<const uint32_t*>(image + 4 + 4 * m);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int64_t s = blockIdx.x; s < n; s += gridDim.x) {
        const int64_t lo = offsets ? offsets[s] : s * stride;
        const int64_t len = (offsets ? offsets[s + 1] : (s + 1) * stride) - lo;
        __syncthreads();   // the previous string's final reads are done
        for (int i = tid; i < 2 * (m + 1); i += nt) stamps[i] = 0;
        if (tid == 0) { act[0] = 0; act[1] = 0; nact = 0; }
        __syncthreads();
        u64* c = stamps;
        u64* nx = stamps + (m + 1);
        u64 S = 2, g = 0;
        if (tid == 0) c[0] = S;   // the root process receives the first message
        __syncthreads();
        bool accept = false;
        for (int64_t t = 0;; ++t) {
            const int b = t < len ? bytes[lo + t] : -1;
            for (;;) {   // rounds of the current macro step
                ++g;
                u64* const a = &act[g & 1];
                for (int i = tid; i < m; i += nt) {
                    if (c[i] != S) continue;
                    c[i] = S + 1;   // consumed for this step
                    const NodeRec r = nodes[i];
                    const int kind = r.kl & 0xff;
                    switch (kind) {
                    case RX_ALT: send(c, r.c0, m, S, g, a); send(c, r.c1, m, S, g, a); break;
                    case RX_CAT:
                    case RX_PLUS: send(c, r.c0, m, S, g, a); break;
                    case RX_STAR:
                    case RX_OPT:
                    case RX_PLUSLOOP: send(c, r.c0, m, S, g, a); send(c, r.cont, m, S, g, a); break;
                    case RX_EPS: send(c, r.cont, m, S, g, a); break;
                    default: {   // leaf: the synchronised move on the next byte
                        if (b < 0) break;
                        const int lab = r.kl >> 8;
                        const bool hit = kind == RX_BYTE ? lab == b : ((classes[lab * 8 + (b >> 5)] >> (b & 31)) & 1u);
                        if (hit) {
                            nx[r.cont < 0 ? m : r.cont] = S + 2;
                            nact = S + 2;
                        }
                    }
                    }
                }
                __syncthreads();
                if (*a != g) break;   // no node was scheduled in this pass: the step is quiescent
            }
            if (t == len) {   // input spent: accept iff null has received a message
                accept = c[m] >= S;
                break;
            }
            if (nact < S + 2) break;   // no thread survived the move on this byte
            u64* tmp = c;
            c = nx;
            nx = tmp;
            S += 2;
        }
        if (tid == 0) out[s] = accept ? 1 : 0;
    }
}

}  // namespace

void node_image(const Program* P, std::vector<uint8_t>& img) {
    const int32_t m = P->m;
    const int32_t ncls = (int32_t)P->classes.size();
    img.assign(16 + 16 * (size_t)m + 32 * (size_t)ncls, 0);
    int32_t head[4] = {m, ncls, 0, 0};
    std::memcpy(img.data(), head, 16);
    for (int32_t i = 0; i < m; ++i) {
        const int32_t lab = P->label[i] < 0 ? 0 : P->label[i];
        const int32_t rec[4] = {P->kind[i] | (lab << 8), P->c0[i], P->c1[i], P->cont[i]};
        std::memcpy(img.data() + 16 + 16 * (size_t)i, rec, 16);
    }
    for (int32_t k = 0; k < ncls; ++k) {
        uint32_t w[8];
        for (int j = 0; j < 4; ++j) {
            w[2 * j] = (uint32_t)P->classes[k][j];
            w[2 * j + 1] = (uint32_t)(P->classes[k][j] >> 32);
        }
        std::memcpy(img.data() + 16 + 16 * (size_t)m + 32 * (size_t)k, w, 32);
    }
}

int launch_nodes(const void* image, int32_t m, const uint8_t* bytes, const int64_t* offsets, int64_t stride, int64_t n,
                 uint8_t* out, void* stream) {
    int threads = ((m + 63) / 64) * 64;
    if (threads > 1024) threads = 1024;
    if (threads < 64) threads = 64;
    const int64_t grid = n < 4096 ? n : 4096;
    const size_t lds = 2 * sizeof(u64) * ((size_t)m + 1);
    static bool attr = false;   // allow more than 64 KiB of dynamic LDS (set once; a failure only limits m)
    if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nodes), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(2 * sizeof(u64) * (kNodesMaxNodes + 1)));
        attr = true;
    }
    hipLaunchKernelGGL(k_nodes, dim3((unsigned)grid), dim3(threads), lds, (hipStream_t)stream,
                       static_cast<const int32_t*>(image), bytes, offsets, stride, n, out);
    return (int)hipGetLastError();
}

}  // namespace rx
