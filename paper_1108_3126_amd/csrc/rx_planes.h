// Bit planes of a slab of strings, for the plane form of the bit-sliced
// circuit (host/device neutral: the device build maps RX_PL_PERM, RX_PL_SEL
// and RX_PL_ALIGN to single gfx950 instructions; a host build may define them
// as plain C to test this file).
//
// A slab is 2048 strings; lane l (0..63) of a wavefront carries strings
// 64 j + l in bit j (j = 0..31).  Tick t is positions 4t .. 4t+3 and holds 36
// words per lane: word 8i + b = bit b of the byte at position 4t + i, word
// 32 + i = the strings whose length exceeds 4t + i.  Stored as nine groups
// of four words, group q of lane l of tick t at u32 index ((t*9 + q)*64 + l)*4.
#pragma once

#include <cstdint>

#ifndef RX_PL_DEV
#define RX_PL_DEV __device__ __forceinline__
#endif
#ifndef RX_PL_PERM   // byte i of the result = byte sel_i of the 64-bit value {hi, lo}
#define RX_PL_PERM(hi, lo, sel) __builtin_amdgcn_perm((hi), (lo), (sel))
#endif
#ifndef RX_PL_SEL    // (a & m) | (b & ~m): 0xE4 is that function on the patterns a=0xF0, b=0xCC, m=0xAA
#define RX_PL_SEL(a, b, m) __builtin_amdgcn_bitop3_b32((a), (b), (m), 0xE4)
#endif
#ifndef RX_PL_ALIGN  // low 32 bits of {hi, lo} >> (8 * r), r = 0..3
#define RX_PL_ALIGN(hi, lo, r) __builtin_amdgcn_alignbyte((hi), (lo), (r))
#endif

namespace rx {

constexpr int kPlaneTickWords = 36;   // words per lane per tick
constexpr int kSlabStrings = 2048;

// 32 x 32 bit transpose: bit k of a[j] moves to bit j of a[k].  Five stages
// swap off-diagonal blocks of 16, 8, 4, 2 and 1 bits; the first two move
// whole bytes (one byte permute per word), the last three use a shift and a
// bit select per word.
RX_PL_DEV void planes_transpose32(uint32_t (&a)[32]) {
    // 16-bit blocks: a[j] (j < 16) keeps its low halves and takes a[j+16]'s low half
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t lo = a[j], hi = a[j + 16];
        a[j] = RX_PL_PERM(hi, lo, 0x05040100u);        // {hi.low16, lo.low16}
        a[j + 16] = RX_PL_PERM(hi, lo, 0x07060302u);   // {hi.high16, lo.high16}
    }
    // 8-bit blocks within each 16-bit half
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        if (j & 8) continue;
        const uint32_t lo = a[j], hi = a[j + 8];
        a[j] = RX_PL_PERM(hi, lo, 0x06020400u);
        a[j + 8] = RX_PL_PERM(hi, lo, 0x07030501u);
    }
    // 4-, 2- and 1-bit blocks
#pragma unroll
    for (int st = 0; st < 3; ++st) {
        const int d = 4 >> st;
        const uint32_t m = st == 0 ? 0x0f0f0f0fu : st == 1 ? 0x33333333u : 0x55555555u;
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            if (j & d) continue;
            const uint32_t x = a[j], y = a[j + d];
            a[j] = RX_PL_SEL(x, y << d, m);
            a[j + d] = RX_PL_SEL(x >> d, y, m);
        }
    }
}

// Bytes [off, off + 16) of a string that starts at `s` and has `len` bytes,
// little-endian in four words (bytes at or past len are unspecified).  Only
// 16-byte aligned blocks that hold at least one byte of the string are read,
// so no access leaves the string's own pages.
RX_PL_DEV void planes_window16(const uint8_t* s, int64_t len, int64_t off, uint32_t (&w)[4]) {
    w[0] = w[1] = w[2] = w[3] = 0u;
    if (off >= len) return;
    const uintptr_t addr = reinterpret_cast<uintptr_t>(s + off);
    const uintptr_t end = reinterpret_cast<uintptr_t>(s + len);
    const uintptr_t a = addr & ~(uintptr_t)15;
    const uint32_t sh = (uint32_t)(addr & 15);
    uint32_t b[8];
    {
        const uint32_t* p0 = reinterpret_cast<const uint32_t*>(a);
        b[0] = p0[0];
        b[1] = p0[1];
        b[2] = p0[2];
        b[3] = p0[3];
    }
    if (a + 16 < end) {
        const uint32_t* p1 = reinterpret_cast<const uint32_t*>(a + 16);
        b[4] = p1[0];
        b[5] = p1[1];
        b[6] = p1[2];
        b[7] = p1[3];
    } else {
        b[4] = b[5] = b[6] = b[7] = 0u;
    }
    // whole words first (sh / 4 of them), then the remaining bytes
    if (sh & 8) {
#pragma unroll
        for (int k = 0; k < 6; ++k) b[k] = b[k + 2];
    }
    if (sh & 4) {
#pragma unroll
        for (int k = 0; k < 5; ++k) b[k] = b[k + 1];
    }
    const uint32_t r = sh & 3;
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = RX_PL_ALIGN(b[k + 1], b[k], r);
}

// The strings of a slab whose length exceeds position p: bit j for len[j] > p.
template <class LT>
RX_PL_DEV uint32_t planes_valid(const LT (&len)[32], int64_t p) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < 32; ++j) v |= (len[j] > p ? 1u : 0u) << j;
    return v;
}

// Tick words of one lane from the 16-byte windows of its 32 strings: tick k
// (0..3) of the windows, i.e. positions off + 4k .. off + 4k + 3.  minlen is
// a lower bound of every length (whole words of ones below it).
template <class LT>
RX_PL_DEV void planes_tick(const uint32_t (&win)[32][4], const LT (&len)[32], int k, int64_t pos0,
                           int64_t minlen, uint32_t (&out)[kPlaneTickWords]) {
    uint32_t x[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) x[j] = win[j][k];
    planes_transpose32(x);
    // after the transpose x[8i + b] is bit b of byte i of every string
#pragma unroll
    for (int i = 0; i < 32; ++i) out[i] = x[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) out[32 + i] = pos0 + i < minlen ? 0xffffffffu : planes_valid(len, pos0 + i);
}

}  // namespace rx
