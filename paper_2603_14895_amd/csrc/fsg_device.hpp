// fsg_device.hpp -- device building blocks of the propagation step on gfx950:
// the counter-based generator, bit-sliced replicate counters and 64-lane
// wavefront helpers.  Replicates are packed 64 to a uint64 word: bit b of
// word w of a node is replicate 64*w + b of the batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsg {

constexpr uint32_t kAlways = 0xFFFFFFFFu;
constexpr uint32_t kDomIcEdge = 1u;
constexpr uint32_t kDomNodeStep = 2u;
constexpr uint32_t kDomLtThresh = 3u;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products on counter words 0 and 2, the high halves mixed
// into words 1 and 3 with the key; the key advances by the Weyl constants
// between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

// Three-input bitwise functions in one gfx950 instruction per 32 bits
// (truth tables: 0x96 = a ^ b ^ c, 0xE8 = majority).  The builtin returns a
// signed int: it goes through uint32_t before any widening.
__device__ __forceinline__ uint32_t xor3_32(uint32_t a, uint32_t b, uint32_t c)
{
    return (uint32_t)__builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint32_t maj3_32(uint32_t a, uint32_t b, uint32_t c)
{
    return (uint32_t)__builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
}

__device__ __forceinline__ uint64_t xor3(uint64_t a, uint64_t b, uint64_t c)
{
    return (uint64_t)xor3_32((uint32_t)a, (uint32_t)b, (uint32_t)c) |
           ((uint64_t)xor3_32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32)) << 32);
}

__device__ __forceinline__ uint64_t maj3(uint64_t a, uint64_t b, uint64_t c)
{
    return (uint64_t)maj3_32((uint32_t)a, (uint32_t)b, (uint32_t)c) |
           ((uint64_t)maj3_32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32)) << 32);
}

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_32((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3_32((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t pick(const U4 &o, uint32_t i)
{
    return i == 0 ? o.x : (i == 1 ? o.y : (i == 2 ? o.z : o.w));
}

__device__ __forceinline__ bool fires(uint32_t u, uint32_t t) { return t == kAlways || u < t; }

// Valid replicate bits of word w for a batch of B replicates.
__device__ __forceinline__ uint64_t tail_mask(int64_t w, int64_t B)
{
    const int64_t valid = B - 64 * w;
    if (valid >= 64) return ~0ull;
    if (valid <= 0) return 0ull;
    return (1ull << valid) - 1ull;
}

// Bits of the word that share one generator block with bit b: a block holds
// the four global replicates 4j .. 4j+3; gbase is the global index of bit 0.
__device__ __forceinline__ uint64_t block_bits(uint64_t gbase, int b)
{
    const int start = b - (int)((gbase + (uint64_t)b) & 3u);
    return start >= 0 ? (0xFull << start) : (0xFull >> (-start));
}

// Bits of the word whose generator block index is congruent to s mod S
// (S a power of two): the share of lane s when S lanes split the draws.
__device__ __forceinline__ uint64_t share_bits(uint64_t gbase, int s, int S)
{
    if (S == 1) return ~0ull;
    uint64_t m = 0;
    const uint64_t b0 = gbase >> 2, b1 = (gbase + 63) >> 2;
    for (uint64_t blk = b0; blk <= b1; ++blk) {
        if ((int)(blk & (uint64_t)(S - 1)) != s) continue;
        const int lo = (int)((int64_t)(blk * 4) - (int64_t)gbase);
        m |= lo >= 0 ? (lo < 64 ? (0xFull << lo) : 0ull) : (0xFull >> (-lo));
    }
    return m;
}

// Value of lane J of the caller's 16-lane row (DPP row broadcast); every lane
// of the row must be active.
template <int J>
__device__ __forceinline__ uint32_t row_bcast(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x150 + J, 0xF, 0xF, false);
}

// ---- bit-sliced counters: c[l] holds bit l of 64 per-replicate counts ----

template <int L>
__device__ __forceinline__ void bs_add1(uint64_t (&c)[L], uint64_t x)
{
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const uint64_t t = c[l] & x;
        c[l] ^= x;
        x = t;
        if (!x) break;
    }
}

// Four one-bit addends at once with carry-save adders: two full adders at
// level 0, one at level 1, and a ripple from level 2 only when a carry
// reaches it (a full adder: sum = a ^ b ^ x, carry = majority(a, b, x)).
template <int L>
__device__ __forceinline__ void bs_add4(uint64_t (&c)[L], uint64_t x0, uint64_t x1, uint64_t x2,
                                        uint64_t x3)
{
    const uint64_t s0 = xor3(c[0], x0, x1);
    const uint64_t k1a = maj3(c[0], x0, x1);
    c[0] = xor3(s0, x2, x3);
    if (L == 1) return;
    const uint64_t k1b = maj3(s0, x2, x3);
    uint64_t k2 = maj3(c[1], k1a, k1b);
    c[1] = xor3(c[1], k1a, k1b);
    if (k2) {
#pragma unroll
        for (int l = 2; l < L; ++l) {
            const uint64_t t = c[l] & k2;
            c[l] ^= k2;
            k2 = t;
            if (!k2) break;
        }
    }
}

template <int L>
__device__ __forceinline__ void bs_add(uint64_t (&c)[L], const uint64_t (&d)[L])
{
    uint64_t carry = 0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const uint64_t a = c[l], b = d[l];
        c[l] = xor3(a, b, carry);
        carry = maj3(a, b, carry);
    }
}

template <int L>
__device__ __forceinline__ uint32_t bs_get(const uint64_t (&c)[L], int b)
{
    uint32_t k = 0;
#pragma unroll
    for (int l = 0; l < L; ++l) k |= (uint32_t)((c[l] >> b) & 1ull) << l;
    return k;
}

template <int L>
__device__ __forceinline__ uint64_t bs_nonzero(const uint64_t (&c)[L])
{
    uint64_t m = 0;
#pragma unroll
    for (int l = 0; l < L; ++l) m |= c[l];
    return m;
}

// Loads through a uniform base and a 32-bit byte offset (the compiler then
// uses scalar-base addressing with a 32-bit vector offset).
__device__ __forceinline__ uint64_t ld64_off32(const uint64_t *base, uint32_t idx)
{
    return *reinterpret_cast<const uint64_t *>(reinterpret_cast<const char *>(base) + (idx << 3));
}

__device__ __forceinline__ int ld32_off32(const int32_t *base, uint32_t idx)
{
    return *reinterpret_cast<const int32_t *>(reinterpret_cast<const char *>(base) + (idx << 2));
}

// Masks of the replicates whose count is 1, 2 or 3 (the common case), so
// most per-replicate counts are read with a select instead of L extractions.
struct SmallCounts {
    uint64_t m1, m2, m3;
};

template <int L>
__device__ __forceinline__ SmallCounts bs_small(const uint64_t (&c)[L])
{
    uint64_t rest = 0;
#pragma unroll
    for (int l = 2; l < L; ++l) rest |= c[l];
    const uint64_t c0 = c[0], c1 = L > 1 ? c[1] : 0ull;
    return SmallCounts{c0 & ~c1 & ~rest, ~c0 & c1 & ~rest, c0 & c1 & ~rest};
}

template <int L>
__device__ __forceinline__ uint32_t bs_get_fast(const uint64_t (&c)[L], const SmallCounts &sm, int b)
{
    if ((sm.m1 >> b) & 1ull) return 1u;
    if ((sm.m2 >> b) & 1ull) return 2u;
    if ((sm.m3 >> b) & 1ull) return 3u;
    return bs_get<L>(c, b);
}

// The four bits of x that belong to the generator block starting at bit gs
// (gs in [-3, 63]; bits outside the word read as 0), as a nibble.
__device__ __forceinline__ uint32_t nibble_at(uint64_t x, int gs)
{
    return (uint32_t)((gs >= 0 ? (x >> gs) : (x << (-gs))) & 0xFull);
}

// A nibble placed back at the block position gs.
__device__ __forceinline__ uint64_t nibble_to_word(uint32_t nib, int gs)
{
    const uint64_t x = (uint64_t)(nib & 0xFu);
    return gs >= 0 ? (x << gs) : (x >> (-gs));
}

// Sum of the counters held by the lanes lane ^ k*G, k < S (butterfly over
// the edge-split lanes); every lane of the group ends with the total.
template <int L>
__device__ __forceinline__ void bs_reduce_lanes(uint64_t (&c)[L], int G, int S)
{
    for (int off = G; off < G * S; off <<= 1) {
        uint64_t d[L];
#pragma unroll
        for (int l = 0; l < L; ++l) d[l] = __shfl_xor(c[l], off, 64);
        bs_add<L>(c, d);
    }
}

__device__ __forceinline__ uint64_t or_reduce_lanes(uint64_t x, int G, int S)
{
    for (int off = G; off < G * S; off <<= 1) x |= __shfl_xor(x, off, 64);
    return x;
}

}  // namespace fsg
