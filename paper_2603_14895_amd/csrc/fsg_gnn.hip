// fsg_gnn.hip -- learned surrogate of the Monte Carlo SIR spread: a
// mean-aggregation message-passing network (the message / aggregate / update
// structure of Eq. ms, Eq. agg, Eq. updata, here with learned functions),
// BF16 weights and activations with FP32 accumulation on MFMA, trained on the
// simulator's own Monte Carlo output by hand-written forward and backward
// kernels and Adam.
//
// Network (per node v, per seed set s; R = n_sets * n rows):
//   x_v  = [seed_v, 20 beta, log1p(indeg_v) / 8, 1,
//           20 beta log1p(indeg_v) / 8, log1p(k_s) / 8, log1p(D_s) / 16, 0 ... 0]
//                                                                   (16 wide)
//   with k_s the number of seeds of the set and D_s the sum of their
//   in-degrees (query-wide terms: a node further than three hops from every
//   seed sees the seed set only through them)
//   h1_v = ReLU(W1 [x_v | mean_{u in N-(v)} x_u] + b1)            (32 -> 64)
//   h2_v = ReLU(W2 [h1_v | mean h1_u] + b2)                        (128 -> 64)
//   h3_v = ReLU(W3 [h2_v | mean h2_u] + b3)                        (128 -> 64)
//   p_v  = sigmoid(wo . h3_v + bo)
// Loss: mean binary cross-entropy against per-node infection frequencies.
// A mean over an empty neighbourhood is 0.  Every stored BF16 value of the
// forward pass is its defining expression rounded once (to nearest even,
// through FP32): the means exactly so (FP64 sums), the layer outputs up to
// the FP32 rounding of the MFMA sums.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/fsg.h"
#include "fsg_internal.hpp"

namespace fsg {
namespace gnn {

constexpr int kF0 = 16;   // input features (padded)
constexpr int kHid = 64;  // hidden width
constexpr int kK1 = 2 * kF0, kK2 = 2 * kHid;
// flat FP32 parameter layout
constexpr int kW1 = 0, kB1 = kW1 + kK1 * kHid, kW2 = kB1 + kHid, kB2 = kW2 + kK2 * kHid,
              kW3 = kB2 + kHid, kB3 = kW3 + kK2 * kHid, kWo = kB3 + kHid, kBo = kWo + kHid,
              kP = kBo + 1;
// BF16 copies of W1, W2, W3 ([K][64] row-major each)
constexpr int kWb1 = 0, kWb2 = kWb1 + kK1 * kHid, kWb3 = kWb2 + kK2 * kHid,
              kWbN = kWb3 + kK2 * kHid;
constexpr int kPartBlocks = 512;  // fixed grid of reduction kernels (deterministic sums)
constexpr int kDwRows = 1024;     // rows per block of the weight-gradient GEMM
constexpr int kMaxMembers = 64;   // ensemble members one spread estimate may combine

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t to_bf16(float f)
{
    union {
        float f;
        uint32_t u;
    } x;
    x.f = f;
    if ((x.u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((x.u >> 16) | ((x.u & 0xFFFF) ? 0x40 : 0));
    x.u += 0x7FFFu + ((x.u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(x.u >> 16);
}

__host__ __device__ inline float from_bf16(uint16_t h)
{
    union {
        uint32_t u;
        float f;
    } x;
    x.u = (uint32_t)h << 16;
    return x.f;
}

// ------------------------------------------------------------- kernels ----

// Query-wide terms of seed set s (one block per set): qs[2s] = number of
// seeds, qs[2s+1] = sum of their in-degrees.  Integer sums, so the result
// does not depend on the order of the additions.
constexpr int kQueryThreads = 1024;

__global__ void __launch_bounds__(kQueryThreads) k_query_stats(const uint8_t *mask,
                                                               const int32_t *ptr, int32_t n,
                                                               unsigned long long *qs)
{
    const int s = blockIdx.x;
    const uint8_t *m = mask + (int64_t)s * n;
    unsigned long long k = 0, d = 0;
    for (int v = threadIdx.x; v < n; v += blockDim.x)
        if (m[v]) {
            ++k;
            d += (unsigned long long)(ptr[v + 1] - ptr[v]);
        }
    for (int off = 32; off >= 1; off >>= 1) {
        k += __shfl_xor(k, off, 64);
        d += __shfl_xor(d, off, 64);
    }
    __shared__ unsigned long long sk[kQueryThreads / 64], sd[kQueryThreads / 64];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sk[wave] = k;
        sd[wave] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tk = 0, td = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            tk += sk[w];
            td += sd[w];
        }
        qs[2 * s] = tk;
        qs[2 * s + 1] = td;
    }
}

// Input features of every (seed set, node) row into X1[:, 0:16].
__global__ void k_input(uint16_t *X1, const uint8_t *mask, const float *beta, const int32_t *ptr,
                        const unsigned long long *qs, int32_t n, int32_t n_sets)
{
    const int64_t R = (int64_t)n * n_sets;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int s = (int)(r / n);
        const int v = (int)(r - (int64_t)s * n);
        const int d = ptr[v + 1] - ptr[v];
        const double xb = 20.0 * (double)beta[s], xd = log1p((double)d) * 0.125;
        uint16_t *x = X1 + r * kK1;
        x[0] = to_bf16(mask[r] ? 1.f : 0.f);
        x[1] = to_bf16((float)xb);
        x[2] = to_bf16((float)xd);
        x[3] = to_bf16(1.f);
        x[4] = to_bf16((float)(xb * xd));
        x[5] = to_bf16((float)(log1p((double)qs[2 * s]) * 0.125));
        x[6] = to_bf16((float)(log1p((double)qs[2 * s + 1]) * 0.0625));
        for (int f = 7; f < kF0; ++f) x[f] = 0;
    }
}

// Adds the four BF16 values packed in q to four FP64 sums (exactly: a BF16
// value widens to FP64 without rounding).
__device__ __forceinline__ void add_bf16x4(double &a0, double &a1, double &a2, double &a3,
                                           uint2 q)
{
    a0 += (double)from_bf16((uint16_t)q.x);
    a1 += (double)from_bf16((uint16_t)(q.x >> 16));
    a2 += (double)from_bf16((uint16_t)q.y);
    a3 += (double)from_bf16((uint16_t)(q.y >> 16));
}

// BF16 of sum / deg: FP64 quotient, rounded to FP32, then to BF16 (nearest
// even at both steps); 0 for an empty neighbourhood.
__device__ __forceinline__ uint16_t mean_bf16(double sum, int deg)
{
    return deg > 0 ? to_bf16((float)(sum / (double)deg)) : (uint16_t)0;
}

// Mean aggregation over in-neighbours (pull CSR), BF16 result:
// X[r][cout + f] = mean_{u in N-(v)} X[s*n + u][cin + f], f < d (d = 16 or 64).
// The BF16 neighbour values are added in FP64, which holds such a sum
// exactly (8-bit significands: exact while the values span fewer than about
// 2^40 and the row has fewer than 2^5 ... 2^31 entries), and divided by the
// degree in FP64; the quotient goes to FP32 and then to BF16, both rounding
// to nearest even.  The stored mean is therefore the exact mean rounded as
// the definition rounds it, whatever the order of the additions.  (An FP32
// sum scaled by a rounded 1/deg lands on the other side of a BF16 tie now and
// then; those one-unit flips then reach every later layer.)
// One wave per row.  A lane covers 4 features (one 8-byte load per
// neighbour), so d/4 lanes cover a neighbour row and the wave has 64/(d/4)
// neighbour rows in flight per load; neighbour indices arrive 64 at a time
// with one coalesced load and reach the lanes by shuffle.  The lane groups'
// partial sums are added at the end (fixed order).
__device__ __forceinline__ void mean_light(uint16_t *X, int ld, int d, int cin, int cout,
                                           const int32_t *ptr, const int32_t *src, int32_t n,
                                           int32_t n_sets, int64_t wave, int64_t nwave)
{
    const int lane = threadIdx.x & 63;
    const int lg = d >> 2, ng = 64 / lg;
    const int gi = lane / lg, li = lane - gi * lg;
    const int64_t R = (int64_t)n * n_sets;
    for (int64_t r = wave; r < R; r += nwave) {
        const int s = (int)(r / n);
        const int v = (int)(r - (int64_t)s * n);
        const int e0 = ptr[v], e1 = ptr[v + 1], deg = e1 - e0;
        if (deg > kWideRow) continue;  // k_mean_wide
        const uint16_t *base = X + (int64_t)s * n * ld + cin + 4 * li;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        for (int c0 = 0; c0 < deg; c0 += 64) {
            const int cnt = min(64, deg - c0);
            const int my = lane < cnt ? src[e0 + c0 + lane] : 0;
            for (int k0 = 0; k0 < cnt; k0 += 2 * ng) {
                const int ka = k0 + gi, kb = k0 + ng + gi;
                const int ua = __shfl(my, ka & 63, 64), ub = __shfl(my, kb & 63, 64);
                uint2 qa = make_uint2(0u, 0u), qb = make_uint2(0u, 0u);
                if (ka < cnt) qa = *reinterpret_cast<const uint2 *>(base + (int64_t)ua * ld);
                if (kb < cnt) qb = *reinterpret_cast<const uint2 *>(base + (int64_t)ub * ld);
                add_bf16x4(a0, a1, a2, a3, qa);
                add_bf16x4(a0, a1, a2, a3, qb);
            }
        }
        for (int off = lg; off < 64; off <<= 1) {
            a0 += __shfl_xor(a0, off, 64);
            a1 += __shfl_xor(a1, off, 64);
            a2 += __shfl_xor(a2, off, 64);
            a3 += __shfl_xor(a3, off, 64);
        }
        if (gi == 0) {
            uint2 o;
            o.x = (uint32_t)mean_bf16(a0, deg) | ((uint32_t)mean_bf16(a1, deg) << 16);
            o.y = (uint32_t)mean_bf16(a2, deg) | ((uint32_t)mean_bf16(a3, deg) << 16);
            *reinterpret_cast<uint2 *>(X + r * ld + cout + 4 * li) = o;
        }
    }
}

// Transpose of the mean aggregation (backward): for row (s, u),
// dH[r][f] = dX[r][f] + sum_{v : u in N-(v)} dX[s*n + v][64 + f] / indeg(v),
// pulled over the out-arcs of u (the in-CSR of the reversed graph).  One wave
// per row: 16 lanes (one float4 each) per neighbour row, four rows in flight.
__global__ void __launch_bounds__(256) k_mean_bwd(float *dH, const float *dX, const int32_t *ptr,
                                                  const int32_t *rptr, const int32_t *rdst,
                                                  int32_t n, int32_t n_sets)
{
    const int lane = threadIdx.x & 63;
    const int gi = lane >> 4, li = lane & 15;
    const int64_t R = (int64_t)n * n_sets;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = wave; r < R; r += nwave) {
        const int s = (int)(r / n);
        const int u = (int)(r - (int64_t)s * n);
        const int e0 = rptr[u], deg = rptr[u + 1] - e0;
        if (deg > kWideRow) continue;  // k_mean_bwd_wide
        const float *blk = dX + (int64_t)s * n * kK2 + kHid + 4 * li;
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int c0 = 0; c0 < deg; c0 += 64) {
            const int cnt = min(64, deg - c0);
            const int my = lane < cnt ? rdst[e0 + c0 + lane] : 0;
            for (int k0 = 0; k0 < cnt; k0 += 4) {
                const int k = k0 + gi;
                const int v = __shfl(my, k & 63, 64);
                if (k < cnt) {
                    const float4 q = *reinterpret_cast<const float4 *>(blk + (int64_t)v * kK2);
                    const float w = 1.f / (float)(ptr[v + 1] - ptr[v]);
                    acc.x += q.x * w;
                    acc.y += q.y * w;
                    acc.z += q.z * w;
                    acc.w += q.w * w;
                }
            }
        }
        for (int off = 16; off < 64; off <<= 1) {
            acc.x += __shfl_xor(acc.x, off, 64);
            acc.y += __shfl_xor(acc.y, off, 64);
            acc.z += __shfl_xor(acc.z, off, 64);
            acc.w += __shfl_xor(acc.w, off, 64);
        }
        if (gi == 0) {
            const float4 self = *reinterpret_cast<const float4 *>(dX + r * kK2 + 4 * li);
            *reinterpret_cast<float4 *>(dH + r * kHid + 4 * li) =
                make_float4(self.x + acc.x, self.y + acc.y, self.z + acc.z, self.w + acc.w);
        }
    }
}

// The same aggregations for rows with more than kWideRow arcs: one block of
// kWideThreads per (seed set, wide row); wave w takes the w-th contiguous
// slice of the row's arcs, and the waves' sums are added in wave order.
constexpr int kWideThreads = 1024;
constexpr int kWideWaves = kWideThreads / 64;

__device__ __forceinline__ void mean_wide(uint16_t *X, int ld, int d, int cin, int cout,
                                          const int32_t *ptr, const int32_t *src, int32_t n,
                                          const int32_t *wide, int32_t n_wide, int blk,
                                          double (*s_part)[kHid])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lg = d >> 2, ng = 64 / lg;
    const int gi = lane / lg, li = lane - gi * lg;
    const int s = blk / n_wide;
    const int v = wide[blk - s * n_wide];
    const int e0 = ptr[v], deg = ptr[v + 1] - e0;
    const int per = (deg + kWideWaves - 1) / kWideWaves;
    const int lo = min(deg, wv * per), hi = min(deg, lo + per);
    const uint16_t *base = X + (int64_t)s * n * ld + cin + 4 * li;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int c0 = lo; c0 < hi; c0 += 64) {
        const int cnt = min(64, hi - c0);
        const int my = lane < cnt ? src[e0 + c0 + lane] : 0;
        for (int k0 = 0; k0 < cnt; k0 += 2 * ng) {
            const int ka = k0 + gi, kb = k0 + ng + gi;
            const int ua = __shfl(my, ka & 63, 64), ub = __shfl(my, kb & 63, 64);
            uint2 qa = make_uint2(0u, 0u), qb = make_uint2(0u, 0u);
            if (ka < cnt) qa = *reinterpret_cast<const uint2 *>(base + (int64_t)ua * ld);
            if (kb < cnt) qb = *reinterpret_cast<const uint2 *>(base + (int64_t)ub * ld);
            add_bf16x4(a0, a1, a2, a3, qa);
            add_bf16x4(a0, a1, a2, a3, qb);
        }
    }
    for (int off = lg; off < 64; off <<= 1) {
        a0 += __shfl_xor(a0, off, 64);
        a1 += __shfl_xor(a1, off, 64);
        a2 += __shfl_xor(a2, off, 64);
        a3 += __shfl_xor(a3, off, 64);
    }
    if (gi == 0) {
        s_part[wv][4 * li] = a0;
        s_part[wv][4 * li + 1] = a1;
        s_part[wv][4 * li + 2] = a2;
        s_part[wv][4 * li + 3] = a3;
    }
    __syncthreads();
    if ((int)threadIdx.x < d) {
        double acc = 0.0;
        for (int w = 0; w < kWideWaves; ++w) acc += s_part[w][threadIdx.x];
        X[((int64_t)s * n + v) * ld + cout + threadIdx.x] = mean_bf16(acc, deg);
    }
}

__global__ void __launch_bounds__(256) k_mean(uint16_t *X, int ld, int d, int cin, int cout,
                                              const int32_t *ptr, const int32_t *src, int32_t n,
                                              int32_t n_sets)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    mean_light(X, ld, d, cin, cout, ptr, src, n, n_sets, wave, nwave);
}

__global__ void __launch_bounds__(kWideThreads) k_mean_wide(uint16_t *X, int ld, int d, int cin,
                                                            int cout, const int32_t *ptr,
                                                            const int32_t *src, int32_t n,
                                                            const int32_t *wide, int32_t n_wide)
{
    __shared__ double s_part[kWideWaves][kHid];
    mean_wide(X, ld, d, cin, cout, ptr, src, n, wide, n_wide, (int)blockIdx.x, s_part);
}

// Forward mean aggregation in one launch: the first n_wide * n_sets blocks
// take the wide rows (largest first), the rest the other rows one wave each,
// so the long rows run alongside the short ones.
__global__ void __launch_bounds__(kWideThreads) k_mean_all(uint16_t *X, int ld, int d, int cin,
                                                           int cout, const int32_t *ptr,
                                                           const int32_t *src, int32_t n,
                                                           int32_t n_sets, const int32_t *wide,
                                                           int32_t n_wide)
{
    __shared__ double s_part[kWideWaves][kHid];
    const int nwb = n_wide * n_sets;
    if ((int)blockIdx.x < nwb) {
        mean_wide(X, ld, d, cin, cout, ptr, src, n, wide, n_wide, (int)blockIdx.x, s_part);
        return;
    }
    const int64_t wave = ((int64_t)(blockIdx.x - nwb) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)(gridDim.x - nwb) * blockDim.x) >> 6;
    mean_light(X, ld, d, cin, cout, ptr, src, n, n_sets, wave, nwave);
}

__global__ void __launch_bounds__(kWideThreads) k_mean_bwd_wide(float *dH, const float *dX,
                                                                const int32_t *ptr,
                                                                const int32_t *rptr,
                                                                const int32_t *rdst, int32_t n,
                                                                const int32_t *wide,
                                                                int32_t n_wide)
{
    __shared__ float s_part[kWideWaves][kHid];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int gi = lane >> 4, li = lane & 15;
    const int s = blockIdx.x / n_wide;
    const int u = wide[blockIdx.x - s * n_wide];
    const int e0 = rptr[u], deg = rptr[u + 1] - e0;
    const int per = (deg + kWideWaves - 1) / kWideWaves;
    const int lo = min(deg, wv * per), hi = min(deg, lo + per);
    const float *blk = dX + (int64_t)s * n * kK2 + kHid + 4 * li;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int c0 = lo; c0 < hi; c0 += 64) {
        const int cnt = min(64, hi - c0);
        const int my = lane < cnt ? rdst[e0 + c0 + lane] : 0;
        for (int k0 = 0; k0 < cnt; k0 += 4) {
            const int k = k0 + gi;
            const int v = __shfl(my, k & 63, 64);
            if (k < cnt) {
                const float4 q = *reinterpret_cast<const float4 *>(blk + (int64_t)v * kK2);
                const float w = 1.f / (float)(ptr[v + 1] - ptr[v]);
                acc.x += q.x * w;
                acc.y += q.y * w;
                acc.z += q.z * w;
                acc.w += q.w * w;
            }
        }
    }
    for (int off = 16; off < 64; off <<= 1) {
        acc.x += __shfl_xor(acc.x, off, 64);
        acc.y += __shfl_xor(acc.y, off, 64);
        acc.z += __shfl_xor(acc.z, off, 64);
        acc.w += __shfl_xor(acc.w, off, 64);
    }
    if (gi == 0) {
        s_part[wv][4 * li] = acc.x;
        s_part[wv][4 * li + 1] = acc.y;
        s_part[wv][4 * li + 2] = acc.z;
        s_part[wv][4 * li + 3] = acc.w;
    }
    __syncthreads();
    if ((int)threadIdx.x < kHid) {
        const int64_t r = (int64_t)s * n + u;
        float a = dX[r * kK2 + threadIdx.x];
        for (int w = 0; w < kWideWaves; ++w) a += s_part[w][threadIdx.x];
        dH[r * kHid + threadIdx.x] = a;
    }
}

// Out[r][0:64] = act(A[r][0:K] . W[0:K][0:64] + bias) on MFMA (16x16x16 BF16,
// FP32 accumulation).  One wave: 16 rows x 64 columns; block: 64 rows.
// W staged in LDS.  relu: 1 -> ReLU and BF16 store to out16, 0 -> FP32 store
// to out32 without bias.
__global__ void __launch_bounds__(256) k_gemm_fwd(const uint16_t *A, int lda, int K,
                                                  const uint16_t *Wb, const float *bias,
                                                  uint16_t *out16, int ldo, int64_t R)
{
    __shared__ uint16_t sW[kK2 * kHid];
    for (int i = threadIdx.x; i < K * kHid; i += blockDim.x) sW[i] = Wb[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int li = lane & 15, lk = lane >> 4;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int64_t ra = r0 + li;
    for (int kb = 0; kb < K; kb += 16) {
        bf16x4 a = (bf16x4){0, 0, 0, 0};
        if (ra < R) {
            const uint16_t *pa = A + ra * lda + kb + 4 * lk;
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = (short)pa[j];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            bf16x4 b;
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = (short)sW[(kb + 4 * lk + j) * kHid + t * 16 + li];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = r0 + 4 * lk + i;
            const int col = t * 16 + li;
            if (row < R) {
                float v = acc[t][i] + bias[col];
                out16[row * ldo + col] = to_bf16(v > 0.f ? v : 0.f);
            }
        }
    }
}

// dX[r][0:K] = dZ[r][0:64] . W^T with W = [K][64]; FP32 out.  One wave:
// 16 rows x K columns.
__global__ void __launch_bounds__(256) k_gemm_dx(const uint16_t *dZ, const uint16_t *Wb, int K,
                                                 float *dX, int64_t R)
{
    __shared__ uint16_t sW[kK2 * kHid];
    for (int i = threadIdx.x; i < K * kHid; i += blockDim.x) sW[i] = Wb[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64 + wave * 16;
    const int li = lane & 15, lk = lane >> 4;
    const int ntiles = K / 16;  // <= 8
    f32x4 acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int64_t ra = r0 + li;
#pragma unroll
    for (int kb = 0; kb < kHid; kb += 16) {
        bf16x4 a = (bf16x4){0, 0, 0, 0};
        if (ra < R) {
            const uint16_t *pa = dZ + ra * kHid + kb + 4 * lk;
#pragma unroll
            for (int j = 0; j < 4; ++j) a[j] = (short)pa[j];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (t >= ntiles) break;
            bf16x4 b;  // B[k][c] = W[c][k]
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = (short)sW[(t * 16 + li) * kHid + kb + 4 * lk + j];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        if (t >= ntiles) break;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = r0 + 4 * lk + i;
            if (row < R) dX[row * K + t * 16 + li] = acc[t][i];
        }
    }
}

// Partial weight gradient of one block of kDwRows rows: part[blk][k][c] =
// sum_rows X[row][k] dZ[row][c] on MFMA (the rows are the contraction).  Row
// chunks of 64 are staged in LDS; wave w owns feature tiles w, w+4, ...
__global__ void __launch_bounds__(256) k_gemm_dw(const uint16_t *X, int ldx, int K,
                                                 const uint16_t *dZ, float *part, int64_t R)
{
    __shared__ uint16_t sX[64 * kK2];
    __shared__ uint16_t sZ[64 * kHid];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int mtiles = K / 16;  // 2 or 8
    f32x4 acc[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[m][t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int64_t rb0 = (int64_t)blockIdx.x * kDwRows;
    for (int64_t c0 = rb0; c0 < rb0 + kDwRows && c0 < R; c0 += 64) {
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * K; i += blockDim.x) {
            const int rr = i / K, kk = i - rr * K;
            sX[i] = (c0 + rr < R) ? X[(c0 + rr) * ldx + kk] : (uint16_t)0;
        }
        for (int i = threadIdx.x; i < 64 * kHid; i += blockDim.x) {
            const int rr = i / kHid;
            sZ[i] = (c0 + rr < R) ? dZ[(c0 + rr) * kHid + (i - rr * kHid)] : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 64; ks += 16) {  // 16 rows per MFMA
            bf16x4 b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) b[t][j] = (short)sZ[(ks + 4 * lk + j) * kHid + t * 16 + li];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int mt = wave + 4 * m;
                if (mt >= mtiles) break;
                bf16x4 a;  // A[feature][row] = X[row][feature]
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = (short)sX[(ks + 4 * lk + j) * K + mt * 16 + li];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[t], acc[m][t], 0, 0, 0);
            }
        }
    }
    float *pb = part + (int64_t)blockIdx.x * K * kHid;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int mt = wave + 4 * m;
        if (mt >= mtiles) break;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) pb[(mt * 16 + 4 * lk + i) * kHid + t * 16 + li] = acc[m][t][i];
    }
}

// out[i] = scale * sum_b part[b][i] (fixed order).
__global__ void k_reduce(const float *part, int nb, int len, float *out, float scale)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int b = 0; b < nb; ++b) s += part[(int64_t)b * len + i];
        out[i] = s * scale;
    }
}

// Output layer and loss.  p = sigmoid(wo . h3 + bo); with targets:
// dz = (p - y) / R, dH3 = dz wo, and per-block partial sums of dz h3 (for
// wo), dz (for bo) and the cross-entropy (stable form from the logit).
__global__ void __launch_bounds__(256) k_head(const uint16_t *H3, const float *wo, const float *bo,
                                              const float *y, float *prob, float *dH3,
                                              float *part_wo, float *part_bo, float *part_loss,
                                              int64_t R)
{
    __shared__ float s_wo[4][kHid];
    __shared__ float s_b[4][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float w = wo[lane];
    const float b = bo[0];
    float gw = 0.f, gb = 0.f, ls = 0.f;
    for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < R; r += (int64_t)gridDim.x * 4) {
        const float h = from_bf16(H3[r * kHid + lane]);
        float z = h * w;
        for (int off = 32; off >= 1; off >>= 1) z += __shfl_xor(z, off, 64);
        z += b;
        const float p = 1.f / (1.f + expf(-z));
        if (lane == 0) prob[r] = p;
        if (y) {
            const float t = y[r];
            const float dz = (p - t) / (float)R;
            dH3[r * kHid + lane] = dz * w;
            gw += dz * h;
            gb += dz;
            ls += fmaxf(z, 0.f) - z * t + log1pf(expf(-fabsf(z)));
        }
    }
    if (!y) return;
    s_wo[wave][lane] = gw;
    if (lane == 0) {
        s_b[wave][0] = gb;
        s_b[wave][1] = ls;
    }
    __syncthreads();
    if (wave == 0) {
        part_wo[blockIdx.x * kHid + lane] = s_wo[0][lane] + s_wo[1][lane] + s_wo[2][lane] + s_wo[3][lane];
        if (lane == 0) {
            part_bo[blockIdx.x] = s_b[0][0] + s_b[1][0] + s_b[2][0] + s_b[3][0];
            part_loss[blockIdx.x] = s_b[0][1] + s_b[1][1] + s_b[2][1] + s_b[3][1];
        }
    }
}

// dZ = BF16(dH * [H > 0]) and per-block partial sums of dZ (bias gradient).
__global__ void __launch_bounds__(256) k_dz(const float *dH, const uint16_t *H, int ldh,
                                            uint16_t *dZ, float *part_b, int64_t R)
{
    __shared__ float s[4][kHid];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float acc = 0.f;
    for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < R; r += (int64_t)gridDim.x * 4) {
        const float g = from_bf16(H[r * ldh + lane]) > 0.f ? dH[r * kHid + lane] : 0.f;
        const uint16_t gb = to_bf16(g);
        dZ[r * kHid + lane] = gb;
        acc += from_bf16(gb);
    }
    s[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) part_b[blockIdx.x * kHid + lane] = s[0][lane] + s[1][lane] + s[2][lane] + s[3][lane];
}

// Adam (Kingma and Ba, ICLR 2015, Algorithm 1) on the FP32 master
// parameters, every operation rounded to FP32 (no contraction; division and
// square root correctly rounded):
//   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
//   p = p - lr (m / c1) / (sqrt(v / c2) + eps),  c1 = 1 - b1^t, c2 = 1 - b2^t,
// then the BF16 copies of W1..W3.
__global__ void k_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2, uint16_t *wb)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * (gi * gi);
        m[i] = mi;
        v[i] = vi;
        const float upd = (mi / c1) / (sqrtf(vi / c2) + eps);
        const float pi = p[i] - lr * upd;
        p[i] = pi;
        if (i < kB1) wb[kWb1 + i] = to_bf16(pi);
        else if (i >= kW2 && i < kB2) wb[kWb2 + (i - kW2)] = to_bf16(pi);
        else if (i >= kW3 && i < kB3) wb[kWb3 + (i - kW3)] = to_bf16(pi);
    }
}

__global__ void k_params_to_bf16(const float *p, uint16_t *wb)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kWbN; i += gridDim.x * blockDim.x) {
        float x;
        if (i < kWb2) x = p[kW1 + i];
        else if (i < kWb3) x = p[kW2 + (i - kWb2)];
        else x = p[kW3 + (i - kWb3)];
        wb[i] = to_bf16(x);
    }
}

// Per-set sums of the node probabilities (the predicted spread) in a fixed
// order: block b of set s
// sums rows [b c, (b+1) c) of the set (c = ceil(n / kSumParts)) into
// part[s][b]; k_set_final then adds the kSumParts partials of each set.
constexpr int kSumParts = 128;

__global__ void __launch_bounds__(256) k_set_part(const float *prob, int32_t n, float *part)
{
    __shared__ float s[256];
    const int set = blockIdx.x / kSumParts, b = blockIdx.x - set * kSumParts;
    const int c = (n + kSumParts - 1) / kSumParts;
    const int lo = min(n, b * c), hi = min(n, lo + c);
    float acc = 0.f;
    for (int v = lo + (int)threadIdx.x; v < hi; v += blockDim.x) acc += prob[(int64_t)set * n + v];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(kSumParts) k_set_final(const float *part, float *out)
{
    __shared__ float s[kSumParts];
    s[threadIdx.x] = part[blockIdx.x * kSumParts + threadIdx.x];
    __syncthreads();
    for (int off = kSumParts / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

__global__ void k_mask_clear(uint8_t *mask, int32_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        mask[i] = 0;
}

__global__ void k_mask_set(uint8_t *mask, const int32_t *seeds, int64_t ns)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns;
         i += (int64_t)gridDim.x * blockDim.x)
        mask[seeds[i]] = 1;
}

}  // namespace gnn
}  // namespace fsg

using namespace fsg;
using namespace fsg::gnn;

// ------------------------------------------------------------------ host ----

struct fsg_gnn {
    int32_t hidden = kHid, layers = 3;
    uint64_t seed = 0;
    std::vector<float> init;
    bool bound = false;
    char *state = nullptr;  // device: params, m, v, grads (FP32 [P] each), BF16 weights
    int64_t step = 0;
    float last_loss = 0.f;
    float *p() const { return (float *)state; }
    float *m() const { return (float *)state + kP; }
    float *v() const { return (float *)state + 2 * kP; }
    float *g() const { return (float *)state + 3 * kP; }
    uint16_t *wb() const { return (uint16_t *)((float *)state + 4 * kP); }
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

#define GNN_TRY(expr)                                                                 \
    do {                                                                              \
        if (fsg::inject_device_fault())                                                       \
            return set_error(FSG_EDEVICE, (std::string(#expr) + ": injected fault").c_str()); \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return set_error(FSG_EDEVICE, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

unsigned grid_of(int64_t work, int block, int cap = 65536)
{
    int64_t g = (work + block - 1) / block;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Workspace of one forward/backward pass over R rows.
struct GnnWs {
    size_t X1, X2, X3, H3, prob, dH, dH2, dZ, dX, part, pwo, pbo, ploss, beta, qstat, sums, mask,
        seeds, total;
};

GnnWs gnn_layout(int64_t n, int32_t n_sets)
{
    GnnWs w;
    const size_t R = (size_t)n * (size_t)n_sets;
    const size_t dw_blocks = (R + kDwRows - 1) / kDwRows;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = al256(off + std::max<size_t>(bytes, 4));
        return o;
    };
    w.X1 = take(R * kK1 * 2);
    w.X2 = take(R * kK2 * 2);
    w.X3 = take(R * kK2 * 2);
    w.H3 = take(R * kHid * 2);
    w.prob = take(R * 4);
    w.dH = take(R * kHid * 4);
    w.dH2 = take(R * kHid * 4);
    w.dZ = take(R * kHid * 2);
    w.dX = take(R * kK2 * 4);
    w.part = take(std::max<size_t>(dw_blocks * kK2 * kHid, (size_t)kPartBlocks * kHid) * 4);
    w.pwo = take((size_t)kPartBlocks * kHid * 4);
    w.pbo = take((size_t)kPartBlocks * 4);
    w.ploss = take((size_t)kPartBlocks * 4);
    w.beta = take((size_t)n_sets * 4);
    w.qstat = take((size_t)n_sets * 16);
    w.sums = take((size_t)std::max<int32_t>(n_sets, kMaxMembers) * 4);
    w.mask = take((size_t)n);
    w.seeds = take((size_t)n * 4);
    w.total = off;
    return w;
}

uint64_t splitmix(uint64_t &x)
{
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct GraphView {
    int64_t n = 0, nnz = 0, dmax = 0, n_wide = 0;
    const int32_t *ptr = nullptr, *src = nullptr, *wide = nullptr;
};

int view_of(const fsg_graph *g, GraphView *v, const char *what)
{
    if (!graph_view(g, &v->n, &v->nnz, &v->dmax, &v->ptr, &v->src, &v->wide, &v->n_wide))
        return set_error(FSG_EINVAL, (std::string(what) + " is NULL or not bound").c_str());
    return FSG_OK;
}

// Mean aggregation of one layer: light rows one wave each, wide rows one
// block each.
int mean_agg(uint16_t *X, int ld, int d, const GraphView &G, int32_t n_sets, hipStream_t st)
{
    const int64_t R = G.n * n_sets;
    if (n_sets == 1) {  // one query: the hubs overlap the short rows in one launch
        const unsigned nwb = (unsigned)G.n_wide;
        hipLaunchKernelGGL(k_mean_all, dim3(nwb + grid_of(R * 64, kWideThreads)),
                           dim3(kWideThreads), 0, st, X, ld, d, 0, d, G.ptr, G.src, (int32_t)G.n,
                           n_sets, G.wide, (int32_t)G.n_wide);
        GNN_TRY(hipGetLastError());
        return FSG_OK;
    }
    // many seed sets (training): short rows fill the GPU on their own
    hipLaunchKernelGGL(k_mean, dim3(grid_of(R * 64, 256)), dim3(256), 0, st, X, ld, d, 0, d,
                       G.ptr, G.src, (int32_t)G.n, n_sets);
    GNN_TRY(hipGetLastError());
    if (G.n_wide > 0) {
        hipLaunchKernelGGL(k_mean_wide, dim3((unsigned)(G.n_wide * n_sets)), dim3(kWideThreads), 0,
                           st, X, ld, d, 0, d, G.ptr, G.src, (int32_t)G.n, G.wide,
                           (int32_t)G.n_wide);
        GNN_TRY(hipGetLastError());
    }
    return FSG_OK;
}

// Forward pass of all layers; probabilities into ws.prob (R rows).
int forward_all(const fsg_gnn *gn, const GraphView &G, int32_t n_sets, const uint8_t *mask,
                char *base, const GnnWs &w, hipStream_t st)
{
    const int64_t R = G.n * n_sets;
    uint16_t *X1 = (uint16_t *)(base + w.X1), *X2 = (uint16_t *)(base + w.X2),
             *X3 = (uint16_t *)(base + w.X3), *H3 = (uint16_t *)(base + w.H3);
    const float *P = gn->p();
    const uint16_t *Wb = gn->wb();
    unsigned long long *qs = (unsigned long long *)(base + w.qstat);
    hipLaunchKernelGGL(k_query_stats, dim3((unsigned)n_sets), dim3(kQueryThreads), 0, st, mask,
                       G.ptr, (int32_t)G.n, qs);
    GNN_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_input, dim3(grid_of(R, 256)), dim3(256), 0, st, X1, mask,
                       (const float *)(base + w.beta), G.ptr, (const unsigned long long *)qs,
                       (int32_t)G.n, n_sets);
    GNN_TRY(hipGetLastError());
    int rc = mean_agg(X1, kK1, kF0, G, n_sets, st);
    if (rc) return rc;
    const unsigned gg = (unsigned)((R + 63) / 64);
    hipLaunchKernelGGL(k_gemm_fwd, dim3(gg), dim3(256), 0, st, X1, kK1, kK1, Wb + kWb1, P + kB1, X2,
                       kK2, R);
    GNN_TRY(hipGetLastError());
    rc = mean_agg(X2, kK2, kHid, G, n_sets, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_gemm_fwd, dim3(gg), dim3(256), 0, st, X2, kK2, kK2, Wb + kWb2, P + kB2, X3,
                       kK2, R);
    GNN_TRY(hipGetLastError());
    rc = mean_agg(X3, kK2, kHid, G, n_sets, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_gemm_fwd, dim3(gg), dim3(256), 0, st, X3, kK2, kK2, Wb + kWb3, P + kB3, H3,
                       kHid, R);
    GNN_TRY(hipGetLastError());
    return FSG_OK;
}

// Backward of one layer with input Xin (ld K) and output H (post-ReLU, ld
// ldh): dZ from dH, bias and weight gradients into the gradient vector, and
// (if dHin) the gradient of the layer input through W^T and the transposed
// mean aggregation.
int backward_layer(const fsg_gnn *gn, const GraphView &G, const GraphView &Gr, int32_t n_sets,
                   char *base, const GnnWs &w, const uint16_t *Xin, int K, const uint16_t *H,
                   int ldh, const float *dH, int wofs, int bofs, int wbofs, float *dHin,
                   hipStream_t st)
{
    const int64_t R = G.n * n_sets;
    uint16_t *dZ = (uint16_t *)(base + w.dZ);
    float *part = (float *)(base + w.part);
    float *grads = gn->g();
    hipLaunchKernelGGL(k_dz, dim3(kPartBlocks), dim3(256), 0, st, dH, H, ldh, dZ, part, R);
    GNN_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(64), 0, st, (const float *)part, kPartBlocks, kHid,
                       grads + bofs, 1.f);
    GNN_TRY(hipGetLastError());
    const int nb = (int)((R + kDwRows - 1) / kDwRows);
    hipLaunchKernelGGL(k_gemm_dw, dim3((unsigned)nb), dim3(256), 0, st, Xin, K, K,
                       (const uint16_t *)dZ, part, R);
    GNN_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(grid_of(K * kHid, 256)), dim3(256), 0, st, (const float *)part,
                       nb, K * kHid, grads + wofs, 1.f);
    GNN_TRY(hipGetLastError());
    if (dHin) {
        float *dX = (float *)(base + w.dX);
        hipLaunchKernelGGL(k_gemm_dx, dim3((unsigned)((R + 63) / 64)), dim3(256), 0, st,
                           (const uint16_t *)dZ, gn->wb() + wbofs, K, dX, R);
        GNN_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_mean_bwd, dim3(grid_of(R * 64, 256)), dim3(256), 0, st, dHin,
                           (const float *)dX, G.ptr, Gr.ptr, Gr.src, (int32_t)G.n, n_sets);
        GNN_TRY(hipGetLastError());
        if (Gr.n_wide > 0) {
            hipLaunchKernelGGL(k_mean_bwd_wide, dim3((unsigned)(Gr.n_wide * n_sets)),
                               dim3(kWideThreads), 0, st, dHin, (const float *)dX, G.ptr, Gr.ptr,
                               Gr.src, (int32_t)G.n, Gr.wide, (int32_t)Gr.n_wide);
            GNN_TRY(hipGetLastError());
        }
    }
    return FSG_OK;
}

int check_ws(void *ws, size_t bytes, size_t need)
{
    if (!ws || bytes < need) return set_error(FSG_EWORKSPACE, "gnn workspace too small");
    if (((uintptr_t)ws & 255) != 0) return set_error(FSG_EWORKSPACE, "workspace not 256-byte aligned");
    return FSG_OK;
}

// One Adam step (step count t = ++g->step) with gradient grads (device [kP]).
int adam_enqueue(fsg_gnn *g, const float *grads, float lr, hipStream_t st)
{
    g->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    // 1 - beta^t: beta^t rounded once to FP32 (powf is correctly rounded)
    const float c1 = 1.f - powf(b1, (float)g->step), c2 = 1.f - powf(b2, (float)g->step);
    hipLaunchKernelGGL(k_adam, dim3(grid_of(kP, 256)), dim3(256), 0, st, g->p(), grads, g->m(),
                       g->v(), (int)kP, lr, b1, b2, 1e-8f, c1, c2, g->wb());
    GNN_TRY(hipGetLastError());
    return FSG_OK;
}

int upload_betas(const float *beta, int32_t n_sets, char *base, const GnnWs &w, hipStream_t st)
{
    for (int32_t i = 0; i < n_sets; ++i)
        if (!(beta[i] >= 0.f && beta[i] <= 1.f)) return set_error(FSG_EINVAL, "beta outside [0, 1]");
    GNN_TRY(hipMemcpyAsync(base + w.beta, beta, (size_t)n_sets * 4, hipMemcpyHostToDevice, st));
    return FSG_OK;
}

}  // namespace

extern "C" {

int fsg_gnn_create(int32_t hidden, int32_t layers, uint64_t init_seed, fsg_gnn **out)
{
    try {
        if (!out) return set_error(FSG_EINVAL, "out is NULL");
        *out = nullptr;
        if (hidden != kHid || layers != 3)
            return set_error(FSG_EUNSUPPORTED, "this build has hidden = 64 and 3 layers");
        fsg::inject_alloc_fault();
        fsg_gnn *g = new fsg_gnn;
        g->seed = init_seed;
        g->init.assign(kP, 0.f);
        uint64_t x = init_seed;
        auto fill = [&](int off, int fan_in, int count) {  // uniform(-a, a), a = sqrt(6 / (fan_in + 64))
            const float a = sqrtf(6.f / (float)(fan_in + kHid));
            for (int i = 0; i < count; ++i) {
                const double u = (double)(splitmix(x) >> 11) * (1.0 / 9007199254740992.0);
                g->init[(size_t)(off + i)] = (float)((2.0 * u - 1.0) * a);
            }
        };
        fill(kW1, kK1, kK1 * kHid);
        fill(kW2, kK2, kK2 * kHid);
        fill(kW3, kK2, kK2 * kHid);
        fill(kWo, kHid, kHid);
        *out = g;
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return set_error(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_gnn_destroy(fsg_gnn *g)
{
    delete g;
    return FSG_OK;
}

int fsg_gnn_param_count(const fsg_gnn *g, int64_t *count)
{
    if (!g || !count) return set_error(FSG_EINVAL, "NULL argument");
    *count = kP;
    return FSG_OK;
}

int fsg_gnn_state_size(const fsg_gnn *g, size_t *bytes)
{
    if (!g || !bytes) return set_error(FSG_EINVAL, "NULL argument");
    *bytes = al256((size_t)4 * kP * 4 + (size_t)kWbN * 2);
    return FSG_OK;
}

int fsg_gnn_bind(fsg_gnn *g, void *dev_state, size_t bytes, void *stream)
{
    if (!g) return set_error(FSG_EINVAL, "gnn is NULL");
    size_t need = 0;
    fsg_gnn_state_size(g, &need);
    int rc = check_ws(dev_state, bytes, need);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    g->state = (char *)dev_state;
    GNN_TRY(hipMemcpyAsync(g->p(), g->init.data(), (size_t)kP * 4, hipMemcpyHostToDevice, st));
    GNN_TRY(hipMemsetAsync(g->m(), 0, (size_t)3 * kP * 4, st));
    hipLaunchKernelGGL(k_params_to_bf16, dim3(grid_of(kWbN, 256)), dim3(256), 0, st,
                       (const float *)g->p(), g->wb());
    GNN_TRY(hipGetLastError());
    GNN_TRY(hipStreamSynchronize(st));
    g->bound = true;
    g->step = 0;
    return FSG_OK;
}

int fsg_gnn_workspace_size(const fsg_gnn *g, const fsg_graph *graph, int32_t n_sets, size_t *bytes)
{
    if (!g || !bytes) return set_error(FSG_EINVAL, "NULL argument");
    GraphView G;
    int rc = view_of(graph, &G, "graph");
    if (rc) return rc;
    if (n_sets < 1) return set_error(FSG_EINVAL, "n_sets must be >= 1");
    if ((int64_t)n_sets * G.n > ((int64_t)1 << 31)) return set_error(FSG_EUNSUPPORTED, "n_sets * n above 2^31");
    *bytes = gnn_layout(G.n, n_sets).total;
    return FSG_OK;
}

}  // extern "C"

namespace fsg {
namespace gnn {
// Forward pass into dev_prob, enqueued on the stream without waiting.
int forward_enqueue(fsg_gnn *g, const fsg_graph *graph, int32_t n_sets, const uint8_t *dev_mask,
                    const float *beta, float *dev_prob, void *ws, size_t ws_bytes, void *stream)
{
    if (!g || !g->bound) return set_error(FSG_EINVAL, "gnn is NULL or not bound");
    GraphView G;
    int rc = view_of(graph, &G, "graph");
    if (rc) return rc;
    if (n_sets < 1 || !dev_mask || !beta || !dev_prob) return set_error(FSG_EINVAL, "bad arguments");
    const GnnWs w = gnn_layout(G.n, n_sets);
    rc = check_ws(ws, ws_bytes, w.total);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    rc = upload_betas(beta, n_sets, base, w, st);
    if (rc) return rc;
    rc = forward_all(g, G, n_sets, dev_mask, base, w, st);
    if (rc) return rc;
    const int64_t R = G.n * n_sets;
    // no gradient partials here, so one wave per row instead of the fixed
    // grid the training pass needs for its deterministic sums
    hipLaunchKernelGGL(k_head, dim3(grid_of(R * 64, 256)), dim3(256), 0, st,
                       (const uint16_t *)(base + w.H3),
                       (const float *)(g->p() + kWo), (const float *)(g->p() + kBo),
                       (const float *)nullptr, dev_prob, (float *)nullptr, (float *)nullptr,
                       (float *)nullptr, (float *)nullptr, R);
    GNN_TRY(hipGetLastError());
    return FSG_OK;
}
}  // namespace gnn
}  // namespace fsg

extern "C" {

int fsg_gnn_forward(fsg_gnn *g, const fsg_graph *graph, int32_t n_sets, const uint8_t *dev_mask,
                    const float *beta, float *dev_prob, void *ws, size_t ws_bytes, void *stream)
{
    const int rc = fsg::gnn::forward_enqueue(g, graph, n_sets, dev_mask, beta, dev_prob, ws,
                                             ws_bytes, stream);
    if (rc) return rc;
    GNN_TRY(hipStreamSynchronize((hipStream_t)stream));
    return FSG_OK;
}

int fsg_gnn_train_step(fsg_gnn *g, const fsg_graph *graph, const fsg_graph *reverse,
                       int32_t n_sets, const uint8_t *dev_mask, const float *beta,
                       const float *dev_target, float lr, int32_t apply_update, float *loss,
                       void *ws, size_t ws_bytes, void *stream)
{
    if (!g || !g->bound) return set_error(FSG_EINVAL, "gnn is NULL or not bound");
    GraphView G, Gr;
    int rc = view_of(graph, &G, "graph");
    if (rc) return rc;
    rc = view_of(reverse, &Gr, "reverse graph");
    if (rc) return rc;
    if (Gr.n != G.n || Gr.nnz != G.nnz) return set_error(FSG_EINVAL, "reverse graph does not match");
    if (n_sets < 1 || !dev_mask || !beta || !dev_target) return set_error(FSG_EINVAL, "bad arguments");
    if (!(lr >= 0.f)) return set_error(FSG_EINVAL, "lr must be >= 0");
    const GnnWs w = gnn_layout(G.n, n_sets);
    rc = check_ws(ws, ws_bytes, w.total);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    rc = upload_betas(beta, n_sets, base, w, st);
    if (rc) return rc;
    rc = forward_all(g, G, n_sets, dev_mask, base, w, st);
    if (rc) return rc;
    const int64_t R = G.n * n_sets;
    float *dH = (float *)(base + w.dH), *dH2 = (float *)(base + w.dH2);
    float *grads = g->g();
    hipLaunchKernelGGL(k_head, dim3(kPartBlocks), dim3(256), 0, st, (const uint16_t *)(base + w.H3),
                       (const float *)(g->p() + kWo), (const float *)(g->p() + kBo), dev_target,
                       (float *)(base + w.prob), dH, (float *)(base + w.pwo),
                       (float *)(base + w.pbo), (float *)(base + w.ploss), R);
    GNN_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(64), 0, st, (const float *)(base + w.pwo),
                       kPartBlocks, kHid, grads + kWo, 1.f);
    GNN_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(64), 0, st, (const float *)(base + w.pbo),
                       kPartBlocks, 1, grads + kBo, 1.f);
    GNN_TRY(hipGetLastError());
    float *dloss = (float *)(base + w.sums);
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(64), 0, st, (const float *)(base + w.ploss),
                       kPartBlocks, 1, dloss, 1.f / (float)R);
    GNN_TRY(hipGetLastError());
    const uint16_t *X1 = (const uint16_t *)(base + w.X1), *X2 = (const uint16_t *)(base + w.X2),
                   *X3 = (const uint16_t *)(base + w.X3), *H3 = (const uint16_t *)(base + w.H3);
    // layer 3: input X3 = [h2 | mean h2], output h3
    rc = backward_layer(g, G, Gr, n_sets, base, w, X3, kK2, H3, kHid, dH, kW3, kB3, kWb3, dH2, st);
    if (rc) return rc;
    // layer 2: output h2 = X3[:, 0:64]
    rc = backward_layer(g, G, Gr, n_sets, base, w, X2, kK2, X3, kK2, dH2, kW2, kB2, kWb2, dH, st);
    if (rc) return rc;
    // layer 1: output h1 = X2[:, 0:64]; no gradient to the inputs
    rc = backward_layer(g, G, Gr, n_sets, base, w, X1, kK1, X2, kK2, dH, kW1, kB1, kWb1, nullptr, st);
    if (rc) return rc;
    if (apply_update) {
        rc = adam_enqueue(g, grads, lr, st);
        if (rc) return rc;
    }
    float hl = 0.f;
    GNN_TRY(hipMemcpyAsync(&hl, dloss, 4, hipMemcpyDeviceToHost, st));
    GNN_TRY(hipStreamSynchronize(st));
    g->last_loss = hl;
    if (loss) *loss = hl;
    return FSG_OK;
}

int fsg_gnn_get_params(const fsg_gnn *g, float *out, int64_t n, void *stream)
{
    if (!g || !g->bound || !out || n != kP) return set_error(FSG_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    GNN_TRY(hipMemcpyAsync(out, g->p(), (size_t)kP * 4, hipMemcpyDeviceToHost, st));
    GNN_TRY(hipStreamSynchronize(st));
    return FSG_OK;
}

int fsg_gnn_set_params(fsg_gnn *g, const float *in, int64_t n, void *stream)
{
    if (!g || !g->bound || !in || n != kP) return set_error(FSG_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    GNN_TRY(hipMemcpyAsync(g->p(), in, (size_t)kP * 4, hipMemcpyHostToDevice, st));
    GNN_TRY(hipMemsetAsync(g->m(), 0, (size_t)2 * kP * 4, st));
    hipLaunchKernelGGL(k_params_to_bf16, dim3(grid_of(kWbN, 256)), dim3(256), 0, st,
                       (const float *)g->p(), g->wb());
    GNN_TRY(hipGetLastError());
    GNN_TRY(hipStreamSynchronize(st));
    g->step = 0;
    return FSG_OK;
}

int fsg_gnn_get_grads(const fsg_gnn *g, float *out, int64_t n, void *stream)
{
    if (!g || !g->bound || !out || n != kP) return set_error(FSG_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    GNN_TRY(hipMemcpyAsync(out, g->g(), (size_t)kP * 4, hipMemcpyDeviceToHost, st));
    GNN_TRY(hipStreamSynchronize(st));
    return FSG_OK;
}

int fsg_gnn_apply_update(fsg_gnn *g, const float *dev_grad, float lr, void *stream)
{
    if (!g || !g->bound) return set_error(FSG_EINVAL, "gnn is NULL or not bound");
    if (!(lr >= 0.f) || !(lr < INFINITY)) return set_error(FSG_EINVAL, "lr must be finite and >= 0");
    hipStream_t st = (hipStream_t)stream;
    const int rc = adam_enqueue(g, dev_grad ? dev_grad : (const float *)g->g(), lr, st);
    if (rc) return rc;
    GNN_TRY(hipStreamSynchronize(st));
    return FSG_OK;
}

int fsg_gnn_get_state(const fsg_gnn *g, float *m, float *v, uint16_t *wb, int64_t *step,
                      int64_t n, void *stream)
{
    if (!g || !g->bound || n != kP) return set_error(FSG_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    if (m) GNN_TRY(hipMemcpyAsync(m, g->m(), (size_t)kP * 4, hipMemcpyDeviceToHost, st));
    if (v) GNN_TRY(hipMemcpyAsync(v, g->v(), (size_t)kP * 4, hipMemcpyDeviceToHost, st));
    if (wb) GNN_TRY(hipMemcpyAsync(wb, g->wb(), (size_t)kWbN * 2, hipMemcpyDeviceToHost, st));
    GNN_TRY(hipStreamSynchronize(st));
    if (step) *step = g->step;
    return FSG_OK;
}

int fsg_estimate_spread(fsg_gnn *const *members, int32_t n_members, const fsg_graph *graph,
                        const int32_t *seeds, int64_t n_seeds, double beta, double gamma,
                        int64_t max_steps, const fsg_spread_gate *gate, int64_t B_fallback,
                        uint64_t rng_key, void *ws, size_t ws_bytes, void *sim_ws,
                        size_t sim_ws_bytes, uint32_t *dev_counts, double *spread,
                        double *uncertainty, int32_t *used_fallback, void *stream)
{
    if (!members || n_members < 1 || n_members > kMaxMembers || !gate || !spread ||
        !uncertainty || !used_fallback)
        return set_error(FSG_EINVAL, "bad arguments (1 <= n_members <= 64, gate not NULL)");
    GraphView G;
    int rc = view_of(graph, &G, "graph");
    if (rc) return rc;
    if (n_seeds < 0 || (n_seeds > 0 && !seeds)) return set_error(FSG_EINVAL, "bad seed array");
    for (int64_t i = 0; i < n_seeds; ++i)
        if (seeds[i] < 0 || seeds[i] >= G.n) return set_error(FSG_EINVAL, "seed out of range");
    std::vector<int32_t> distinct(seeds, seeds + n_seeds);
    std::sort(distinct.begin(), distinct.end());
    const int64_t k = std::unique(distinct.begin(), distinct.end()) - distinct.begin();
    *used_fallback = 0;
    *uncertainty = 0.0;
    if (k == 0) {  // nothing is ever infected
        *spread = 0.0;
        return FSG_OK;
    }
    const GnnWs w = gnn_layout(G.n, 1);
    rc = check_ws(ws, ws_bytes, w.total);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)ws;
    uint8_t *mask = (uint8_t *)(base + w.mask);
    int32_t *dseeds = (int32_t *)(base + w.seeds);
    hipLaunchKernelGGL(k_mask_clear, dim3(grid_of(G.n, 256)), dim3(256), 0, st, mask, (int32_t)G.n);
    GNN_TRY(hipGetLastError());
    if (n_seeds > 0) {
        GNN_TRY(hipMemcpyAsync(dseeds, seeds, (size_t)n_seeds * 4, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_mask_set, dim3(grid_of(n_seeds, 256)), dim3(256), 0, st, mask,
                           (const int32_t *)dseeds, n_seeds);
        GNN_TRY(hipGetLastError());
    }
    // every member's spread into the device sums, then one copy
    float *sums = (float *)(base + w.sums);
    const float fb = (float)beta;
    for (int32_t m = 0; m < n_members; ++m) {
        rc = forward_enqueue(members[m], graph, 1, mask, &fb, (float *)(base + w.prob), ws,
                             ws_bytes, stream);
        if (rc) return rc;
        float *part = (float *)(base + w.part);  // kSumParts floats (unused by the forward)
        hipLaunchKernelGGL(k_set_part, dim3(kSumParts), dim3(256), 0, st,
                           (const float *)(base + w.prob), (int32_t)G.n, part);
        GNN_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_set_final, dim3(1), dim3(kSumParts), 0, st, (const float *)part,
                           sums + m);
        GNN_TRY(hipGetLastError());
    }
    float hs[kMaxMembers];
    GNN_TRY(hipMemcpyAsync(hs, sums, (size_t)n_members * 4, hipMemcpyDeviceToHost, st));
    GNN_TRY(hipStreamSynchronize(st));
    std::vector<double> sp(hs, hs + n_members);
    double mean = 0, var = 0;
    for (double x : sp) mean += x;
    mean /= n_members;
    for (double x : sp) var += (x - mean) * (x - mean);
    var = n_members > 1 ? var / (n_members - 1) : 0.0;
    const double unc = mean > 0 ? sqrt(var) / mean : 1e30;
    *uncertainty = unc;
    *spread = mean;
    if (gate->calibrated) {
        const double x = 20.0 * beta, kd = (double)k, lk = log(kd);
        const double f[FSG_CALIB_TERMS] = {1.0, x, x * x, x * x * x, 1.0 / kd, x / kd,
                                           1.0 / (kd * kd), lk, x * lk};
        double z = 0.0;
        for (int i = 0; i < FSG_CALIB_TERMS; ++i) z += gate->calib[i] * f[i];
        *spread = mean * exp(z);
    }
    if (unc > gate->tau || k < gate->min_seeds) {
        if (B_fallback < 1 || !dev_counts) return set_error(FSG_EINVAL, "fallback needs B_fallback and counts");
        fsg_params prm;
        memset(&prm, 0, sizeof(prm));
        prm.model = FSG_SIR;
        prm.beta = beta;
        prm.gamma = gamma;
        prm.max_steps = max_steps;
        fsg_run_info info;
        rc = fsg_simulate(graph, &prm, seeds, n_seeds, B_fallback, 0, rng_key, nullptr, sim_ws,
                          sim_ws_bytes, nullptr, dev_counts, &info, stream);
        if (rc) return rc;
        std::vector<uint32_t> cnt((size_t)G.n);
        GNN_TRY(hipMemcpyAsync(cnt.data(), dev_counts, (size_t)G.n * 4, hipMemcpyDeviceToHost, st));
        GNN_TRY(hipStreamSynchronize(st));
        double tot = 0;
        for (uint32_t c : cnt) tot += c;
        *spread = tot / (double)B_fallback;
        *used_fallback = 1;
    }
    return FSG_OK;
}

}  // extern "C"
