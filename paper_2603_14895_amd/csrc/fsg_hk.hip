// fsg_hk.hip -- batched Hegselmann-Krause opinion dynamics as synchronous
// pull message passing (Appendix A.2, "Micro-accelerated implementation of
// HK model"): every arc j -> i carries the pair (h_j, 1) when
// |h_i - h_j| < eps and (0, 0) otherwise; node i sums the pairs and takes
// the quotient, keeping h_i when no pair is non-zero.  B independent
// replicates (initial opinion vectors) run side by side.
//
// State: FP32 opinions [n][B] (replicate fastest), double-buffered between
// the caller's array and the workspace.  No randomness.
//
// Arithmetic contract: per (node, replicate) the filtered opinions are
// summed in IEEE single precision in CSR order of the in-arcs, one rounding
// per addition, then divided once (round to nearest even) by the count.
// The kernels keep that order exactly, so the result is the same bits as a
// plain sequential loop, and so are all later eps decisions.
//
// Kernel (one launch per step):
//   * rows with more than kWideRow in-arcs ("hubs", largest first) get
//     the first blocks of the grid: one block per (hub, 64 replicates);
//     its four waves gather tiles of 64 arcs x 64 replicates into LDS two
//     tiles ahead (source indices one tile further), and wave 0 adds each
//     replicate's column in arc order;
//   * every other row: one lane per (row, 4 replicates) when B % 4 == 0
//     (16-byte gathers of the source rows), else per (row, replicate),
//     looping over the row's in-arcs with the next source indices in
//     flight.
// A step that changes no opinion leaves its ring flag clear; the next step's
// kernel then returns at once, so several steps can be queued between host
// polls.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/fsg.h"
#include "fsg_internal.hpp"

namespace fsg {
namespace hk {

constexpr int kBlock = 256;
constexpr int kCols = 64;          // replicates per hub block (one per lane)
constexpr int kTile = 64;          // arcs per LDS tile
constexpr int kPerWave = kTile / 4;  // arcs of a tile each wave gathers
constexpr int kRowUnroll = 4;      // arcs per light-row batch

struct Args {
    const int32_t *ptr;   // [n+1]
    const int32_t *src;   // [nnz]
    const int32_t *wide;  // [n_wide] hub rows, largest first
    int32_t n;
    int32_t n_wide;
    int32_t chunks;       // ceil(B / kCols)
    int32_t hub_blocks;   // n_wide * chunks
    int64_t B;
    int64_t lanes;        // n * B / vec
    float eps;
    float mu, omm;        // weighted HK: fraction moved towards the mean, and 1 - mu
    const float *x;       // opinions after the previous step
    float *y;             // opinions after this step
    uint32_t *flags;      // ring: 1 iff the step changed an opinion
    int32_t slot;         // this step's ring index
    int32_t prev;         // previous step's ring index, -1: none
};

__device__ __forceinline__ void mark_changed(const Args &a, bool ch)
{
    if (__ballot(ch) != 0ull && (threadIdx.x & 63) == 0) a.flags[a.slot] = 1u;
}

// One eps-filtered message: adds h_j to the sum and 1 to the count when the
// two opinions differ by less than eps.  Adding +0.0 instead of skipping is
// the same bits: the sum starts at +0.0 and round-to-nearest never yields
// -0.0 from it.
__device__ __forceinline__ void take(float hv, float hj, float eps, float &mc, int &mv)
{
    const bool in = fabsf(hv - hj) < eps;
    mc += in ? hj : 0.0f;
    mv += in ? 1 : 0;
}

__device__ __forceinline__ float settle(const Args &a, float hv, float mc, int mv)
{
    if (mv == 0) return hv;
    const float m = __fdiv_rn(mc, (float)mv);
    // weighted HK: (1 - mu) h + mu m, two rounded products and a rounded sum
    // (no contraction); mu = 1 is plain HK
    return a.mu == 1.0f ? m : __fadd_rn(__fmul_rn(a.omm, hv), __fmul_rn(a.mu, m));
}

// ---- hub rows ---------------------------------------------------------------

// Read-only view of the source indices in the constant address space: the
// hub path reads them with wave-uniform addresses, so they come in through
// scalar loads and the gathers that use them wait on the scalar counter
// only, never on older gathers still in flight.
typedef const __attribute__((address_space(4))) int32_t csrc_t;

struct HubTile {
    int32_t s[kPerWave];
    float g[kPerWave];
};

// Sources of tile t (clamped to the last tile; arcs past the row end repeat
// its last arc), this wave's quarter.
__device__ __forceinline__ void hub_src(csrc_t *src, int64_t e0, int64_t e1, int nt, int w, int t,
                                        int32_t (&s)[kPerWave])
{
    const int64_t base = e0 + (int64_t)min(t, nt - 1) * kTile + w * kPerWave;
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) s[i] = src[min(base + i, e1 - 1)];
}

// One buffer resource per source row (its B opinions; base and range in
// scalar registers) and one fixed 32-bit lane offset: the gathers need no
// per-load address registers, and lanes past column B read 0 through the
// range check instead of touching memory.
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit buffer access (gfx9 family)

__device__ __forceinline__ void hub_gather(const Args &a, uint32_t voff, const int32_t (&s)[kPerWave],
                                           float (&g)[kPerWave])
{
    const uint32_t row_bytes = (uint32_t)a.B * 4u;
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) {
        __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(a.x + (int64_t)s[i] * a.B), (short)0, (int)row_bytes, kRsrcWord3);
        g[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, 0));
    }
}

__device__ __forceinline__ void hub_store(float (*buf)[kCols], int w, int lane,
                                          const float (&g)[kPerWave])
{
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) buf[w * kPerWave + i][lane] = g[i];
}

__device__ __forceinline__ void hub_sum(float (*buf)[kCols], int lane, int count, float hv, float eps,
                                        float &mc, int &mv)
{
    for (int i = 0; i < count; ++i) take(hv, buf[i][lane], eps, mc, mv);
}

// Tiles t = 0 .. nt-1 (nt >= 5: a hub has more than kWideRow arcs).  Per
// half-iteration k: sources of tile k+3 (scalar loads), gathers of tile k+2,
// the sum of tile k from LDS by wave 0, then the gathers of tile k+1, issued
// one half earlier, go to the other LDS buffer.  Loads past the last tile
// re-read it, so the loop body has no conditional loads.
__device__ void hub_row(const Args &a, float (*lds)[kTile][kCols])
{
    const int hb = blockIdx.x;
    const int32_t v = a.wide[hb / a.chunks];
    const int64_t c0 = (int64_t)(hb % a.chunks) * kCols;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool live = c0 + lane < a.B;
    const int64_t col = live ? c0 + lane : a.B - 1;
    const uint32_t voff = (uint32_t)(c0 + lane) * 4u;  // past the row for idle lanes: reads 0
    csrc_t *src = (csrc_t *)a.src;
    const int64_t e0 = a.ptr[v], e1 = a.ptr[v + 1];
    const int nt = (int)((e1 - e0 + kTile - 1) / kTile);
    const float hv = a.x[(int64_t)v * a.B + col];
    float mc = 0.0f;
    int mv = 0;
    HubTile A, Bt;  // tiles with even / odd index
    hub_src(src, e0, e1, nt, w, 0, A.s);
    hub_src(src, e0, e1, nt, w, 1, Bt.s);
    hub_gather(a, voff, A.s, A.g);
    hub_src(src, e0, e1, nt, w, 2, A.s);
    hub_gather(a, voff, Bt.s, Bt.g);
    hub_store(lds[0], w, lane, A.g);
    __syncthreads();
    // at even k: lds[0] = tile k, Bt.g = tile k+1 in flight, A.s = sources
    // of tile k+2
    for (int k = 0; k < nt; k += 2) {
        hub_src(src, e0, e1, nt, w, k + 3, Bt.s);
        hub_gather(a, voff, A.s, A.g);
        if (w == 0)
            hub_sum(lds[0], lane, (int)min<int64_t>(kTile, e1 - e0 - (int64_t)k * kTile), hv, a.eps, mc, mv);
        hub_store(lds[1], w, lane, Bt.g);
        __syncthreads();
        if (k + 1 >= nt) break;
        hub_src(src, e0, e1, nt, w, k + 4, A.s);
        hub_gather(a, voff, Bt.s, Bt.g);
        if (w == 0)
            hub_sum(lds[1], lane, (int)min<int64_t>(kTile, e1 - e0 - (int64_t)(k + 1) * kTile), hv, a.eps,
                    mc, mv);
        hub_store(lds[0], w, lane, A.g);
        __syncthreads();
    }
    if (w == 0) {
        const float nv = settle(a, hv, mc, mv);
        if (live) a.y[(int64_t)v * a.B + col] = nv;
        mark_changed(a, live && nv != hv);
    }
}

// ---- light rows -------------------------------------------------------------

template <int VEC>
struct Vec;
template <>
struct Vec<1> {
    typedef float T;
    static __device__ __forceinline__ float get(const T &x, int) { return x; }
    static __device__ __forceinline__ void set(T &x, int, float f) { x = f; }
};
template <>
struct Vec<4> {
    typedef float4 T;
    static __device__ __forceinline__ float get(const T &x, int i)
    {
        return i == 0 ? x.x : i == 1 ? x.y : i == 2 ? x.z : x.w;
    }
    static __device__ __forceinline__ void set(T &x, int i, float f)
    {
        if (i == 0) x.x = f;
        else if (i == 1) x.y = f;
        else if (i == 2) x.z = f;
        else x.w = f;
    }
};

template <int VEC>
__device__ void light_row(const Args &a, int64_t idx)
{
    typedef typename Vec<VEC>::T T;
    const int64_t V = a.B / VEC;
    bool ch = false;
    if (idx < a.lanes) {
        const int64_t v = idx / V;
        const int64_t q = idx - v * V;
        const int64_t e0 = a.ptr[v], e1 = a.ptr[v + 1];
        if (e1 - e0 <= kWideRow) {
            const T *X = reinterpret_cast<const T *>(a.x);
            const T hv = X[v * V + q];
            float mc[VEC];
            int mv[VEC];
#pragma unroll
            for (int c = 0; c < VEC; ++c) {
                mc[c] = 0.0f;
                mv[c] = 0;
            }
            if (e0 < e1) {
                // indices past the row end repeat its last arc (loaded, never taken)
                const int64_t last = e1 - 1;
                int32_t s[kRowUnroll];
#pragma unroll
                for (int i = 0; i < kRowUnroll; ++i) s[i] = a.src[min(e0 + i, last)];
                for (int64_t e = e0; e < e1; e += kRowUnroll) {
                    T g[kRowUnroll];
#pragma unroll
                    for (int i = 0; i < kRowUnroll; ++i) g[i] = X[(int64_t)s[i] * V + q];
                    // the next batch's sources go out while the gathers are in flight
#pragma unroll
                    for (int i = 0; i < kRowUnroll; ++i) s[i] = a.src[min(e + kRowUnroll + i, last)];
#pragma unroll
                    for (int i = 0; i < kRowUnroll; ++i) {
                        if (e + i < e1) {
#pragma unroll
                            for (int c = 0; c < VEC; ++c)
                                take(Vec<VEC>::get(hv, c), Vec<VEC>::get(g[i], c), a.eps, mc[c], mv[c]);
                        }
                    }
                }
            }
            T out;
#pragma unroll
            for (int c = 0; c < VEC; ++c) {
                const float h = Vec<VEC>::get(hv, c);
                const float nv = settle(a, h, mc[c], mv[c]);
                Vec<VEC>::set(out, c, nv);
                ch |= nv != h;
            }
            reinterpret_cast<T *>(a.y)[v * V + q] = out;
        }
    }
    mark_changed(a, ch);
}

template <int VEC>
__global__ __launch_bounds__(kBlock) void k_hk_step(Args a)
{
    __shared__ float lds[2][kTile][kCols];
    if (a.prev >= 0 && a.flags[a.prev] == 0u) return;  // converged: nothing moves
    if ((int)blockIdx.x < a.hub_blocks) {
        hub_row(a, lds);
        return;
    }
    light_row<VEC>(a, (int64_t)(blockIdx.x - a.hub_blocks) * kBlock + threadIdx.x);
}

// Per replicate: nodes with opinion above `act`.
__global__ void k_hk_count(const float *h, int64_t n, int64_t B, int64_t slabs, float act,
                           uint32_t *counts)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= B * slabs) return;
    const int64_t r = t % B, s = t / B;
    uint32_t c = 0;
    for (int64_t v = s; v < n; v += slabs) c += h[v * B + r] > act ? 1u : 0u;
    if (c) atomicAdd(&counts[r], c);
}

__global__ void k_fill_u32(uint32_t *p, int64_t count)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct View {
    int64_t n = 0, nnz = 0, dmax = 0, n_wide = 0;
    const int32_t *ptr = nullptr, *src = nullptr, *wide = nullptr;
};

int view_of(const fsg_graph *g, View *v)
{
    if (!graph_view(g, &v->n, &v->nnz, &v->dmax, &v->ptr, &v->src, &v->wide, &v->n_wide))
        return set_error(FSG_EINVAL, "graph is NULL or not bound");
    return FSG_OK;
}

#define HK_TRY(expr)                                                                          \
    do {                                                                                      \
        if (fsg::inject_device_fault())                                                        \
            return set_error(FSG_EDEVICE, (std::string(#expr) + ": injected fault").c_str());  \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return set_error(FSG_EDEVICE, (std::string(#expr) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

constexpr int kMaxSync = 256;

int sync_of(const fsg_schedule *s)
{
    int v = s && s->steps_per_sync > 0 ? s->steps_per_sync : 16;
    return std::min(v, kMaxSync);
}

size_t ws_bytes_for(int64_t n, int64_t B, int sync)
{
    return al256((size_t)n * (size_t)B * 4) + al256((size_t)(sync + 1) * 4);
}

}  // namespace hk
}  // namespace fsg

using namespace fsg;
using namespace fsg::hk;

extern "C" {

int fsg_hk_workspace_size(const fsg_graph *g, int64_t B, const fsg_schedule *sched, size_t *bytes)
{
    View G;
    int rc = view_of(g, &G);
    if (rc) return rc;
    if (!bytes) return set_error(FSG_EINVAL, "bytes is NULL");
    if (B < 1) return set_error(FSG_EINVAL, "B must be >= 1");
    *bytes = ws_bytes_for(G.n, B, sync_of(sched));
    return FSG_OK;
}

int fsg_hk(const fsg_graph *g, float eps, int64_t max_steps, int64_t B, float *dev_h,
           const fsg_schedule *sched, void *dev_ws, size_t ws_bytes, float act,
           uint32_t *dev_counts, fsg_run_info *info, void *stream)
{
    return fsg_whk(g, eps, 1.0f, max_steps, B, dev_h, sched, dev_ws, ws_bytes, act, dev_counts,
                   info, stream);
}

int fsg_whk(const fsg_graph *g, float eps, float mu, int64_t max_steps, int64_t B, float *dev_h,
            const fsg_schedule *sched, void *dev_ws, size_t ws_bytes, float act,
            uint32_t *dev_counts, fsg_run_info *info, void *stream)
{
    View G;
    int rc = view_of(g, &G);
    if (rc) return rc;
    if (!dev_h) return set_error(FSG_EINVAL, "dev_h is NULL");
    if (B < 1) return set_error(FSG_EINVAL, "B must be >= 1");
    if (max_steps < 0) return set_error(FSG_EINVAL, "max_steps must be >= 0");
    if (!(eps >= 0.0f) || isinf(eps)) return set_error(FSG_EINVAL, "eps must be finite and >= 0");
    if (!(mu >= 0.0f && mu <= 1.0f)) return set_error(FSG_EINVAL, "mu must be in [0, 1]");
    if (isnan(act)) return set_error(FSG_EINVAL, "act is NaN");
    const int vec = (B % 4 == 0) ? 4 : 1;
    const int64_t lanes = G.n * (B / vec);
    if (lanes >= ((int64_t)1 << 31) - kBlock || B >= ((int64_t)1 << 28))
        return set_error(FSG_EUNSUPPORTED, "n * B too large");
    const int chunks = (int)((B + kCols - 1) / kCols);
    if (G.n_wide * (int64_t)chunks >= ((int64_t)1 << 30))
        return set_error(FSG_EUNSUPPORTED, "too many hub blocks");
    const int sync = sync_of(sched);
    const size_t need = ws_bytes_for(G.n, B, sync);
    if (!dev_ws || ws_bytes < need) return set_error(FSG_EWORKSPACE, "HK workspace too small");
    if (((uintptr_t)dev_ws & 255) != 0 || ((uintptr_t)dev_h & 15) != 0)
        return set_error(FSG_EWORKSPACE, "workspace not 256-byte aligned or dev_h not 16-byte aligned");
    const bool timed = sched && sched->time_kernels;
    hipStream_t st = (hipStream_t)stream;

    float *buf[2] = {dev_h, (float *)dev_ws};
    uint32_t *flags = (uint32_t *)((char *)dev_ws + al256((size_t)G.n * (size_t)B * 4));
    const int ring = sync + 1;
    Args a;
    memset(&a, 0, sizeof(a));
    a.ptr = G.ptr;
    a.src = G.src;
    a.wide = G.wide;
    a.n = (int32_t)G.n;
    a.n_wide = (int32_t)G.n_wide;
    a.chunks = chunks;
    a.hub_blocks = (int32_t)(G.n_wide * chunks);
    a.B = B;
    a.lanes = lanes;
    a.eps = eps;
    a.mu = mu;
    a.omm = 1.0f - mu;
    a.flags = flags;
    const int64_t grid = a.hub_blocks + (lanes + kBlock - 1) / kBlock;

    std::vector<hipEvent_t> ev;
    struct Ev {
        std::vector<hipEvent_t> &e;
        ~Ev()
        {
            for (auto x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev_guard{ev};
    if (timed) {
        ev.assign(2 * (size_t)sync, nullptr);
        for (auto &x : ev) HK_TRY(hipEventCreate(&x));
    }
    std::vector<uint32_t> hflags((size_t)ring);
    double kernel_ms = 0.0;
    int64_t launches = 0, t = 0;
    bool converged = false;
    while (!converged && t < max_steps) {
        const int64_t c = std::min<int64_t>(sync, max_steps - t);
        HK_TRY(launch_ring_clear(flags, ring, (int32_t)(t % ring), st));
        for (int64_t i = 1; i <= c; ++i) {
            const int64_t step = t + i;
            a.x = buf[(step - 1) & 1];
            a.y = buf[step & 1];
            a.slot = (int32_t)(step % ring);
            a.prev = step > 1 ? (int32_t)((step - 1) % ring) : -1;
            if (timed) HK_TRY(hipEventRecord(ev[2 * (i - 1)], st));
            if (vec == 4)
                hipLaunchKernelGGL(k_hk_step<4>, dim3((unsigned)grid), dim3(kBlock), 0, st, a);
            else
                hipLaunchKernelGGL(k_hk_step<1>, dim3((unsigned)grid), dim3(kBlock), 0, st, a);
            HK_TRY(hipGetLastError());
            if (timed) HK_TRY(hipEventRecord(ev[2 * (i - 1) + 1], st));
        }
        HK_TRY(hipMemcpyAsync(hflags.data(), flags, (size_t)ring * 4, hipMemcpyDeviceToHost, st));
        HK_TRY(hipStreamSynchronize(st));
        int64_t done = t + c;
        for (int64_t i = 1; i <= c; ++i)
            if (hflags[(size_t)((t + i) % ring)] == 0u) {
                done = t + i;
                converged = true;
                break;
            }
        if (timed)
            for (int64_t i = 1; i <= done - t; ++i) {
                float ms = 0.f;
                HK_TRY(hipEventElapsedTime(&ms, ev[2 * (i - 1)], ev[2 * (i - 1) + 1]));
                kernel_ms += ms;
                ++launches;
            }
        t = done;
    }
    if (t & 1)
        HK_TRY(hipMemcpyAsync(dev_h, buf[1], (size_t)G.n * (size_t)B * 4, hipMemcpyDeviceToDevice, st));
    if (dev_counts) {
        const int64_t slabs = std::max<int64_t>(1, std::min<int64_t>(G.n, (1 << 18) / B));
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, dev_counts, B);
        HK_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_hk_count, dim3((unsigned)((B * slabs + 255) / 256)), dim3(256), 0, st,
                           (const float *)dev_h, G.n, B, slabs, act, dev_counts);
        HK_TRY(hipGetLastError());
    }
    HK_TRY(hipStreamSynchronize(st));
    if (info) {
        info->steps_run = t;
        info->absorbed = converged ? 1 : 0;
        info->tail_steps = 0;
        info->step_kernel_ms = kernel_ms;
        info->step_launches = launches;
        info->setup_ms = 0.0;
        info->finalize_ms = 0.0;
        info->philox_calls = 0;
    }
    return FSG_OK;
}

}  // extern "C"
