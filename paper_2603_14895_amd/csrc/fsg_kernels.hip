// fsg_kernels.hip -- the synchronous pull step of batched Monte Carlo
// propagation for gfx950 (FS_GPlib, arxiv 2603.14895, Sec. 3.1: message
// Eq. ms, aggregation Eq. agg, update Eq. updata; batched over replicates as
// Eq. batch).
//
// Work decomposition.  A row v of the pull CSR lists the sources of the arcs
// into v.  Rows are grouped into contiguous tiles of roughly equal in-edge
// load (the target-node partition of Sec. 3.2 applied per workgroup).  Inside
// a wave, G * S lanes own one row: G lanes over the row's replicate words
// (64 replicates per uint64 word, so the G lanes of a neighbour gather read
// 8*G contiguous bytes) and S lanes over its in-edge list.  Per-lane partial
// results are merged with order-free operations (OR for cascades, integer
// addition of bit-sliced counters for counts), so every schedule gives the
// same bits.  Rows with more than `heavy` in-edges are cut into segments whose
// partial results go to a workspace and are merged by k_combine.
//
// No MFMA here: the step is a sparse gather plus integer/ALU work.
#include "fsg_device.hpp"
#include "fsg_internal.hpp"

#include <algorithm>

namespace fsg {

// Infection thresholds staged in LDS by the step kernel (k = 0 .. kTinfLds-1).
constexpr int kTinfLds = 2048;

// Threshold of k infected neighbours: LDS copy when staged, global otherwise.
__device__ __forceinline__ uint32_t tinf_at(const StepArgs &a, const uint32_t *tl, int tl_n,
                                            uint32_t k)
{
    if (k > (uint32_t)a.khat) k = (uint32_t)a.khat;
    return (int)k < tl_n ? tl[k] : a.tinf[k];
}

// ---------------------------------------------------------------- IC ----
// Message of arc e = (u -> v) in replicate r: u newly active at t-1 and the
// arc's one trial fires (the trial does not depend on t, and an arc is
// consulted only once per replicate since u is newly active only once).
// Aggregation: OR over arcs.  Update: 0 -> 1 on any message, 1 -> 2.
__device__ __forceinline__ void ic_edge(const StepArgs &a, int e, uint64_t f, uint64_t gbase,
                                        uint32_t tv, uint64_t &acc)
{
    if (!f) return;
    const uint32_t te = a.edge_t ? a.edge_t[e] : tv;
    if (te == 0u) return;
    if (te == kAlways) {
        acc |= f;
        return;
    }
    while (f) {
        const int b = __builtin_ctzll(f);
        const int gs = b - (int)((gbase + (uint64_t)b) & 3u);  // block's first bit
        const uint64_t gm = block_bits(gbase, b);
        const uint64_t bits = f & gm;
        f &= ~gm;
        const uint32_t blk = (uint32_t)((gbase + (uint64_t)b) >> 2);
        const U4 o = philox10((uint32_t)e, blk, 0u, kDomIcEdge << 24, a.key0, a.key1);
        const uint32_t ou[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int bb = gs + j;
            if (bb < 0 || bb > 63) continue;
            if (((bits >> bb) & 1ull) && ou[j] < te) acc |= 1ull << bb;
        }
    }
}

__device__ __forceinline__ void ic_row_word(const StepArgs &a, int G, int S, bool valid, int v,
                                            int w, int e0, int e1, uint32_t tv, int s, int seg,
                                            uint64_t lm, bool &any)
{
    const int64_t idx = (int64_t)v * a.W + w;
    const int64_t W = a.W;
    const uint64_t gbase = a.goff + 64ull * (uint64_t)w;
    const uint64_t A = valid ? a.aux[idx] : ~0ull;
    const uint64_t cand = valid ? (~A & tail_mask(w, a.B) & lm) : 0ull;
    uint64_t acc = 0;
    if (S == 1 && G >= 16 && a.fast32 && seg < 0) {
        // 16 arcs of the row per pass: lane lr of each 16-lane DPP row loads
        // source e0 + base + lr, the row's lanes receive them by row
        // broadcast and gather their word of each; arcs past the row's end
        // read the all-zero row n, so they never reach a trial
        const int lr = (int)(threadIdx.x & 15u);
        int dmax = 0;
        const int d = valid ? e1 - e0 : 0;
        for (int l = 0; l < 64; l += G) dmax = max(dmax, __builtin_amdgcn_readlane(d, l));
        if (dmax > 0 && __ballot(cand != 0ull) != 0ull) {
            const uint32_t W8 = (uint32_t)a.W * 8u, w8 = (uint32_t)w * 8u, zero = (uint32_t)a.n;
            const char *prev = reinterpret_cast<const char *>(a.prev);
            auto src_at = [&](int base) -> uint32_t {
                const int e = e0 + base + lr;
                return e < e1 ? (uint32_t)ld32_off32(a.src, (uint32_t)e) : zero;
            };
            auto word = [&](uint32_t u) -> uint64_t {
                return *reinterpret_cast<const uint64_t *>(prev + __umul24(cand ? u : zero, W8) + w8);
            };
            uint32_t cur = src_at(0);
            for (int base = 0; base < dmax; base += 16) {
                const uint32_t nxt = base + 16 < dmax ? src_at(base + 16) : zero;
                {
                    const uint64_t x0 = word(row_bcast<0>(cur)), x1 = word(row_bcast<1>(cur)),
                                   x2 = word(row_bcast<2>(cur)), x3 = word(row_bcast<3>(cur)),
                                   x4 = word(row_bcast<4>(cur)), x5 = word(row_bcast<5>(cur)),
                                   x6 = word(row_bcast<6>(cur)), x7 = word(row_bcast<7>(cur));
                    const int eb = e0 + base;
                    ic_edge(a, eb, x0 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 1, x1 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 2, x2 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 3, x3 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 4, x4 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 5, x5 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 6, x6 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 7, x7 & cand & ~acc, gbase, tv, acc);
                }
                if (dmax - base > 8) {
                    const uint64_t x0 = word(row_bcast<8>(cur)), x1 = word(row_bcast<9>(cur)),
                                   x2 = word(row_bcast<10>(cur)), x3 = word(row_bcast<11>(cur)),
                                   x4 = word(row_bcast<12>(cur)), x5 = word(row_bcast<13>(cur)),
                                   x6 = word(row_bcast<14>(cur)), x7 = word(row_bcast<15>(cur));
                    const int eb = e0 + base + 8;
                    ic_edge(a, eb, x0 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 1, x1 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 2, x2 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 3, x3 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 4, x4 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 5, x5 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 6, x6 & cand & ~acc, gbase, tv, acc);
                    ic_edge(a, eb + 7, x7 & cand & ~acc, gbase, tv, acc);
                }
                cur = nxt;
            }
        }
    } else if (cand && a.fast32) {
        const uint32_t Wu = (uint32_t)a.W, ww = (uint32_t)w;
        int e = e0 + s;
        for (; e + 3 * S < e1; e += 4 * S) {
            const uint32_t u0 = (uint32_t)ld32_off32(a.src, (uint32_t)e);
            const uint32_t u1 = (uint32_t)ld32_off32(a.src, (uint32_t)(e + S));
            const uint32_t u2 = (uint32_t)ld32_off32(a.src, (uint32_t)(e + 2 * S));
            const uint32_t u3 = (uint32_t)ld32_off32(a.src, (uint32_t)(e + 3 * S));
            const uint64_t f0 = ld64_off32(a.prev, __umul24(u0, Wu) + ww);
            const uint64_t f1 = ld64_off32(a.prev, __umul24(u1, Wu) + ww);
            const uint64_t f2 = ld64_off32(a.prev, __umul24(u2, Wu) + ww);
            const uint64_t f3 = ld64_off32(a.prev, __umul24(u3, Wu) + ww);
            ic_edge(a, e, f0 & cand & ~acc, gbase, tv, acc);
            ic_edge(a, e + S, f1 & cand & ~acc, gbase, tv, acc);
            ic_edge(a, e + 2 * S, f2 & cand & ~acc, gbase, tv, acc);
            ic_edge(a, e + 3 * S, f3 & cand & ~acc, gbase, tv, acc);
        }
        for (; e < e1; e += S) {
            const uint32_t u = (uint32_t)ld32_off32(a.src, (uint32_t)e);
            ic_edge(a, e, ld64_off32(a.prev, __umul24(u, Wu) + ww) & cand & ~acc, gbase, tv, acc);
        }
    } else if (cand) {
        int e = e0 + s;
        // four independent gathers in flight per lane
        for (; e + 3 * S < e1; e += 4 * S) {
            const int u0 = a.src[e], u1 = a.src[e + S], u2 = a.src[e + 2 * S],
                      u3 = a.src[e + 3 * S];
            const uint64_t f0 = a.prev[(int64_t)u0 * W + w], f1 = a.prev[(int64_t)u1 * W + w],
                           f2 = a.prev[(int64_t)u2 * W + w], f3 = a.prev[(int64_t)u3 * W + w];
            ic_edge(a, e, f0 & cand & ~acc, gbase, tv, acc);
            ic_edge(a, e + S, f1 & cand & ~acc, gbase, tv, acc);
            ic_edge(a, e + 2 * S, f2 & cand & ~acc, gbase, tv, acc);
            ic_edge(a, e + 3 * S, f3 & cand & ~acc, gbase, tv, acc);
        }
        for (; e < e1; e += S)
            ic_edge(a, e, a.prev[(int64_t)a.src[e] * W + w] & cand & ~acc, gbase, tv, acc);
    }
    acc = or_reduce_lanes(acc, G, S);
    if (!valid || s != 0) return;
    if (seg >= 0) {
        a.partial[(int64_t)seg * a.W + w] = acc;
    } else {
        a.next[idx] = acc;
        a.aux[idx] = A | acc;
        any |= acc != 0;
    }
}

// Bit-sliced count of the in-neighbours whose word has the replicate's bit
// set: four independent gathers in flight per lane, folded in with carry-save
// adders.  Counts are kept for every replicate of the word; callers use them
// only under their own state mask.  The fast path addresses sources and
// planes with 32-bit offsets from uniform bases and 24-bit index products.
template <int L>
__device__ __forceinline__ void count_edges(const StepArgs &a, int e, int e1, int S, int w,
                                            uint64_t (&c)[L])
{
    if (a.fast32) {
        const uint32_t W = (uint32_t)a.W, ww = (uint32_t)w;
        for (; e + 3 * S < e1; e += 4 * S) {
            const uint32_t u0 = (uint32_t)ld32_off32(a.src, (uint32_t)e);
            const uint32_t u1 = (uint32_t)ld32_off32(a.src, (uint32_t)(e + S));
            const uint32_t u2 = (uint32_t)ld32_off32(a.src, (uint32_t)(e + 2 * S));
            const uint32_t u3 = (uint32_t)ld32_off32(a.src, (uint32_t)(e + 3 * S));
            const uint64_t x0 = ld64_off32(a.prev, __umul24(u0, W) + ww);
            const uint64_t x1 = ld64_off32(a.prev, __umul24(u1, W) + ww);
            const uint64_t x2 = ld64_off32(a.prev, __umul24(u2, W) + ww);
            const uint64_t x3 = ld64_off32(a.prev, __umul24(u3, W) + ww);
            bs_add4<L>(c, x0, x1, x2, x3);
        }
        for (; e < e1; e += S) {
            const uint32_t u = (uint32_t)ld32_off32(a.src, (uint32_t)e);
            bs_add1<L>(c, ld64_off32(a.prev, __umul24(u, W) + ww));
        }
        return;
    }
    const int64_t W = a.W;
    for (; e + 3 * S < e1; e += 4 * S) {
        const int u0 = a.src[e], u1 = a.src[e + S], u2 = a.src[e + 2 * S], u3 = a.src[e + 3 * S];
        bs_add4<L>(c, a.prev[(int64_t)u0 * W + w], a.prev[(int64_t)u1 * W + w],
                   a.prev[(int64_t)u2 * W + w], a.prev[(int64_t)u3 * W + w]);
    }
    for (; e < e1; e += S) bs_add1<L>(c, a.prev[(int64_t)a.src[e] * W + w]);
}

// The same count when a row owns whole 16-lane rows of the wave (G >= 16,
// S = 1) and 32-bit offsets apply: the 16 lanes load 16 consecutive sources
// of their row with one vector load (the next chunk's load issued before the
// current chunk's gathers), and each source reaches every lane of the row by a
// DPP row broadcast; the gathers then go out eight at a time without waiting
// on index loads.  Positions past the row's end carry source n, whose plane
// row is all zero, as does every position of a lane whose word needs no
// count.  All 64 lanes of the wave must call this together.
template <int L>
__device__ __forceinline__ void count_edges_bcast(const StepArgs &a, int G, bool valid, int e0,
                                                  int e1, int w, bool need, uint64_t (&c)[L])
{
    const int lr = (int)(threadIdx.x & 15u);
    int dmax = 0;  // longest valid row of the wave (word 0 of a row is valid iff the row is)
    const int d = valid ? e1 - e0 : 0;
    for (int l = 0; l < 64; l += G) dmax = max(dmax, __builtin_amdgcn_readlane(d, l));
    if (dmax == 0 || __ballot(need) == 0ull) return;
    const uint32_t W8 = (uint32_t)a.W * 8u, w8 = (uint32_t)w * 8u, zero = (uint32_t)a.n;
    const char *prev = reinterpret_cast<const char *>(a.prev);
    auto src_at = [&](int base) -> uint32_t {
        const int e = e0 + base + lr;
        return e < e1 ? (uint32_t)ld32_off32(a.src, (uint32_t)e) : zero;
    };
    auto word = [&](uint32_t u) -> uint64_t {
        return *reinterpret_cast<const uint64_t *>(prev + __umul24(need ? u : zero, W8) + w8);
    };
    uint32_t cur = src_at(0);
    for (int base = 0; base < dmax; base += 16) {
        const uint32_t nxt = base + 16 < dmax ? src_at(base + 16) : zero;
        {
            const uint64_t x0 = word(row_bcast<0>(cur)), x1 = word(row_bcast<1>(cur)),
                           x2 = word(row_bcast<2>(cur)), x3 = word(row_bcast<3>(cur)),
                           x4 = word(row_bcast<4>(cur)), x5 = word(row_bcast<5>(cur)),
                           x6 = word(row_bcast<6>(cur)), x7 = word(row_bcast<7>(cur));
            bs_add4<L>(c, x0, x1, x2, x3);
            bs_add4<L>(c, x4, x5, x6, x7);
        }
        if (dmax - base > 8) {
            const uint64_t x0 = word(row_bcast<8>(cur)), x1 = word(row_bcast<9>(cur)),
                           x2 = word(row_bcast<10>(cur)), x3 = word(row_bcast<11>(cur)),
                           x4 = word(row_bcast<12>(cur)), x5 = word(row_bcast<13>(cur)),
                           x6 = word(row_bcast<14>(cur)), x7 = word(row_bcast<15>(cur));
            bs_add4<L>(c, x0, x1, x2, x3);
            bs_add4<L>(c, x4, x5, x6, x7);
        }
        cur = nxt;
    }
}

// ------------------------------------------------------ SI / SIS / SIR ----
// Appendix A.1: the log-survival messages of the k infected in-neighbours sum
// to k log(1-beta), so a susceptible node is infected with probability
// 1 - (1-beta)^k; the k-indexed thresholds come from the host.  One draw per
// (node, replicate, step) decides whichever transition the node's state
// allows (infection if S, recovery if I).
// Draw classes of the aligned decision path: a 5-bit code per replicate from
// five bit planes, code = k for k = 1 .. 15 infected in-neighbours, 16 for
// sixteen or more (threshold from the exact count), 17 = infected with a
// recovery draw, 18 = latent (SEIR / SEIS) with an E -> I draw.  The table
// maps a code to its threshold (0 for codes that never fire here); its last
// entry is not a threshold but the mask of the codes 1 .. 15 whose threshold
// always fires (those replicates take no draw).
constexpr int kCodeTable = 32;
constexpr int kCodeAlwaysMask = kCodeTable - 1;

__device__ __forceinline__ uint32_t code_threshold(const StepArgs &a, int code)
{
    if (code >= 1 && code <= 15) return a.tinf[code < a.khat ? code : a.khat];
    if (code == 17) return a.trec;
    if (code == 18) return a.talpha;
    if (code == kCodeAlwaysMask) {
        uint32_t m = 0;
        for (int k = 1; k <= 15; ++k)
            if (a.tinf[k < a.khat ? k : a.khat] == kAlways) m |= 1u << k;
        return m;
    }
    return 0u;
}

// Bit plane K of a bit-sliced counter (zero past its last plane).
template <int K, int L>
__device__ __forceinline__ uint64_t plane(const uint64_t (&c)[L])
{
    if constexpr (K < L) return c[K];
    else return 0ull;
}

// Spread the four bits of a nibble to bit 0 of the four bytes of a word.
__device__ __forceinline__ uint32_t spread4(uint32_t n, uint32_t mul, uint32_t mask)
{
    return __umul24(n, mul) & mask;
}

// SWIR (states S, W weakened, I, R; a reading of the model the paper only
// names): with k infected in-neighbours a susceptible replicate becomes I if
// its draw fires against thr(1-(1-kappa)^k), else W if it fires against
// thr(1-(1-kappa-mu)^k); a weakened one becomes I against thr(1-(1-nu)^k);
// an infected one is removed after one step.  One draw per (node, replicate,
// step), taken only where k >= 1; counts are exact per replicate here (the
// model is off the hot path).  `wk` is the weakened plane.
__device__ __forceinline__ uint32_t swir_table(const uint32_t *t, int32_t khat, uint32_t k)
{
    return t[k > (uint32_t)khat ? (uint32_t)khat : k];
}

template <int LC>
__device__ __forceinline__ void swir_decide(const StepArgs &a, int G, int S, bool valid, int v,
                                            int w, int64_t idx, uint64_t h, uint64_t r, uint64_t wk,
                                            uint64_t sus, const uint64_t (&c)[LC], int s,
                                            uint64_t share, bool &any)
{
    const uint64_t gbase = a.goff + 64ull * (uint64_t)w;
    uint64_t need = (sus | wk) & bs_nonzero<LC>(c) & share;
    uint64_t toI = 0, toW = 0;
    while (need) {
        const int b = __builtin_ctzll(need);
        const int gs = b - (int)((gbase + (uint64_t)b) & 3u);  // first bit of the block
        const uint32_t blk = (uint32_t)((gbase + (uint64_t)b) >> 2);
        const uint32_t nn = nibble_at(need, gs);
        need &= ~nibble_to_word(0xFu, gs);
        const U4 o = philox10((uint32_t)v, blk, a.step, kDomNodeStep << 24, a.key0, a.key1);
        const uint32_t ou[4] = {o.x, o.y, o.z, o.w};
        const uint32_t ns = nibble_at(sus, gs);
        uint32_t fi = 0, fw = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!((nn >> j) & 1u)) continue;
            const uint32_t k = bs_get<LC>(c, gs + j);
            if ((ns >> j) & 1u) {
                if (fires(ou[j], swir_table(a.tinf, a.khat, k)))
                    fi |= 1u << j;
                else if (fires(ou[j], swir_table(a.tsiw, a.khat_siw, k)))
                    fw |= 1u << j;
            } else if (fires(ou[j], swir_table(a.twi, a.khat_wi, k))) {
                fi |= 1u << j;
            }
        }
        toI |= nibble_to_word(fi, gs);
        toW |= nibble_to_word(fw, gs);
    }
    toI = or_reduce_lanes(toI, G, S);
    toW = or_reduce_lanes(toW, G, S);
    if (!valid || s != 0) return;
    a.next[idx] = toI;               // infected for one step
    a.lat[idx] = (wk & ~toI) | toW;
    a.aux[idx] = r | h;              // removed after it
    any |= toI != 0;
}

template <int LC>
__device__ __forceinline__ void epi_decide(const StepArgs &a, int G, int S, bool valid, int v,
                                           int w, int64_t idx, uint64_t h, uint64_t r, uint64_t e,
                                           uint64_t sus, const uint64_t (&c)[LC], int s,
                                           uint64_t share, const uint32_t *tl, int tl_n,
                                           const uint32_t *tcode, bool &any)
{
    if (a.model == kSWIR) {
        swir_decide<LC>(a, G, S, valid, v, w, idx, h, r, e, sus, c, s, share, any);
        return;
    }
    const uint64_t gbase = a.goff + 64ull * (uint64_t)w;
    const bool draw_rec = a.trec != 0u && a.trec != kAlways;
    const bool draw_lat = a.talpha != 0u && a.talpha != kAlways;
    const uint32_t trec = a.trec, tlat = a.talpha;
    uint64_t inf = 0, rec = 0, act = 0;  // S -> I or E, I -> R or S, E -> I
    uint32_t ncalls = 0;                 // generator calls of this lane
    if (tcode != nullptr && (a.goff & 3u) == 0u) {
        // generator blocks are nibbles of the word: one draw per block with
        // any replicate that needs one, the class of each replicate read from
        // five bit planes, its threshold from the code table
        uint64_t rest = 0;  // sixteen or more
#pragma unroll
        for (int l = 4; l < LC; ++l) rest |= c[l];
        const uint64_t c0 = plane<0>(c), c1 = plane<1>(c), c2 = plane<2>(c), c3 = plane<3>(c);
        const uint64_t ninf = sus & share & (c0 | c1 | c2 | c3 | rest);  // k >= 1
        uint64_t always = 0;  // classes whose threshold always fires
        const uint32_t acodes = tcode[kCodeAlwaysMask];
        if (acodes) {
            for (int k = 1; k <= 15; ++k)
                if ((acodes >> k) & 1u)
                    always |= ~rest & ((k & 1) ? c0 : ~c0) & ((k & 2) ? c1 : ~c1) &
                              ((k & 4) ? c2 : ~c2) & ((k & 8) ? c3 : ~c3);
            always &= ninf;
        }
        const uint64_t ndraw = ninf & ~always;
        const uint64_t nrec = draw_rec ? (h & share) : 0ull;
        const uint64_t nlat = draw_lat ? (e & share) : 0ull;
        const uint64_t low = ndraw & ~rest;
        const uint64_t P0 = (low & c0) | nrec, P1 = (low & c1) | nlat, P2 = low & c2,
                       P3 = low & c3, P4 = (ndraw & rest) | nrec | nlat;
        uint64_t need = ndraw | nrec | nlat;
        uint64_t fire = 0;
        const uint32_t blk0 = (uint32_t)(gbase >> 2);
        while (need) {
            const int b = __builtin_ctzll(need);
            const int gs = b & ~3;
            need &= ~(0xFull << gs);
            const bool hi = gs >= 32;
            const uint32_t sh = (uint32_t)gs & 31u;
            auto nib = [&](uint64_t P) -> uint32_t {
                return ((hi ? (uint32_t)(P >> 32) : (uint32_t)P) >> sh) & 0xFu;
            };
            const uint32_t n0 = nib(P0), n1 = nib(P1), n2 = nib(P2), n3 = nib(P3), n4 = nib(P4);
            // byte j of T = 4 * code of replicate j (a byte offset into the table)
            const uint32_t T = spread4(n0, 0x810204u, 0x04040404u) |
                               (spread4(n1, 0x204081u, 0x01010101u) << 3) |
                               (spread4(n2, 0x204081u, 0x01010101u) << 4) |
                               (spread4(n3, 0x204081u, 0x01010101u) << 5) |
                               (spread4(n4, 0x204081u, 0x01010101u) << 6);
            const char *tb = reinterpret_cast<const char *>(tcode);
            const uint32_t q0 = *reinterpret_cast<const uint32_t *>(tb + (T & 0xFFu));
            const uint32_t q1 = *reinterpret_cast<const uint32_t *>(tb + ((T >> 8) & 0xFFu));
            const uint32_t q2 = *reinterpret_cast<const uint32_t *>(tb + ((T >> 16) & 0xFFu));
            const uint32_t q3 = *reinterpret_cast<const uint32_t *>(tb + (T >> 24));
            const U4 o = philox10((uint32_t)v, blk0 + ((uint32_t)gs >> 2), a.step,
                                  kDomNodeStep << 24, a.key0, a.key1);
            ++ncalls;
            uint32_t f = (o.w < q3) ? 1u : 0u;
            f = f + f + ((o.z < q2) ? 1u : 0u);
            f = f + f + ((o.y < q1) ? 1u : 0u);
            f = f + f + ((o.x < q0) ? 1u : 0u);
            const uint32_t nb = n4 & ~n0 & ~n1;  // code 16: sixteen or more infected neighbours
            if (nb) {
                const uint32_t ou[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if ((nb >> j) & 1u)
                        f |= (fires(ou[j], tinf_at(a, tl, tl_n, bs_get<LC>(c, gs + j))) ? 1u : 0u)
                             << j;
            }
            fire |= (uint64_t)f << gs;
        }
        inf = (fire & ~h & ~e) | always;
        rec = fire & h;
        act = fire & e;
    } else {
        uint64_t need = sus & bs_nonzero<LC>(c);
        if (draw_rec) need |= h;
        if (draw_lat) need |= e;
        need &= share;
        const SmallCounts sm = bs_small<LC>(c);
        const uint64_t big = sus & ~(sm.m1 | sm.m2 | sm.m3) & bs_nonzero<LC>(c);  // k >= 4
        const uint32_t t1 = tinf_at(a, tl, tl_n, 1u), t2 = tinf_at(a, tl, tl_n, 2u),
                       t3 = tinf_at(a, tl, tl_n, 3u);
        while (need) {
            const int b = __builtin_ctzll(need);
            const int gs = b - (int)((gbase + (uint64_t)b) & 3u);  // first bit of the block
            const uint32_t blk = (uint32_t)((gbase + (uint64_t)b) >> 2);
            const uint32_t nn = nibble_at(need, gs);
            need &= ~nibble_to_word(0xFu, gs);
            const U4 o = philox10((uint32_t)v, blk, a.step, kDomNodeStep << 24, a.key0, a.key1);
            ++ncalls;
            const uint32_t ou[4] = {o.x, o.y, o.z, o.w};
            const uint32_t nh = nibble_at(h, gs), ne = nibble_at(e, gs), n1 = nibble_at(sm.m1, gs),
                           n2 = nibble_at(sm.m2, gs), n3 = nibble_at(sm.m3, gs),
                           nb = nibble_at(big, gs);
            uint32_t tb[4] = {0u, 0u, 0u, 0u};
            if (nb) {  // a replicate of this block has four or more infected neighbours
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if ((nb >> j) & 1u) tb[j] = tinf_at(a, tl, tl_n, bs_get<LC>(c, gs + j));
            }
            uint32_t fi = 0, fr = 0, fe = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool isI = (nh >> j) & 1u, isE = (ne >> j) & 1u;
                uint32_t t = ((n1 >> j) & 1u) ? t1
                                              : (((n2 >> j) & 1u) ? t2 : (((n3 >> j) & 1u) ? t3 : tb[j]));
                t = isI ? trec : (isE ? tlat : t);
                const uint32_t f = (((nn >> j) & 1u) && fires(ou[j], t)) ? 1u : 0u;
                fi |= ((isI || isE) ? 0u : f) << j;
                fr |= (isI ? f : 0u) << j;
                fe |= (isE ? f : 0u) << j;
            }
            inf |= nibble_to_word(fi, gs);
            rec |= nibble_to_word(fr, gs);
            act |= nibble_to_word(fe, gs);
        }
    }
    if (a.draws) {  // counting runs only (all 64 lanes are here together)
        for (int off = 32; off >= 1; off >>= 1) ncalls += (uint32_t)__shfl_xor((int)ncalls, off, 64);
        if ((threadIdx.x & 63) == 0 && ncalls) atomicAdd(a.draws, (unsigned long long)ncalls);
    }
    inf = or_reduce_lanes(inf, G, S);
    rec = or_reduce_lanes(rec, G, S);
    act = or_reduce_lanes(act, G, S);
    if (a.trec == kAlways) rec = h;
    if (a.talpha == kAlways) act = e;
    if (!valid || s != 0) return;
    if (a.lat) {  // SEIR / SEIS: infection leads to E, E -> I
        const uint64_t nh = (h & ~rec) | act;
        const uint64_t ne = (e & ~act) | inf;
        a.next[idx] = nh;
        a.lat[idx] = ne;
        if (a.model == kSEIR) a.aux[idx] = r | rec;
        any |= (nh | ne) != 0;
        return;
    }
    const uint64_t nh = (h & ~rec) | inf;
    const uint64_t nr = (a.model == kSIS) ? r : (r | rec);
    a.next[idx] = nh;
    a.aux[idx] = nr;
    any |= nh != 0;
}

// Tail mode: node v has an infected replicate after step t (bitmap t % 4).
__device__ __forceinline__ void mark_infected(const StepArgs &a, int v)
{
    atomicOr(&a.ibm[(size_t)(a.step & 3u) * (size_t)a.ibm_words + (size_t)(v >> 5)], 1u << (v & 31));
}

template <int L>
__device__ __forceinline__ void epi_row_word(const StepArgs &a, int G, int S, bool valid, int v,
                                             int w, int e0, int e1, int s, int seg,
                                             uint64_t share, const uint32_t *tl, int tl_n,
                                             const uint32_t *tcode, uint64_t lm, bool &any)
{
    const int64_t idx = (int64_t)v * a.W + w;
    const uint64_t h = valid ? a.prev[idx] : 0ull;
    const uint64_t r = valid ? a.aux[idx] : 0ull;
    const uint64_t e = (valid && a.lat) ? a.lat[idx] : 0ull;
    const uint64_t sus = valid ? (~(h | r | e) & tail_mask(w, a.B) & lm) : 0ull;
    // replicates whose decision needs the count (SWIR: weakened ones too)
    const uint64_t counted = a.model == kSWIR ? (sus | (e & lm)) : sus;
    uint64_t c[L];
#pragma unroll
    for (int l = 0; l < L; ++l) c[l] = 0;
    if (S == 1 && G >= 16 && a.fast32)
        count_edges_bcast<L>(a, G, valid, e0, e1, w, counted != 0ull, c);
    else if (counted)
        count_edges<L>(a, e0 + s, e1, S, w, c);
    bs_reduce_lanes<L>(c, G, S);
    if (seg >= 0) {
        if (valid && s == 0) {
#pragma unroll
            for (int l = 0; l < L; ++l) a.partial[((int64_t)seg * L + l) * a.W + w] = c[l];
        }
        return;
    }
    epi_decide<L>(a, G, S, valid, v, w, idx, h, r, e, sus, c, s, share, tl, tl_n, tcode, any);
}

// ---------------------------------------------------------------- LT ----
// In-weights 1/indeg and threshold U/2^32 drawn once per (node, replicate):
// v activates once c active in-neighbours satisfy c >= ceil(U indeg / 2^32)
// (and c >= 1).
constexpr int kPlaneBlocks = 4;

template <int LC>
__device__ __forceinline__ void lt_decide(const StepArgs &a, int G, int S, bool valid, int v,
                                          int w, int64_t idx, uint64_t act, uint64_t inact,
                                          uint32_t indeg, const uint64_t (&c)[LC], int s,
                                          uint64_t share, bool use_need, bool &any)
{
    const uint64_t gbase = a.goff + 64ull * (uint64_t)w;
    uint64_t nw = 0;
    const int P = indeg ? 32 - __builtin_clz(indeg) : 0;  // planes of the stored thresholds
    uint64_t nz = 0;
#pragma unroll
    for (int l = 0; l < LC; ++l) nz |= c[l];
    const uint64_t cand = inact & share & nz;
    // Stored thresholds cost bitlen(indeg) word loads, a fresh draw one
    // Philox call per 4-replicate block with a candidate: the wave reads the
    // planes when some lane has more than kPlaneBlocks such blocks.
    bool planes = false;
    if (use_need && a.need != nullptr) {
        uint64_t blk = cand | (cand >> 1) | (cand >> 2) | (cand >> 3);
        blk &= 0x1111111111111111ull;
        planes = __ballot(__popcll(blk) > kPlaneBlocks) != 0ull;
    }
    if (planes && P <= LC) {
        // v activates in replicate r iff c_r >= need_r, i.e. iff c - need
        // does not borrow (the chain runs plane by plane over the word)
        if (cand) {
            const uint64_t *np = a.need + (int64_t)v * a.Lp * a.W + w;
            uint64_t borrow = 0;
#pragma unroll
            for (int l = 0; l < LC; ++l) {
                const uint64_t nl = l < P ? np[(int64_t)l * a.W] : 0ull;
                borrow = maj3(~c[l], nl, borrow);
            }
            nw = cand & ~borrow;
        }
    } else if ((a.goff & 3u) == 0u) {
        // aligned generator blocks, branch-free per block: c = c0 + 2 c1
        // when no higher plane is set; v activates iff c 2^32 >= U indeg,
        // i.e. iff c > hi or (c == hi and lo == 0) for U indeg = hi 2^32 + lo.
        // Replicates whose every in-neighbour is active (c == indeg) always
        // activate and need no draw.
        uint64_t rest = 0;
#pragma unroll
        for (int l = 2; l < LC; ++l) rest |= c[l];
        const uint64_t c0 = c[0], c1 = LC > 1 ? c[LC > 1 ? 1 : 0] : 0ull;
        const uint64_t cand = inact & share & (c0 | c1 | rest);
        uint64_t full = cand;  // c == indeg, plane by plane
#pragma unroll
        for (int l = 0; l < LC; ++l) full &= ((indeg >> l) & 1u) ? c[l] : ~c[l];
        if (((uint64_t)indeg >> LC) != 0ull) full = 0;  // c < 2^LC <= indeg
        uint64_t need = cand & ~full;
        uint64_t fire = 0;
        const uint32_t blk0 = (uint32_t)(gbase >> 2);
        while (need) {
            const int b = __builtin_ctzll(need);
            const int gs = b & ~3;
            const bool hi32 = gs >= 32;
            const uint32_t sh = (uint32_t)gs & 31u;
            const uint32_t nn = ((hi32 ? (uint32_t)(need >> 32) : (uint32_t)need) >> sh) & 0xFu;
            need &= ~(0xFull << gs);
            const uint32_t n0 = ((hi32 ? (uint32_t)(c0 >> 32) : (uint32_t)c0) >> sh) & 0xFu;
            const uint32_t n1 = ((hi32 ? (uint32_t)(c1 >> 32) : (uint32_t)c1) >> sh) & 0xFu;
            const uint32_t nr = ((hi32 ? (uint32_t)(rest >> 32) : (uint32_t)rest) >> sh) & 0xFu;
            const U4 o = philox10((uint32_t)v, blk0 + ((uint32_t)gs >> 2), 0u, kDomLtThresh << 24,
                                  a.key0, a.key1);
            const uint32_t ou[4] = {o.x, o.y, o.z, o.w};
            uint32_t f = 0;
#pragma unroll
            for (int j = 3; j >= 0; --j) {
                uint32_t k = ((n0 >> j) & 1u) + 2u * ((n1 >> j) & 1u);
                if ((nr >> j) & 1u) k = bs_get<LC>(c, gs + j);  // four or more active
                const uint64_t prod = (uint64_t)ou[j] * (uint64_t)indeg;
                const uint32_t ph = (uint32_t)(prod >> 32), pl = (uint32_t)prod;
                f = f + f + ((k > ph || (k == ph && pl == 0u)) ? 1u : 0u);
            }
            fire |= (uint64_t)(f & nn) << gs;
        }
        nw = fire | full;
    } else {
    uint64_t cand = inact & bs_nonzero<LC>(c) & share;
    const SmallCounts sm = bs_small<LC>(c);
    while (cand) {
        const int b = __builtin_ctzll(cand);
        const int gs = b - (int)((gbase + (uint64_t)b) & 3u);
        const uint32_t blk = (uint32_t)((gbase + (uint64_t)b) >> 2);
        const uint32_t nc = nibble_at(cand, gs);
        cand &= ~nibble_to_word(0xFu, gs);
        const U4 o = philox10((uint32_t)v, blk, 0u, kDomLtThresh << 24, a.key0, a.key1);
        const uint32_t ou[4] = {o.x, o.y, o.z, o.w};
        const uint32_t n1 = nibble_at(sm.m1, gs), n2 = nibble_at(sm.m2, gs),
                       n3 = nibble_at(sm.m3, gs);
        uint32_t fa = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!((nc >> j) & 1u)) continue;
            uint32_t k = ((n1 >> j) & 1u) ? 1u : (((n2 >> j) & 1u) ? 2u : (((n3 >> j) & 1u) ? 3u : 0u));
            if (k == 0u) k = bs_get<LC>(c, gs + j);  // four or more active neighbours
            // c >= 1 here, so max(1, need) = need
            const uint64_t need = ((uint64_t)ou[j] * (uint64_t)indeg + 0xFFFFFFFFull) >> 32;
            if ((uint64_t)k >= need) fa |= 1u << j;
        }
        nw |= nibble_to_word(fa, gs);
    }
    }
    nw = or_reduce_lanes(nw, G, S);
    if (!valid || s != 0) return;
    a.next[idx] = act | nw;
    if (nw != 0ull && a.stamp != nullptr)
        a.stamp[(size_t)(a.step & 1u) * (size_t)a.n + (size_t)v] = a.step;
    any |= nw != 0;
}

template <int L>
__device__ __forceinline__ void lt_row_word(const StepArgs &a, int G, int S, bool valid, int v,
                                            int w, int e0, int e1, uint32_t indeg, int s, int seg,
                                            uint64_t share, uint64_t lm, bool &any)
{
    const int64_t idx = (int64_t)v * a.W + w;
    const uint64_t act = valid ? a.prev[idx] : 0ull;
    const uint64_t inact = valid ? (~act & tail_mask(w, a.B) & lm) : 0ull;
    uint64_t c[L];
#pragma unroll
    for (int l = 0; l < L; ++l) c[l] = 0;
    if (S == 1 && G >= 16 && a.fast32)
        count_edges_bcast<L>(a, G, valid, e0, e1, w, inact != 0ull, c);
    else if (inact)
        count_edges<L>(a, e0 + s, e1, S, w, c);
    bs_reduce_lanes<L>(c, G, S);
    if (seg >= 0) {
        if (valid && s == 0) {
#pragma unroll
            for (int l = 0; l < L; ++l) a.partial[((int64_t)seg * L + l) * a.W + w] = c[l];
        }
        return;
    }
    lt_decide<L>(a, G, S, valid, v, w, idx, act, inact, indeg, c, s, share, true, any);
}

__device__ __forceinline__ uint32_t wc_threshold(uint32_t indeg)
{
    // weighted cascade p = 1/indeg: floor(2^32 / indeg), 1 -> always
    return indeg <= 1u ? kAlways : (uint32_t)(0x100000000ull / (uint64_t)indeg);
}

template <int KIND, int L>
__device__ __forceinline__ void row_word(const StepArgs &a, int G, int S, bool valid, int v, int w,
                                         int e0, int e1, uint32_t indeg, int s, int seg,
                                         uint64_t share_fixed, const uint32_t *tl, int tl_n,
                                         const uint32_t *tcode, uint64_t lm,
                                         bool &any)
{
    // draws of lane s: generator blocks congruent to s mod S; for S <= 16 the
    // pattern repeats every word, otherwise it depends on the word
    const uint64_t share =
        S <= 16 ? share_fixed : share_bits(a.goff + 64ull * (uint64_t)w, s, S);
    if (KIND == kKindIC) {
        uint32_t tv = a.ic_t;
        if (a.ic_prob == kIcWeightedCascade) tv = wc_threshold(indeg);
        ic_row_word(a, G, S, valid, v, w, e0, e1, tv, s, seg, lm, any);
    } else if (KIND == kKindEpidemic) {
        epi_row_word<L>(a, G, S, valid, v, w, e0, e1, s, seg, share, tl, tl_n, tcode, lm, any);
    } else {
        lt_row_word<L>(a, G, S, valid, v, w, e0, e1, indeg, s, seg, share, lm, any);
    }
}

// Words a wave works on at step t = a.step.  A word whose flag is clear
// after step t-1 cannot change at step t (no frontier, no infectious or
// latent replicate, or no activation under fixed thresholds).  If its flag
// after step t-2 is clear too, the state buffer step t writes already holds
// the word's state (state t-2 = t-1 = t) and the word is left out; otherwise
// it takes a pass with its candidates masked off, which copies it forward.
// `any` lists the words worked on, `live` those with candidates; with word
// flags, pass k gives lane gw the (k G + gw)-th word of `any`.
struct WordMap {
    uint64_t any, live;
    int passes, count;
    bool compact;
};

// All 64 lanes of the wave call this together.
__device__ __forceinline__ WordMap word_map(const StepArgs &a, int G)
{
    WordMap m;
    m.compact = a.wflags != nullptr;
    if (!m.compact) {
        m.any = m.live = ~0ull;
        m.count = a.W;
    } else {
        const uint32_t t = a.step, wr = (uint32_t)a.wring;
        const uint32_t *f1 = a.wflags + (size_t)((t - 1u) % wr) * (size_t)a.W;
        const uint32_t *f2 = a.wflags + (size_t)((t + wr - 2u) % wr) * (size_t)a.W;
        const int lane = (int)(threadIdx.x & 63u);
        uint32_t x1 = 0u, x2 = 0u;
        if (lane < a.W) {
            x1 = f1[lane];
            x2 = f2[lane];
        }
        m.live = __ballot(x1 != 0u);
        m.any = __ballot((x1 | x2) != 0u);
        m.count = __popcll(m.any);
    }
    m.passes = (m.count + G - 1) / G;
    return m;
}

// Position of the j-th (from 0) set bit of m; j < popcount(m).
__device__ __forceinline__ int nth_set_bit(uint64_t m, int j)
{
    int pos = 0;
    int c = __popc((uint32_t)m);
    if (j >= c) {
        j -= c;
        m >>= 32;
        pos = 32;
    }
    uint32_t x = (uint32_t)m;
    c = __popc(x & 0xFFFFu);
    if (j >= c) { j -= c; x >>= 16; pos += 16; }
    c = __popc(x & 0xFFu);
    if (j >= c) { j -= c; x >>= 8; pos += 8; }
    c = __popc(x & 0xFu);
    if (j >= c) { j -= c; x >>= 4; pos += 4; }
    c = __popc(x & 0x3u);
    if (j >= c) { j -= c; x >>= 2; pos += 2; }
    if (j >= (int)(x & 1u)) pos += 1;
    return pos;
}

// Word of lane gw in pass k, whether it exists, and its candidate mask.
__device__ __forceinline__ int word_of(const WordMap &m, int k, int G, int gw, bool &ok,
                                       uint64_t &lm)
{
    const int j = k * G + gw;
    ok = j < m.count;
    if (!m.compact) {
        lm = ~0ull;
        return ok ? j : 0;
    }
    const int w = ok ? nth_set_bit(m.any, j) : 0;
    lm = ((m.live >> w) & 1ull) ? ~0ull : 0ull;
    return w;
}

// Records the word flags of step a.step: lanes of one pass that share gw
// share the word, so the ballot is folded onto its low G bits and lane gw
// stores for its word.  All 64 lanes of the wave call this together.
__device__ __forceinline__ void note_words(const StepArgs &a, int G, int w, bool ok, bool anyw)
{
    if (a.wflags == nullptr) return;
    uint64_t m = __ballot(anyw);
    if (m == 0ull) return;
    for (int sh = 32; sh >= G; sh >>= 1) m |= m >> sh;
    const int lane = (int)(threadIdx.x & 63u);
    if (lane < G && ((m >> lane) & 1ull) && ok)
        a.wflags[(size_t)(a.step % (uint32_t)a.wring) * (size_t)a.W + (size_t)w] = 1u;
}

// Work of one block of the pull step: block `bid` < seg_blocks owns heavy-row
// segments (one per row slot; long, so they start first), the rest own light
// tiles.  Returns through `any` whether a state-1 node remains.
template <int KIND, int L, bool TAIL = false>
__device__ __forceinline__ void step_block(const StepArgs &a, int bid, const uint32_t *tl,
                                           int tl_n, const uint32_t *tcode, bool &any)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int S = a.S;
    const WordMap wm = word_map(a, a.G);
    // heavy-row segments take a whole wave each: G lanes over words, the
    // other 64 / G lanes over the segment's arcs
    const int seg_blocks = (a.n_seg + nwaves - 1) / nwaves;
    if (bid >= seg_blocks) {
        // light rows: once fewer words are left than the row has word lanes,
        // the row gets next_pow2(words) lanes (not below 16, which keeps the
        // DPP source broadcast) and the wave takes more rows
        int lgGe = a.lgG;
        if (wm.compact) {
            int lg = 0;
            while ((1 << lg) < wm.count) ++lg;
            const int lo = a.lgG < 4 ? a.lgG : 4;
            lgGe = lg < lo ? lo : (lg > a.lgG ? a.lgG : lg);
        }
        const int Ge = 1 << lgGe;
        const int rpwe = 64 >> (lgGe + a.lgS);
        const int slote = lane >> (lgGe + a.lgS);
        const int se = (lane >> lgGe) & (S - 1);
        const int gwe = lane & (Ge - 1);
        const uint64_t share_e = S <= 16 ? share_bits(a.goff, se, S) : 0ull;
        const int passes = (wm.count + Ge - 1) / Ge;
        const int tile = bid - seg_blocks;
        const int t0 = a.tiles[2 * tile], t1 = a.tiles[2 * tile + 1];
        // LT once at most half of the words are left: thresholds are fixed,
        // so a row none of whose in-neighbours gained an activation at step
        // t-1 has the counts it was last decided on and cannot activate; it
        // takes the copy pass without counting (earlier, nearly every row
        // has such a neighbour and the test would only add loads)
        // tail mode: a row that is not a candidate -- itself and its
        // in-neighbours without an infected replicate (SI family) or without
        // a new activation (IC, LT) after step t-1 -- cannot change at step t
        constexpr bool kTailKind = TAIL;
        const bool fresh_test = KIND == kKindLT && a.stamp != nullptr && wm.compact &&
                                wm.count * 2 <= a.W && !(kTailKind && a.ibm != nullptr);
        const int rl = 1 << (lgGe + a.lgS);  // lanes of a row
        const uint64_t rowmask = (rl == 64 ? ~0ull : ((1ull << rl) - 1ull)) << (slote * rl);
        for (int rb = t0 + wave * rpwe; rb < t1; rb += nwaves * rpwe) {
            const int v = rb + slote;
            bool act = v < t1;
            int e0 = 0, e1 = 0;
            if (act) {
                e0 = a.ptr[v];
                e1 = a.ptr[v + 1];
                if (e1 - e0 > a.heavy) act = false;
            }
            uint64_t rowlm = ~0ull;
            if (kTailKind && a.ibm != nullptr && act) {
                const uint32_t *cand = a.cand + (size_t)(a.step & 1u) * a.ibm_words;
                if (!((cand[v >> 5] >> (v & 31)) & 1u)) {
                    // left out: its state after step t is its state after
                    // t-1.  The buffer step t writes holds the state after
                    // t-2: for LT that is the same (no activation at t-1);
                    // for the SI family it differs only if the node had an
                    // infected replicate then (none after t-1), for IC (the
                    // buffer holds new activations) if it had a new
                    // activation then (none at t)
                    if (KIND != kKindLT) {
                        const uint32_t *inf2 = a.ibm + (size_t)((a.step - 2u) & 3u) * a.ibm_words;
                        if ((inf2[v >> 5] >> (v & 31)) & 1u)
                            for (int w = lane & (rl - 1); w < a.W; w += rl)
                                a.next[(int64_t)v * a.W + w] = 0ull;
                    }
                    act = false;
                }
            }
            if (fresh_test) {
                const uint32_t *gained = a.stamp + (size_t)((a.step - 1u) & 1u) * (size_t)a.n;
                bool f = false;
                if (act)
                    for (int e = e0 + (lane & (rl - 1)); e < e1 && !f; e += rl)
                        f = gained[a.src[e]] == a.step - 1u;
                if ((__ballot(f) & rowmask) == 0ull) rowlm = 0ull;
            }
            for (int k = 0; k < passes; ++k) {
                bool ok;
                uint64_t lm;
                const int w = word_of(wm, k, Ge, gwe, ok, lm);
                bool anyw = false;
                row_word<KIND, L>(a, Ge, S, act && ok, v, w, e0, e1, (uint32_t)(e1 - e0), se, -1,
                                  share_e, tl, tl_n, tcode, lm & rowlm, anyw);
                note_words(a, Ge, w, ok, anyw);
                // anyw: an infected replicate (SI family) or a new activation
                // (IC, LT) in this word after the step
                if (kTailKind && anyw && a.ibm != nullptr) mark_infected(a, v);
                any |= anyw;
            }
        }
    } else {
        // with fewer words left than word lanes, next_pow2(words) word lanes
        // and the rest over the segment's arcs (a shorter chain per lane)
        int lgGs = a.lgG;
        if (wm.compact) {
            int lg = 0;
            while ((1 << lg) < wm.count) ++lg;
            lgGs = lg > a.lgG ? a.lgG : lg;
        }
        const int Gs = 1 << lgGs;
        const int Ss = 64 >> lgGs;  // edge lanes of a segment
        const int ss = lane >> lgGs;
        const int gws = lane & (Gs - 1);
        const int passes = (wm.count + Gs - 1) / Gs;
        const uint64_t share_seg = Ss <= 16 ? share_bits(a.goff, ss, Ss) : 0ull;
        const int seg = bid * nwaves + wave;
        const bool act = seg < a.n_seg;
        int v = 0, e0 = 0, e1 = 0;
        uint32_t indeg = 0;
        if (act) {
            v = a.seg_row[seg];
            e0 = a.seg_e0[seg];
            e1 = a.seg_e1[seg];
            indeg = (uint32_t)(a.ptr[v + 1] - a.ptr[v]);
        }
        for (int k = 0; k < passes; ++k) {
            bool ok;
            uint64_t lm;
            const int w = word_of(wm, k, Gs, gws, ok, lm);
            row_word<KIND, L>(a, Gs, Ss, act && ok, v, w, e0, e1, indeg, ss, act ? seg : 0,
                              share_seg, tl, tl_n, tcode, lm, any);
        }
    }
}

// Tail mode: whether light-row block `bid` has nothing to do at step t -- no
// candidate row and no row infected (IC: newly activated) after t-2, whose
// buffer word must be cleared, in its tile.  The bitmap words at the tile's
// ends may hold other tiles' rows, which only makes the test keep a tile it
// could have left.
// Every wave of the block reads the same words and gets the same answer.
__device__ __forceinline__ bool tail_tile_idle(const StepArgs &a, int bid, bool zero_store)
{
    const int nwaves = blockDim.x >> 6;
    const int seg_blocks = (a.n_seg + nwaves - 1) / nwaves;
    if (bid < seg_blocks) return false;
    const int tile = bid - seg_blocks;
    const int t0 = a.tiles[2 * tile], t1 = a.tiles[2 * tile + 1];
    if (t1 <= t0) return true;
    const uint32_t *cand = a.cand + (size_t)(a.step & 1u) * a.ibm_words;
    const uint32_t *inf2 = a.ibm + (size_t)((a.step - 2u) & 3u) * a.ibm_words;
    bool busy = false;
    for (int i = (t0 >> 5) + (int)(threadIdx.x & 63); i <= ((t1 - 1) >> 5) && !busy; i += 64)
        busy = (cand[i] | (zero_store ? inf2[i] : 0u)) != 0u;
    return __ballot(busy) == 0ull;
}

// One synchronous step t = a.step of one job.
template <int KIND, int L, bool TAIL = false>
__global__ void __launch_bounds__(1024) k_step(StepArgs a)
{
    if (a.flags[(a.step - 1) % (uint32_t)a.ring] == 0u) return;  // nothing left to change
    if (TAIL && a.ibm != nullptr) {
        // the bitmaps step t+1 sets, then whether this block has work
        uint32_t *clr = a.ibm + (size_t)((a.step + 1u) & 3u) * a.ibm_words;
        uint32_t *cclr = a.cand + (size_t)((a.step + 1u) & 1u) * a.ibm_words;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.ibm_words;
             i += (int64_t)gridDim.x * blockDim.x) {
            clr[i] = 0u;
            cclr[i] = 0u;
        }
        if (tail_tile_idle(a, blockIdx.x, KIND != kKindLT)) return;
    }
    __shared__ uint32_t s_tinf[KIND == kKindEpidemic ? kTinfLds : 1];
    __shared__ uint32_t s_code[kCodeTable];
    int tl_n = 0;
    if (KIND == kKindEpidemic) {
        tl_n = a.khat + 1 < kTinfLds ? a.khat + 1 : kTinfLds;
        for (int i = threadIdx.x; i < tl_n; i += blockDim.x) s_tinf[i] = a.tinf[i];
        if (threadIdx.x < kCodeTable) s_code[threadIdx.x] = code_threshold(a, threadIdx.x);
        __syncthreads();
    }
    bool any = false;
    step_block<KIND, L, TAIL>(a, blockIdx.x, s_tinf, tl_n, s_code, any);
    if (__ballot(any) != 0ull && (threadIdx.x & 63) == 0) a.flags[a.step % (uint32_t)a.ring] = 1u;
}

// Merge of the segment partials of heavy row group `bid` (rows_per_block
// heavy rows), then the same update as a light row.  G lanes per row over
// words, no edge split.
template <int KIND, int LP>
__device__ __forceinline__ void combine_block(const StepArgs &a, int bid, const uint32_t *tcode,
                                              bool &any)
{
    constexpr int LC = 32;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int G = a.G;
    // G lanes over words times S2 lanes over the row's segments (S2 <= 16,
    // the widest split the draw-sharing masks cover), combine_rows_per_wave
    // rows per wave; the segment lanes' counts are summed across lanes
    const int lanes = 64 >> a.lgG;
    const int S2 = lanes < 16 ? lanes : 16;
    const int rpw = combine_rows_per_wave(a.lgG);
    const int slot = lane / (G * S2);
    const int ss = (lane >> a.lgG) % S2;
    const int gw = lane & (G - 1);
    const int j = (bid * nwaves + wave) * rpw + slot;
    const bool act = j < a.n_heavy;
    const int v = act ? a.heavy_rows[j] : 0;
    const int sg0 = act ? a.heavy_seg[j] : 0, sg1 = act ? a.heavy_seg[j + 1] : 0;
    const uint64_t share = share_bits(a.goff, ss, S2);
    const WordMap wm = word_map(a, G);
    for (int k = 0; k < wm.passes; ++k) {
        bool ok;
        uint64_t lm;
        const int ww = word_of(wm, k, G, gw, ok, lm);
        const bool valid = act && ok;
        const int64_t idx = (int64_t)v * a.W + ww;
        bool anyw = false;
        if (KIND == kKindIC) {
            uint64_t acc = 0;
            if (valid && lm)
                for (int sg = sg0 + ss; sg < sg1; sg += S2) acc |= a.partial[(int64_t)sg * a.W + ww];
            acc = or_reduce_lanes(acc, G, S2);
            if (valid && ss == 0) {
                const uint64_t A = a.aux[idx];
                acc &= ~A;
                a.next[idx] = acc;
                a.aux[idx] = A | acc;
                anyw = acc != 0;
            }
            if (a.ibm != nullptr && anyw) mark_infected(a, v);  // tail mode
        } else {
            uint64_t c[LC];
#pragma unroll
            for (int l = 0; l < LC; ++l) c[l] = 0;
            if (valid && lm) {
                for (int sg = sg0 + ss; sg < sg1; sg += S2) {
                    uint64_t d[LC];
#pragma unroll
                    for (int l = 0; l < LC; ++l)
                        d[l] = (l < LP) ? a.partial[((int64_t)sg * LP + l) * a.W + ww] : 0ull;
                    bs_add<LC>(c, d);
                }
            }
            bs_reduce_lanes<LC>(c, G, S2);
            if (KIND == kKindEpidemic) {
                const uint64_t h = valid ? a.prev[idx] : 0ull;
                const uint64_t r = valid ? a.aux[idx] : 0ull;
                const uint64_t e = (valid && a.lat) ? a.lat[idx] : 0ull;
                const uint64_t sus = valid ? (~(h | r | e) & tail_mask(ww, a.B) & lm) : 0ull;
                const uint64_t counted = a.model == kSWIR ? (sus | (e & lm)) : sus;
#pragma unroll
                for (int l = 0; l < LC; ++l) c[l] &= counted;
                epi_decide<LC>(a, G, S2, valid, v, ww, idx, h, r, e, sus, c, ss, share, nullptr, 0,
                               tcode, anyw);
                if (a.ibm != nullptr && anyw) mark_infected(a, v);  // tail mode
            } else {
                const uint64_t act_w = valid ? a.prev[idx] : 0ull;
                const uint64_t inact = valid ? (~act_w & tail_mask(ww, a.B) & lm) : 0ull;
#pragma unroll
                for (int l = 0; l < LC; ++l) c[l] &= inact;
                const uint32_t indeg = act ? (uint32_t)(a.ptr[v + 1] - a.ptr[v]) : 0u;
                lt_decide<LC>(a, G, S2, valid, v, ww, idx, act_w, inact, indeg, c, ss, share, false,
                              anyw);
                if (a.ibm != nullptr && anyw) mark_infected(a, v);  // tail mode
            }
        }
        note_words(a, G, ww, ok, anyw);
        any |= anyw;
    }
}

template <int KIND, int LP>
__global__ void __launch_bounds__(256) k_combine(StepArgs a)
{
    if (a.flags[(a.step - 1) % (uint32_t)a.ring] == 0u) return;
    __shared__ uint32_t s_code[kCodeTable];
    if (KIND == kKindEpidemic) {
        if (threadIdx.x < kCodeTable) s_code[threadIdx.x] = code_threshold(a, threadIdx.x);
        __syncthreads();
    }
    bool any = false;
    combine_block<KIND, LP>(a, blockIdx.x, s_code, any);
    if (__ballot(any) != 0ull && (threadIdx.x & 63) == 0) a.flags[a.step % (uint32_t)a.ring] = 1u;
}

// ------------------------------------------- IC, one word per node ----
// Edge-parallel variant for B <= 64 (W = 1): persistent blocks stream the
// whole arc array once per step, four 16-byte source loads per thread per
// pass, and test each source against the frontier: first the summary (one bit
// per 2^sum_shift nodes, in LDS), then, for summary hits, the frontier bitmap
// (N bits, cache-resident).  Only a frontier arc reads its target row (the
// arc's entry of dst), gathers the source word, runs the arc's trials and ORs
// fired replicates into the target's words with atomics; the target joins the
// next frontier.  The step has no tiles and no block barriers, and it reads
// neither the row pointers (except a frontier arc's target degree under the
// weighted cascade) nor the words of rows that do not change.
__device__ __forceinline__ uint32_t ic_threshold(const StepArgs &a, uint32_t indeg)
{
    return a.ic_prob == kIcWeightedCascade ? wc_threshold(indeg) : a.ic_t;
}

// Summary bit of source u's group of 2^sum_shift nodes (LDS copy).
__device__ __forceinline__ bool summary_hit(const StepArgs &a, const uint32_t *s_sum, int u)
{
    const int i = u >> a.sum_shift;
    return (s_sum[i >> 5] >> (i & 31)) & 1u;
}

__device__ __forceinline__ void mark_frontier(const StepArgs &a, int v)
{
    atomicOr(&a.bm_next[v >> 5], 1u << (v & 31));
    const int i = v >> a.sum_shift;
    atomicOr(&a.sum_next[i >> 5], 1u << (i & 31));
}

// Work item k of node v whose out-arcs are oarc[o0 .. o1): (v, k, first arc,
// end of its arcs).
__device__ __forceinline__ uint4 out_item(int v, uint32_t k, int o0, int o1)
{
    const int b = o0 + (int)k * kOutChunk;
    const int e = o1 - b < kOutChunk ? o1 : b + kOutChunk;
    return make_uint4((uint32_t)v, k, (uint32_t)b, (uint32_t)e);
}

// Joins node v to the frontier of step t (its bit in the next bitmap; the
// first thread to set the bit also sets the summary bit and, with a queue,
// appends v's work items and adds its out-degree to the queue's arc count).
template <bool Q>
__device__ __forceinline__ void join_frontier(const StepArgs &a, int v)
{
    if (!Q) {
        mark_frontier(a, v);
        return;
    }
    const uint32_t bit = 1u << (v & 31);
    const uint32_t old = atomicOr(&a.bm_next[v >> 5], bit);
    if (old & bit) return;
    const int i = v >> a.sum_shift;
    atomicOr(&a.sum_next[i >> 5], 1u << (i & 31));
    if (a.ever) atomicOr(&a.ever[v >> 5], bit);
    const int o0 = a.optr[v], o1 = a.optr[v + 1];
    const int deg = o1 - o0;
    const uint32_t nch = deg > kOutChunk ? (uint32_t)((deg + kOutChunk - 1) / kOutChunk) : 1u;
    const uint32_t at = atomicAdd(&a.qcnt[a.qi_out], nch);
    for (uint32_t k = 0; k < nch; ++k) a.q_out[at + k] = out_item(v, k, o0, o1);
    if (deg > 0) atomicAdd(&a.qarcs[a.qi_out], (unsigned long long)deg);
}

// Claims node v for the frontier of step t: sets its bit in the next bitmap
// and returns true for the one thread that set it first (which then sets
// the summary bit and must queue v).
__device__ __forceinline__ bool claim_frontier(const StepArgs &a, int v)
{
    const uint32_t bit = 1u << (v & 31);
    const uint32_t old = atomicOr(&a.bm_next[v >> 5], bit);
    if (old & bit) return false;
    const int i = v >> a.sum_shift;
    atomicOr(&a.sum_next[i >> 5], 1u << (i & 31));
    if (a.ever) atomicOr(&a.ever[v >> 5], bit);
    return true;
}

// Queues the nodes the lanes of a wave claimed (v < 0: none), called by all
// 64 lanes together: one atomic add per wave reserves the items of all of
// them (a shuffle scan gives each lane its offset) and one adds their
// out-arcs; a node with more than 64 items has them written by the whole
// wave.
__device__ __forceinline__ void queue_claimed(const StepArgs &a, int v, int o0, int o1)
{
    const int lane = threadIdx.x & 63;
    const int deg = v >= 0 ? o1 - o0 : 0;
    const uint32_t nch = v < 0 ? 0u : (deg > kOutChunk ? (uint32_t)((deg + kOutChunk - 1) / kOutChunk) : 1u);
    if (__ballot(nch != 0u) == 0ull) return;
    uint32_t incl = nch;
    unsigned long long arcs = (unsigned long long)deg;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t x = (uint32_t)__shfl_up((int)incl, off, 64);
        if (lane >= off) incl += x;
        arcs += __shfl_xor(arcs, off, 64);
    }
    uint32_t base = 0;
    if (lane == 63) {
        base = atomicAdd(&a.qcnt[a.qi_out], incl);
        if (arcs) atomicAdd(&a.qarcs[a.qi_out], arcs);
    }
    base = (uint32_t)__shfl((int)base, 63, 64);
    const uint32_t at = base + incl - nch;
    if (nch <= 64u) {
        for (uint32_t k = 0; k < nch; ++k) a.q_out[at + k] = out_item(v, k, o0, o1);
    }
    uint64_t big = __ballot(nch > 64u);
    while (big) {
        const int l = __builtin_ctzll(big);
        big &= big - 1;
        const int bv = __shfl(v, l, 64), b0 = __shfl(o0, l, 64), b1 = __shfl(o1, l, 64);
        const uint32_t bat = (uint32_t)__shfl((int)at, l, 64), bn = (uint32_t)__shfl((int)nch, l, 64);
        for (uint32_t k = (uint32_t)lane; k < bn; k += 64) a.q_out[bat + k] = out_item(bv, k, b0, b1);
    }
}

// One pass of the streaming step over the source array (see above).
template <bool Q>
__device__ __forceinline__ void ic_stream_pass(const StepArgs &a, const uint32_t *s_sum, bool &any)
{
    const uint64_t tail = tail_mask(0, a.B);
    const uint64_t gbase = a.goff;
    const int64_t nnz = a.nnz;
    // pass: chunk c of thread t covers arcs base + c*stride .. +3
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    constexpr int kChunks = 8;  // 32 arcs in flight per thread and pass
    for (int64_t base = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; base < nnz;
         base += stride * kChunks) {
        int us[4 * kChunks];
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int64_t eb = base + c * stride;
            int4 q = make_int4(0, 0, 0, 0);
            if (eb < nnz) q = *reinterpret_cast<const int4 *>(a.src + eb);  // sources padded by 16 B
            us[4 * c] = q.x;
            us[4 * c + 1] = q.y;
            us[4 * c + 2] = q.z;
            us[4 * c + 3] = q.w;
        }
        uint32_t cand = 0;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (base + c * stride + j < nnz && summary_hit(a, s_sum, us[4 * c + j]))
                    cand |= 1u << (4 * c + j);
        }
        // when any lane of the wave has a candidate, every slot loads its
        // bitmap word (word 0 where the slot is no candidate) in one
        // branch-free run, so the pass waits on these loads once
        uint32_t hit = 0;
        if (__ballot(cand != 0u) != 0ull) {
            uint32_t bw[4 * kChunks];
#pragma unroll
            for (int k = 0; k < 4 * kChunks; ++k)
                bw[k] = a.bm_prev[((cand >> k) & 1u) ? ((uint32_t)us[k] >> 5) : 0u];
#pragma unroll
            for (int k = 0; k < 4 * kChunks; ++k)
                hit |= (((cand >> k) & 1u) & (bw[k] >> ((uint32_t)us[k] & 31u))) << k;
        }
        while (hit) {
            const int k = __builtin_ctz(hit);
            hit &= hit - 1;
            const int64_t e = base + (k >> 2) * stride + (k & 3);
            const int u = us[k];
            const int v = a.dst[e];
            const uint32_t tv = a.edge_t ? 0u : ic_threshold(a, (uint32_t)(a.ptr[v + 1] - a.ptr[v]));
            const uint64_t cand_r = ~a.aux[v] & tail;
            uint64_t acc = 0;
            ic_edge(a, (int)e, a.prev[u] & cand_r, gbase, tv, acc);
            if (acc) {
                atomicOr((unsigned long long *)&a.next[v], (unsigned long long)acc);
                atomicOr((unsigned long long *)&a.aux[v], (unsigned long long)acc);
                join_frontier<Q>(a, v);
                any = true;
            }
        }
    }
}

__global__ void __launch_bounds__(1024) k_ic_stream(StepArgs a)
{
    if (a.flags[(a.step - 1) % (uint32_t)a.ring] == 0u) return;
    __shared__ uint32_t s_sum[kSumWords];
    for (int i = threadIdx.x; i < a.sum_words; i += blockDim.x) s_sum[i] = a.sum_prev[i];
    __syncthreads();
    bool any = false;
    ic_stream_pass<false>(a, s_sum, any);
    if (__ballot(any) != 0ull && (threadIdx.x & 63) == 0) a.flags[a.step % (uint32_t)a.ring] = 1u;
}

// Push over the out-arcs of the frontier of t-1: one wave per work item
// (a chunk of at most kOutChunk out-arcs of a frontier node u), lanes over
// the chunk's arcs.  An arc u -> v with edge id e runs the same trials the
// pull step would (keyed by e, threshold of v), for the replicates where u
// is newly active and v is not yet active.
__device__ __forceinline__ void ic_push_pass(const StepArgs &a, bool &any)
{
    const uint64_t tail = tail_mask(0, a.B);
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t nitems = a.qcnt[a.qi_in];
    const bool wc = a.ic_prob == kIcWeightedCascade && !a.edge_t;
    for (int64_t i = wave; i < nitems; i += nwave) {
        // an item carries its arc range, so the chain of dependent loads
        // is: item; arc and source word; target's active word, in-degree
        // and out-arc range; then the trials and the atomics
        const uint4 it = a.q_in[i];
        const int u = (int)it.x;
        const int j = (int)it.z + lane;
        const bool has = j < (int)it.w;
        const uint64_t fu = a.prev[u] & tail;
        const int2 ve = has ? a.oarc[j] : make_int2(0, 0);
        const int v = ve.x;
        uint64_t av = ~0ull;
        int p0 = 0, p1 = 0, o0 = 0, o1 = 0;
        if (has) {
            av = a.aux[v];
            if (wc) {
                p0 = a.ptr[v];
                p1 = a.ptr[v + 1];
            }
        }
        const uint64_t cand = fu & ~av;
        int claimed = -1;
        if (cand) {
            const uint32_t tv = a.edge_t ? 0u : (wc ? wc_threshold((uint32_t)(p1 - p0)) : a.ic_t);
            uint64_t acc = 0;
            ic_edge(a, ve.y, cand, a.goff, tv, acc);
            if (acc) {
                atomicOr((unsigned long long *)&a.next[v], (unsigned long long)acc);
                atomicOr((unsigned long long *)&a.aux[v], (unsigned long long)acc);
                if (claim_frontier(a, v)) {
                    claimed = v;
                    o0 = a.optr[v];
                    o1 = a.optr[v + 1];
                }
                any = true;
            }
        }
        queue_claimed(a, claimed, o0, o1);
    }
}

// The nodes of the queue a.qi_clr leave their frontier plane and bitmap, and
// the summary is cleared; thread `r` of `nthr`.
__device__ __forceinline__ void ic_clear_pass(const StepArgs &a, int64_t r, int64_t nthr)
{
    const int64_t nclr = a.qcnt[a.qi_clr];
    for (int64_t i = r; i < nclr; i += nthr) {
        const uint4 it = a.q_clr[i];
        if (it.y == 0u) {
            a.f_clr[it.x] = 0ull;
            a.bm_clr[it.x >> 5] = 0u;  // every set bit of this bitmap is such a node
        }
    }
    for (int64_t i = r; i < a.sum_words; i += nthr) a.sum_clr[i] = 0u;
}

// One step of the frontier-driven IC path (see StepArgs): first the nodes of
// the frontier of t-2 leave their plane, bitmap and summary (buffers step t
// does not touch) and the counters of the queue of t+1 are reset; then the
// frontier of t-1 is pushed over its out-arcs when it has at most
// push_limit of them, else the step streams every source.  The choice
// depends only on counts from step t-1, so every block makes the same one.
__global__ void __launch_bounds__(512) k_ic_front(StepArgs a)
{
    if (a.flags[(a.step - 1) % (uint32_t)a.ring] == 0u) return;
    __shared__ uint32_t s_sum[kSumWords];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    // when pushing, the clearing takes the threads after the push items'
    // waves (still in the first blocks dispatched), so no thread's chain of
    // loads holds both
    const bool push = a.qarcs[a.qi_in] <= a.push_limit;
    const int64_t skip = push ? (int64_t)a.qcnt[a.qi_in] * 64 : 0;
    const int64_t rtid = (tid - skip + nthr) % nthr;
    ic_clear_pass(a, rtid, nthr);
    if (tid == 0) {
        a.qcnt[a.qi_rst] = 0u;
        a.qarcs[a.qi_rst] = 0ull;
    }
    bool any = false;
    if (push) {
        ic_push_pass(a, any);
    } else {
        for (int i = threadIdx.x; i < a.sum_words; i += blockDim.x) s_sum[i] = a.sum_prev[i];
        __syncthreads();
        ic_stream_pass<true>(a, s_sum, any);
    }
    if (__ballot(any) != 0ull && (threadIdx.x & 63) == 0) a.flags[a.step % (uint32_t)a.ring] = 1u;
}

// A finalize queued before the host knew the run had ended: the first step
// of t0+1 .. t0+c whose absorption flag is clear (the run's last step), or
// -1 (the run goes on; nothing to do).  A load and a ballot per 64 steps;
// every lane of the wave gets the same answer.
__device__ __forceinline__ int64_t spec_last_step(const SpecFin &s)
{
    const int lane = (int)(threadIdx.x & 63u);
    for (int b = 0; b < s.c; b += 64) {
        const int i = b + lane;
        const bool clear =
            i < s.c && s.flags[(uint32_t)(s.t0 + 1 + i) % (uint32_t)s.ring] == 0u;
        const uint64_t m = __ballot(clear);
        if (m) return s.t0 + 1 + b + __builtin_ctzll(m);
    }
    return -1;
}

// Entry i of a 3- or 4-entry pointer array held in kernel arguments, with
// constant indices only (a run-time index would copy the arguments to
// per-lane scratch).
template <typename P>
__device__ __forceinline__ P pick3(const P (&a)[3], int i)
{
    return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}
template <typename P>
__device__ __forceinline__ P pick4(const P (&a)[4], int i)
{
    return i == 0 ? a[0] : (i == 1 ? a[1] : (i == 2 ? a[2] : a[3]));
}

// The planes of a speculative finalize: the frontier of the run's last step
// (empty, since that step activated nothing), or false when the run has not
// ended.
__device__ __forceinline__ bool spec_planes(FinArgs &f)
{
    if (f.spec.flags == nullptr) return true;
    const int64_t T = spec_last_step(f.spec);
    if (T < 0) return false;
    const int m = (int)(T % 3);
    f.one = pick3(f.spec.front3, m);
    f.bm = pick3(f.spec.bm3, m);
    return true;
}

// End of a frontier-driven run: the last two frontiers, which no later step
// clears, leave their buffers (one launch per frontier).
__global__ void __launch_bounds__(256) k_ic_scrub(StepArgs a)
{
    ic_clear_pass(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                  (int64_t)gridDim.x * blockDim.x);
}

// The same, queued before the host knew the run had ended (SpecFin): the
// frontier of step T - 2 + which, T the run's last step; after the second
// one the tag records that the run left its buffers clear.
__global__ void __launch_bounds__(256) k_ic_scrub_spec(StepArgs a, SpecFin sp, int which,
                                                      uint64_t *tag, uint64_t tag_value)
{
    const int64_t T = spec_last_step(sp);
    if (T < 0) return;
    const int64_t t = T + which;  // the step whose clear duty this is
    const int m = (int)((t - 2) % 3);
    a.qi_clr = (int32_t)((t + 2) % 4);
    a.q_clr = pick4(sp.queue4, a.qi_clr);
    a.f_clr = pick3(sp.front3, m);
    a.bm_clr = pick3(sp.bm3, m);
    a.sum_clr = pick3(sp.sum3, m);
    ic_clear_pass(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                  (int64_t)gridDim.x * blockDim.x);
    if (tag != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *tag = tag_value;
}

// Seeds of a frontier-driven run: joined to the frontier of step 0 (bitmap,
// summary, queue 0) once each, duplicates included.
__global__ void k_seed_queue(StepArgs a, const int32_t *seeds, int64_t ns)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns;
         i += (int64_t)gridDim.x * blockDim.x)
        join_frontier<true>(a, seeds[i]);
}

// Out-adjacency of a bound graph: out-degrees, then every arc placed in its
// source's range (any order inside a range: the steps that read it combine
// with OR).
__global__ void k_out_count(const int32_t *src, int64_t nnz, int32_t *cnt)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[src[e]], 1);
}

__global__ void k_out_fill(const int32_t *src, const int32_t *dst, int64_t nnz, int32_t *cursor,
                           int2 *oarc)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int at = atomicAdd(&cursor[src[e]], 1);
        oarc[at] = make_int2(dst[e], (int)e);
    }
}

// LT thresholds of one run, bit-sliced (one thread per node word): replicate
// g = goff + 64 w + b of node v gets need = max(1, ceil(U indeg / 2^32)) with
// U = D(LT threshold, v, g, 0), the same draw the per-step path takes; v
// activates iff its count of active in-neighbours reaches need.  Nodes
// whose in-degree needs more planes than the counter has are left to the
// per-step path (they are heavy rows, merged by the combine kernel).
__global__ void k_lt_need(StepArgs a)
{
    const int64_t total = (int64_t)a.n * a.W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int v = (int)(i / a.W);
        const int w = (int)(i - (int64_t)v * a.W);
        const uint32_t indeg = (uint32_t)(a.ptr[v + 1] - a.ptr[v]);
        const int P = indeg ? 32 - __builtin_clz(indeg) : 0;
        if (P == 0 || P > a.Lp) continue;
        uint64_t pl[16];
#pragma unroll
        for (int p = 0; p < 16; ++p) pl[p] = 0;
        const uint64_t g0 = a.goff + 64ull * (uint64_t)w;
        U4 o = {0u, 0u, 0u, 0u};
        for (int b = 0; b < 64; ++b) {
            const uint64_t g = g0 + (uint64_t)b;
            if (b == 0 || (g & 3u) == 0u)
                o = philox10((uint32_t)v, (uint32_t)(g >> 2), 0u, kDomLtThresh << 24, a.key0, a.key1);
            const uint32_t j = (uint32_t)g & 3u;
            const uint32_t u = j == 0 ? o.x : j == 1 ? o.y : j == 2 ? o.z : o.w;
            uint64_t need = ((uint64_t)u * (uint64_t)indeg + 0xFFFFFFFFull) >> 32;
            need = need ? need : 1ull;
#pragma unroll
            for (int p = 0; p < 16; ++p) pl[p] |= ((need >> p) & 1ull) << b;
        }
        uint64_t *np = a.need + (int64_t)v * a.Lp * a.W + w;
#pragma unroll
        for (int p = 0; p < 16; ++p)
            if (p < P) np[(int64_t)p * a.W] = pl[p];
    }
}

// Target row of every arc: one thread per row (grid-stride), used once when
// a graph is bound.
__global__ void k_expand_rows(const int32_t *ptr, int64_t n, int32_t *dst)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        for (int e = ptr[v]; e < ptr[v + 1]; ++e) dst[e] = (int32_t)v;
}

// Before a step of the edge-parallel kernel: the next-frontier bitmap still
// holds the frontier of two steps back, whose words in the next plane are the
// only nonzero ones there; zero those words (the step ORs into them), then
// clear the bitmap and its summary.
__global__ void k_ic_clear(StepArgs a)
{
    if (a.flags[(a.step - 1) % (uint32_t)a.ring] == 0u) return;
    const int64_t nw = ((int64_t)a.n + 31) >> 5;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t x = a.bm_next[i];
        if (x) {
            a.bm_next[i] = 0u;
            while (x) {
                const int b = __builtin_ctz(x);
                x &= x - 1u;
                a.next[i * 32 + b] = 0ull;
            }
        }
        if (i < a.sum_words) a.sum_next[i] = 0u;
    }
}

// ------------------------------------------------------------ batches ----
// One launch per synchronous step for every job of a batch: persistent
// blocks dequeue work items from one counter across all jobs (so jobs of very
// different sizes share the chip), find the job by binary search over the
// item prefix (LDS), skip jobs that are absorbed or past their step cap, and
// run the job's own pull-step block.  Ordering between steps comes from the
// kernel boundaries; the host captures a chunk of steps in a hipGraph.

__device__ __forceinline__ int find_job(const int32_t *off, int n_jobs, int item)
{
    int lo = 0, hi = n_jobs - 1;  // last job whose first item is <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ StepArgs job_at_step(const BatchCtl &c, int j, uint32_t t)
{
    StepArgs a = c.jobs[j];
    const uint64_t *p0 = a.prev;
    uint64_t *p1 = a.next;
    a.prev = (t & 1u) ? p0 : p1;   // state of step t-1
    a.next = (t & 1u) ? p1 : const_cast<uint64_t *>(p0);
    a.step = t;
    if (c.tail_on[j] == 0) {  // not in the tail mode this chunk
        a.ibm = nullptr;
        a.cand = nullptr;
    }
    return a;
}

__device__ __forceinline__ bool job_live(const BatchCtl &c, const StepArgs &a, int j, uint32_t t)
{
    return t <= (uint32_t)c.max_step[j] && a.flags[(t - 1) % (uint32_t)a.ring] != 0u;
}

__global__ void __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(kBatchWavesPerSimd)))
k_batch_step(BatchCtl c)
{
    __shared__ int32_t s_off[kMaxBatchJobs + 1];
    __shared__ int s_item;
    __shared__ uint32_t s_code[kCodeTable];
    const uint32_t t = *c.cur_step;
    for (int i = threadIdx.x; i <= c.n_jobs; i += blockDim.x) s_off[i] = c.item_off[i];
    __syncthreads();
    const int total = s_off[c.n_jobs];
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&c.queue[0], 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= total) break;
        const int j = __builtin_amdgcn_readfirstlane(find_job(s_off, c.n_jobs, item));
        const StepArgs a = job_at_step(c, j, t);
        if (!job_live(c, a, j, t)) continue;
        const int local = item - s_off[j];
        // tail mode: a tile with no candidate row leaves at once (every
        // thread of the block reads the same words)
        if (a.ibm != nullptr && tail_tile_idle(a, local, c.code[j] / 32 != kKindLT)) continue;
        if (c.code[j] / 32 == kKindEpidemic) {  // block-uniform
            if (threadIdx.x < kCodeTable) s_code[threadIdx.x] = code_threshold(a, threadIdx.x);
            __syncthreads();
        }
        bool any = false;
        switch (c.code[j]) {
        case kKindIC * 32 + 1: step_block<kKindIC, 1, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindEpidemic * 32 + 2: step_block<kKindEpidemic, 2, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindEpidemic * 32 + 4: step_block<kKindEpidemic, 4, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindEpidemic * 32 + 8: step_block<kKindEpidemic, 8, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindEpidemic * 32 + 12: step_block<kKindEpidemic, 12, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindEpidemic * 32 + 16: step_block<kKindEpidemic, 16, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindLT * 32 + 2: step_block<kKindLT, 2, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindLT * 32 + 4: step_block<kKindLT, 4, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindLT * 32 + 8: step_block<kKindLT, 8, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindLT * 32 + 12: step_block<kKindLT, 12, true>(a, local, nullptr, 0, s_code, any); break;
        case kKindLT * 32 + 16: step_block<kKindLT, 16, true>(a, local, nullptr, 0, s_code, any); break;
        default: break;
        }
        if (__ballot(any) != 0ull && (threadIdx.x & 63) == 0) a.flags[t % (uint32_t)a.ring] = 1u;
    }
}

__global__ void __launch_bounds__(kBatchBlock) k_batch_combine(BatchCtl c)
{
    __shared__ int32_t s_off[kMaxBatchJobs + 1];
    __shared__ int s_item;
    __shared__ uint32_t s_code[kCodeTable];
    const uint32_t t = *c.cur_step;
    for (int i = threadIdx.x; i <= c.n_jobs; i += blockDim.x) s_off[i] = c.comb_off[i];
    __syncthreads();
    const int total = s_off[c.n_jobs];
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&c.queue[1], 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= total) break;
        const int j = __builtin_amdgcn_readfirstlane(find_job(s_off, c.n_jobs, item));
        const StepArgs a = job_at_step(c, j, t);
        if (!job_live(c, a, j, t)) continue;
        const int local = item - s_off[j];
        if (c.code[j] / 32 == kKindEpidemic) {  // block-uniform
            if (threadIdx.x < kCodeTable) s_code[threadIdx.x] = code_threshold(a, threadIdx.x);
            __syncthreads();
        }
        bool any = false;
        switch (c.code[j]) {
        case kKindIC * 32 + 1: combine_block<kKindIC, 1>(a, local, s_code, any); break;
        case kKindEpidemic * 32 + 2: combine_block<kKindEpidemic, 2>(a, local, s_code, any); break;
        case kKindEpidemic * 32 + 4: combine_block<kKindEpidemic, 4>(a, local, s_code, any); break;
        case kKindEpidemic * 32 + 8: combine_block<kKindEpidemic, 8>(a, local, s_code, any); break;
        case kKindEpidemic * 32 + 12: combine_block<kKindEpidemic, 12>(a, local, s_code, any); break;
        case kKindEpidemic * 32 + 16: combine_block<kKindEpidemic, 16>(a, local, s_code, any); break;
        case kKindLT * 32 + 2: combine_block<kKindLT, 2>(a, local, s_code, any); break;
        case kKindLT * 32 + 4: combine_block<kKindLT, 4>(a, local, s_code, any); break;
        case kKindLT * 32 + 8: combine_block<kKindLT, 8>(a, local, s_code, any); break;
        case kKindLT * 32 + 12: combine_block<kKindLT, 12>(a, local, s_code, any); break;
        case kKindLT * 32 + 16: combine_block<kKindLT, 16>(a, local, s_code, any); break;
        default: break;
        }
        if (__ballot(any) != 0ull && (threadIdx.x & 63) == 0) a.flags[t % (uint32_t)a.ring] = 1u;
    }
}

// Tail mode of the batched launch, before batched step t: for every job in
// the mode, the bitmaps step t+1 sets are cleared and the nodes of bitmap
// t-1 and their out-neighbours are marked in candidate bitmap t % 2 (a wave
// per bitmap word, over the words of all jobs that can take the mode).  The
// job offsets and mode switches are staged in LDS; a wave keeps a job's
// arguments while its words follow one another, and jumps past the words of
// a job that is not in the mode or has stopped.
__global__ void __launch_bounds__(256) k_batch_expand(BatchCtl c)
{
    __shared__ int32_t s_off[kMaxBatchJobs + 1];
    __shared__ int32_t s_on[kMaxBatchJobs];
    const uint32_t t = *c.cur_step;
    for (int i = threadIdx.x; i <= c.n_jobs; i += blockDim.x) {
        s_off[i] = c.word_off[i];
        if (i < c.n_jobs) s_on[i] = c.tail_on[i];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t total = s_off[c.n_jobs];
    int jc = -1;  // the job `a` holds
    bool on = false;
    StepArgs a{};
    for (int64_t item = wave; item < total; item += nwave) {
        const int j = __builtin_amdgcn_readfirstlane(find_job(s_off, c.n_jobs, (int)item));
        if (j != jc) {
            jc = j;
            on = s_on[j] != 0;
            if (on) {
                a = job_at_step(c, j, t);
                on = job_live(c, a, j, t);
            }
        }
        if (!on) {
            // the loop step then lands on this wave's first word of a later job
            item += ((int64_t)s_off[j + 1] - 1 - item) / nwave * nwave;
            continue;
        }
        const int i = (int)item - s_off[j];
        if (lane == 0) {
            a.ibm[(size_t)((t + 1u) & 3u) * a.ibm_words + i] = 0u;
            a.cand[(size_t)((t + 1u) & 1u) * a.ibm_words + i] = 0u;
        }
        uint32_t m = a.ibm[(size_t)((t - 1u) & 3u) * a.ibm_words + i];
        if (m == 0u) continue;
        uint32_t *cand = a.cand + (size_t)(t & 1u) * a.ibm_words;
        if (lane == 0) atomicOr(&cand[i], m);
        while (m) {
            const int u = 32 * i + __builtin_ctz(m);
            m &= m - 1u;
            const int o1 = a.optr[u + 1];
            for (int e = a.optr[u] + lane; e < o1; e += 64) {
                const int v = a.oarc[e].x;
                atomicOr(&cand[v >> 5], 1u << (v & 31));
            }
        }
    }
}

// Per job that can take the tail mode, the nodes with an infected replicate
// or a new activation after step t into counts[j] (zeroed by the caller): a
// nonzero word of the state plane after step t (SI family: the infected
// plane; IC: the frontier plane), or activation stamp t (LT).  A job in the tail mode has these nodes in its bitmap t % 4
// already (a node that is no candidate keeps no infected replicate and gains
// no activation), so one bit is read instead of its row; a job that did not
// run step t counts nothing (the host no longer reads its count).
__global__ void k_batch_count(BatchCtl c, uint32_t t, unsigned long long *counts)
{
    const int total = c.row_off[c.n_jobs];
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // a wave takes 64 consecutive rows at a time, job by job within them;
    // state planes of several words a row are read with lanes over words
    // (64 / W whole rows a pass), so the loads of a pass are contiguous
    for (int64_t r0 = wave * 64; r0 < total; r0 += nwave * 64) {
        const int64_t rend = r0 + 64 < total ? r0 + 64 : total;
        for (int64_t r = r0; r < rend;) {
            const int j = __builtin_amdgcn_readfirstlane(find_job(c.row_off, c.n_jobs, (int)r));
            const int64_t je = c.row_off[j + 1] < rend ? (int64_t)c.row_off[j + 1] : rend;
            const StepArgs &a = c.jobs[j];
            const int64_t v0 = r - c.row_off[j];  // first row of the job in [r, je)
            const int64_t nr = je - r;
            unsigned long long cnt = 0;
            if (job_live(c, a, j, t)) {
                if (c.tail_on[j] != 0 && a.ibm != nullptr) {
                    const int64_t v = v0 + lane;
                    const bool hit = lane < nr &&
                                     ((a.ibm[(size_t)(t & 3u) * a.ibm_words + (v >> 5)] >> (v & 31)) & 1u);
                    cnt = (unsigned long long)__popcll(__ballot(hit));
                } else if (c.code[j] / 32 == kKindLT) {
                    const int64_t v = v0 + lane;
                    const bool hit = lane < nr && a.stamp[(size_t)(t & 1u) * (size_t)a.n + (size_t)v] == t;
                    cnt = (unsigned long long)__popcll(__ballot(hit));
                } else {
                    const uint64_t *pl = (t & 1u) ? a.next : a.prev;  // state after step t
                    const int W = a.W;
                    if (W <= 64) {
                        const int R = 64 / W;  // rows a pass
                        const int slot = lane / W, w = lane - slot * W;
                        const uint64_t gmask = W == 64 ? ~0ull : ((1ull << W) - 1ull);
                        for (int64_t q = 0; q < nr; q += R) {
                            const bool in = slot < R && q + slot < nr;
                            const uint64_t x = in ? pl[(v0 + q + slot) * W + w] : 0ull;
                            const uint64_t m = __ballot(x != 0ull);
                            for (int k = 0; k < R; ++k) cnt += ((m >> (k * W)) & gmask) != 0ull ? 1ull : 0ull;
                        }
                    } else {
                        for (int64_t q = 0; q < nr; ++q) {
                            uint64_t x = 0;
                            for (int w = lane; w < W; w += 64) x |= pl[(v0 + q) * W + w];
                            cnt += __ballot(x != 0ull) != 0ull ? 1ull : 0ull;
                        }
                    }
                }
            }
            if (lane == 0 && cnt) atomicAdd(&counts[j], cnt);  // cnt is wave-uniform
            r = je;
        }
    }
}

// End of step t: clear every job's flag slot for step t+1, reset the
// dequeue counters and advance the step.
__global__ void k_batch_advance(BatchCtl c)
{
    const uint32_t t = *c.cur_step;
    for (int j = threadIdx.x; j < c.n_jobs; j += blockDim.x)
        c.jobs[j].flags[(t + 1) % (uint32_t)c.ring] = 0u;
    for (int j = 0; j < c.n_jobs; ++j) {
        uint32_t *wf = c.jobs[j].wflags;
        if (wf == nullptr) continue;
        const int W = c.jobs[j].W;
        wf += (size_t)((t + 1) % (uint32_t)c.jobs[j].wring) * (size_t)W;
        for (int i = threadIdx.x; i < W; i += blockDim.x) wf[i] = 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        c.queue[0] = 0u;
        c.queue[1] = 0u;
        *c.cur_step = t + 1;
    }
}

// ------------------------------------------------------- init / output ----

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Zeroes count16 16-byte words with non-temporal stores (the zeroed planes
// are next touched a step or more later, sparsely).
__global__ void k_zero16(u32x4 *p, int64_t count16)
{
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count16;
         i += (int64_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(z, p + i);
}

// Bitmaps of the tail mode for step t: bit v of bitmap (t-1) % 4 set iff
// `cur` (the state after t-1) has a nonzero word in row v, of bitmap
// (t-2) % 4 iff `old` (the state after t-2) does; bitmap t % 4 cleared.  One
// thread per bitmap word (32 rows).
__global__ void k_mark_rows(const uint64_t *cur, const uint64_t *old, uint32_t *ibm, uint32_t *cand,
                            int32_t ibm_words, int64_t n, int64_t W, uint32_t t)
{
    uint32_t *b1 = ibm + (size_t)((t - 1u) & 3u) * ibm_words;
    uint32_t *b2 = ibm + (size_t)((t - 2u) & 3u) * ibm_words;
    uint32_t *b0 = ibm + (size_t)(t & 3u) * ibm_words;
    uint32_t *c0 = cand + (size_t)(t & 1u) * ibm_words;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ibm_words;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t m1 = 0, m2 = 0;
        for (int j = 0; j < 32; ++j) {
            const int64_t v = 32 * i + j;
            if (v >= n) break;
            uint64_t c = 0, o = 0;
            for (int64_t w = 0; w < W; ++w) {
                c |= cur[v * W + w];
                o |= old[v * W + w];
            }
            m1 |= (c ? 1u : 0u) << j;
            m2 |= (o ? 1u : 0u) << j;
        }
        b1[i] = m1;
        b2[i] = m2;
        b0[i] = 0u;
        c0[i] = 0u;
    }
}

// Candidates of tail-mode step t: every node with an infected replicate
// after t-1 (bitmap t-1) and its out-neighbours are marked in candidate
// bitmap t % 2.  Wave k takes bitmap words k, k + waves, ...; each set bit is
// a node whose out-arcs the wave's lanes mark.
__global__ void __launch_bounds__(256) k_tail_expand(StepArgs a)
{
    if (a.flags[(a.step - 1) % (uint32_t)a.ring] == 0u) return;  // as the step: nothing left
    const uint32_t *inf1 = a.ibm + (size_t)((a.step - 1u) & 3u) * a.ibm_words;
    uint32_t *cand = a.cand + (size_t)(a.step & 1u) * a.ibm_words;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = wave; i < a.ibm_words; i += nwave) {
        uint32_t m = inf1[i];
        if (m == 0u) continue;
        if (lane == 0) atomicOr(&cand[i], m);
        while (m) {
            const int u = (int)(32 * i) + __builtin_ctz(m);
            m &= m - 1u;
            const int o1 = a.optr[u + 1];
            for (int e = a.optr[u] + lane; e < o1; e += 64) {
                const int v = a.oarc[e].x;
                atomicOr(&cand[v >> 5], 1u << (v & 31));
            }
        }
    }
}

// The same for LT from its activation stamps: bitmap (t-1) % 4 marks the
// nodes with a new activation at t-1, bitmap (t-2) % 4 those at t-2.
__global__ void k_mark_gained(const uint32_t *stamp, uint32_t *ibm, uint32_t *cand,
                              int32_t ibm_words, int64_t n, uint32_t t)
{
    const uint32_t *s1 = stamp + (size_t)((t - 1u) & 1u) * (size_t)n;
    const uint32_t *s2 = stamp + (size_t)(t & 1u) * (size_t)n;
    uint32_t *b1 = ibm + (size_t)((t - 1u) & 3u) * ibm_words;
    uint32_t *b2 = ibm + (size_t)((t - 2u) & 3u) * ibm_words;
    uint32_t *b0 = ibm + (size_t)(t & 3u) * ibm_words;
    uint32_t *c0 = cand + (size_t)(t & 1u) * ibm_words;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ibm_words;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t m1 = 0, m2 = 0;
        for (int j = 0; j < 32; ++j) {
            const int64_t v = 32 * i + j;
            if (v >= n) break;
            m1 |= (s1[v] == t - 1u ? 1u : 0u) << j;
            m2 |= (s2[v] == t - 2u ? 1u : 0u) << j;
        }
        b1[i] = m1;
        b2[i] = m2;
        b0[i] = 0u;
        c0[i] = 0u;
    }
}

// Number of LT nodes with a new activation at step t (stamp t in array t & 1).
__global__ void k_count_stamped(const uint32_t *stamp, int64_t n, uint32_t t, unsigned long long *count)
{
    const uint32_t *s = stamp + (size_t)(t & 1u) * (size_t)n;
    unsigned long long c = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x)
        c += s[v] == t ? 1ull : 0ull;
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

// Nodes with a nonzero word in `plane` ([n][W]) into *count (zeroed by the
// caller).  Lanes go over words so that a wave's loads are contiguous: with
// W <= 64 a pass of the wave takes 64 / W whole rows (R W consecutive words)
// and counts the rows whose W-bit group of the ballot is nonzero; wider rows
// take a wave each, its lanes striding over the row.
__global__ void k_count_rows(const uint64_t *plane, int64_t n, int64_t W, unsigned long long *count)
{
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long c = 0;
    if (W <= 64) {
        const int Wi = (int)W;
        const int R = 64 / Wi;  // rows per pass
        const int slot = lane / Wi, w = lane - slot * Wi;
        const uint64_t gmask = Wi == 64 ? ~0ull : ((1ull << Wi) - 1ull);
        for (int64_t r0 = wave * R; r0 < n; r0 += nwave * R) {
            const int64_t v = r0 + slot;
            const uint64_t x = (slot < R && v < n) ? plane[v * W + w] : 0ull;
            const uint64_t m = __ballot(x != 0ull);
            if (Wi == 1) {
                c += (unsigned long long)__popcll(m);
            } else {
                for (int k = 0; k < R; ++k) c += ((m >> (k * Wi)) & gmask) != 0ull ? 1ull : 0ull;
            }
        }
    } else {
        for (int64_t v = wave; v < n; v += nwave) {
            uint64_t x = 0;
            for (int64_t w = lane; w < W; w += 64) x |= plane[v * W + w];
            c += __ballot(x != 0ull) != 0ull ? 1ull : 0ull;
        }
    }
    if (lane == 0 && c) atomicAdd(count, c);  // c is the same in every lane of the wave
}

__global__ void k_zero16_unless(u32x4 *p, int64_t count16, const uint64_t *tag, uint64_t expect)
{
    if (*tag == expect) return;
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count16;
         i += (int64_t)gridDim.x * blockDim.x)
        __builtin_nontemporal_store(z, p + i);
}

__global__ void k_fill64(uint64_t *p, int64_t count, uint64_t value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_stamp_seeds(uint32_t *stamp, const int32_t *seeds, int64_t ns)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ns;
         i += (int64_t)gridDim.x * blockDim.x)
        stamp[seeds[i]] = 0u;
}

__global__ void k_fill32(uint32_t *p, int64_t count, uint32_t value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// Clears every absorption flag of the ring except slot `keep` (the step
// before the next chunk).
// With word flags, the slots of steps t and t-1 are kept (the next step
// reads both).
__global__ void k_ring_clear(uint32_t *flags, int32_t ring, int32_t keep, uint32_t *wflags,
                             int32_t W, int32_t wring, int64_t t)
{
    for (int i = threadIdx.x; i < ring; i += blockDim.x)
        if (i != keep) flags[i] = 0u;
    if (wflags == nullptr) return;
    const int64_t k1 = t % wring, k2 = (t + wring - 1) % wring;
    for (int64_t i = threadIdx.x; i < (int64_t)wring * W; i += blockDim.x) {
        const int64_t sl = i / W;
        if (sl != k1 && sl != k2) wflags[i] = 0u;
    }
}

// Seeds are in state 1 in every replicate (Algorithm 1, initial states).
__global__ void k_seed(uint64_t *p1, uint64_t *p2, const int32_t *seeds, int64_t ns, int32_t W,
                       int64_t B, uint32_t *flag0, uint32_t *bm, uint32_t *sum, int sum_shift)
{
    const int64_t total = ns * W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = i / W;
        const int w = (int)(i - k * W);
        const int64_t idx = (int64_t)seeds[k] * W + w;
        const uint64_t m = tail_mask(w, B);
        p1[idx] = m;
        if (p2) p2[idx] = m;
        if (bm && w == 0) {
            const int u = seeds[k];
            atomicOr(&bm[u >> 5], 1u << (u & 31));
            atomicOr(&sum[(u >> sum_shift) >> 5], 1u << ((u >> sum_shift) & 31));
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && ns > 0) flag0[0] = 1u;
}

// Packed planes -> uint8 states [n][B] and per-node counts.
__global__ void __launch_bounds__(256) k_finalize(FinArgs f)
{
    if (!spec_planes(f)) return;
    const int lane = threadIdx.x & 63;
    const int G = f.G;
    const int rpw = 64 >> f.lgG;
    const int gw = lane & (G - 1);
    const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave_total = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t rb = gwave * rpw; rb < f.n; rb += nwave_total * rpw) {
        const int64_t v = rb + (lane >> f.lgG);
        const bool act = v < f.n;
        uint32_t cnt = 0;
        for (int w0 = 0; w0 < f.W; w0 += G) {
            const int w = w0 + gw;
            if (!act || w >= f.W) continue;
            const int64_t idx = v * f.W + w;
            const uint64_t tail = tail_mask(w, f.B);
            const bool live = !f.bm || ((f.bm[v >> 5] >> (v & 31)) & 1u);
            const bool live2 = f.two && (!f.two_bm || ((f.two_bm[v >> 5] >> (v & 31)) & 1u));
            const uint64_t one = live ? (f.one[idx] & tail) : 0ull;
            const uint64_t two = live2 ? (f.two[idx] & tail) : 0ull;
            const uint64_t three = f.three ? (f.three[idx] & tail) : 0ull;
            if (f.scrub && live2) f.two[idx] = 0ull;
            cnt += (uint32_t)__popcll(f.model == kSIS ? one : (one | two | three));
            if (!f.states) continue;
            // state codes: with a latent plane E 1, I 2, R 3 (the planes are
            // disjoint); else 1 for the first plane, 2 for the second only
            const uint32_t m1 = f.three ? 2u : 1u, m2 = f.three ? 3u : 2u;
            uint8_t *dst = f.states + v * f.B + 64ll * w;
            const int64_t nb = f.B - 64ll * w < 64 ? f.B - 64ll * w : 64;
            if (nb == 64 && (f.B & 15) == 0 && ((uintptr_t)f.states & 15u) == 0) {
                uint4 *d4 = reinterpret_cast<uint4 *>(dst);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t wd[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        uint32_t x = 0;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int bit = q * 16 + k * 4 + j;
                            const uint32_t s1 = (uint32_t)(one >> bit) & 1u;
                            const uint32_t s2 = (uint32_t)(two >> bit) & 1u & ~s1;
                            const uint32_t s3 = (uint32_t)(three >> bit) & 1u;
                            x |= (s1 * m1 + s2 * m2 + s3) << (8 * j);
                        }
                        wd[k] = x;
                    }
                    d4[q] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
                }
            } else {
                for (int j = 0; j < nb; ++j) {
                    const uint32_t s1 = (uint32_t)(one >> j) & 1u;
                    const uint32_t s2 = (uint32_t)(two >> j) & 1u & ~s1;
                    const uint32_t s3 = (uint32_t)(three >> j) & 1u;
                    dst[j] = (uint8_t)(s1 * m1 + s2 * m2 + s3);
                }
            }
        }
        for (int off = 1; off < G; off <<= 1) cnt += __shfl_xor(cnt, off, 64);
        if (act && gw == 0 && f.counts) f.counts[v] = cnt;
        // scrubbing runs have one word per node (G = 1), so the wave's 64
        // nodes cover whole bitmap words, all read above
        if (f.scrub && act && (v & 31) == 0) f.two_bm[v >> 5] = 0u;
    }
}

// The same when B = 64 W and W is a power of two up to 64 (so G = W and a
// wave holds one word per lane): the uint8 states of a wave's 64 words form
// one contiguous 4 KB block, and each store instruction writes 1 KB of it
// (pass q, lane l: bytes 16 (64 q + l) .. +15 of the block, whose word is
// held by lane 16 q + l / 4 and reaches lane l by shuffle), instead of 16
// bytes at a 64-byte stride per lane.  Needs a 16-byte aligned state array.
__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), src, 64);
    return ((uint64_t)hi << 32) | lo;
}

// Loads the packed words of lane's node word for the dense finalize.
struct DenseWords {
    uint64_t one, two, three;
    bool act;
};

__device__ __forceinline__ DenseWords dense_words(const FinArgs &f, int64_t rb, int lane)
{
    DenseWords d = {0ull, 0ull, 0ull, false};
    const int64_t v = rb + (lane >> f.lgG);
    d.act = v < f.n;
    if (d.act) {
        const int64_t idx = v * f.W + (lane & (f.G - 1));
        const bool live = !f.bm || ((f.bm[v >> 5] >> (v & 31)) & 1u);
        const bool live2 = f.two && (!f.two_bm || ((f.two_bm[v >> 5] >> (v & 31)) & 1u));
        d.one = live ? f.one[idx] : 0ull;
        d.two = live2 ? f.two[idx] : 0ull;
        d.three = f.three ? f.three[idx] : 0ull;
        if (f.scrub && live2) f.two[idx] = 0ull;
    }
    return d;
}

// Counts and states of one wave's 64 words (rows rb .. rb + 64 / G - 1).
__device__ __forceinline__ void dense_out(const FinArgs &f, int64_t rb, int lane,
                                          const DenseWords &d)
{
    const int G = f.G;
    uint32_t cnt = (uint32_t)__popcll(f.model == kSIS ? d.one : (d.one | d.two | d.three));
    for (int off = 1; off < G; off <<= 1) cnt += __shfl_xor(cnt, off, 64);
    if (d.act && (lane & (G - 1)) == 0 && f.counts) f.counts[rb + (lane >> f.lgG)] = cnt;
    if (!f.states) return;
    // state byte = s1 m1 + s2 m2 + s3 (at most 3, so bytes never carry)
    const uint32_t m1 = f.three ? 2u : 1u, m2 = f.three ? 3u : 2u;
    uint8_t *blk = f.states + rb * f.B;
    const int64_t limit = (f.n - rb) * f.B;  // bytes of the block inside the array
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int src = 16 * q + (lane >> 2);
        const uint64_t o1 = shfl64(d.one, src), o2 = shfl64(d.two, src), o3 = shfl64(d.three, src);
        const int sh = 16 * (lane & 3);
        const uint32_t h1 = (uint32_t)(o1 >> sh) & 0xFFFFu, h2 = (uint32_t)(o2 >> sh) & 0xFFFFu & ~h1,
                       h3 = (uint32_t)(o3 >> sh) & 0xFFFFu;
        uint32_t wd[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t n1 = (h1 >> (4 * k)) & 0xFu, n2 = (h2 >> (4 * k)) & 0xFu,
                           n3 = (h3 >> (4 * k)) & 0xFu;
            wd[k] = spread4(n1, 0x204081u, 0x01010101u) * m1 +
                    spread4(n2, 0x204081u, 0x01010101u) * m2 + spread4(n3, 0x204081u, 0x01010101u);
        }
        const int64_t byte = 16 * (64 * q + lane);
        if (byte < limit) {
            const u32x4 o = {wd[0], wd[1], wd[2], wd[3]};
            __builtin_nontemporal_store(o, reinterpret_cast<u32x4 *>(blk + byte));
        }
    }
}

// Two blocks of 64 words per pass, their loads issued before either's stores.
__global__ void __launch_bounds__(256) k_finalize_dense(FinArgs f)
{
    if (!spec_planes(f)) return;
    const int lane = threadIdx.x & 63;
    const int rpw = 64 >> f.lgG;
    const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave_total = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int64_t stride = nwave_total * rpw;
    for (int64_t rb = gwave * rpw; rb < f.n; rb += 2 * stride) {
        const DenseWords d0 = dense_words(f, rb, lane);
        const bool two_blocks = rb + stride < f.n;
        const DenseWords d1 = two_blocks ? dense_words(f, rb + stride, lane)
                                         : DenseWords{0ull, 0ull, 0ull, false};
        if (f.scrub) {  // one word per node: a wave's 64 nodes are two whole bitmap words
            const int64_t v = rb + lane;
            if (d0.act && (v & 31) == 0) f.two_bm[v >> 5] = 0u;
            if (d1.act && ((v + stride) & 31) == 0) f.two_bm[(v + stride) >> 5] = 0u;
        }
        dense_out(f, rb, lane, d0);
        if (two_blocks) dense_out(f, rb + stride, lane, d1);
    }
}

// State tally after a step (per-step trajectories): popcounts of the state
// planes summed over nodes and replicates; integer atomics, so the totals are
// exact and independent of the order.
__global__ void __launch_bounds__(256) k_tally(FinArgs f)
{
    if (f.flags && f.step > 1u && f.flags[(f.step - 1u) % (uint32_t)f.ring] == 0u) {
        if (blockIdx.x == 0 && threadIdx.x < 3) f.tally[threadIdx.x] = f.tally[(int)threadIdx.x - 3];
        return;
    }
    unsigned long long c1 = 0, c2 = 0, c3 = 0;
    const int64_t words = (int64_t)f.n * f.W;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = i / f.W;
        const int w = (int)(i - v * f.W);
        const uint64_t tail = tail_mask(w, f.B);
        const bool live = !f.bm || ((f.bm[v >> 5] >> (v & 31)) & 1u);
        const uint64_t one = live ? (f.one[i] & tail) : 0ull;
        const uint64_t two = f.two ? (f.two[i] & tail & ~one) : 0ull;
        const uint64_t three = f.three ? (f.three[i] & tail) : 0ull;
        if (f.three) {  // E 1, I 2, R 3
            c1 += (unsigned long long)__popcll(three);
            c2 += (unsigned long long)__popcll(one);
            c3 += (unsigned long long)__popcll(two);
        } else {
            c1 += (unsigned long long)__popcll(one);
            c2 += (unsigned long long)__popcll(two);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        c1 += __shfl_xor(c1, off, 64);
        c2 += __shfl_xor(c2, off, 64);
        c3 += __shfl_xor(c3, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (c1) atomicAdd(&f.tally[0], c1);
        if (c2) atomicAdd(&f.tally[1], c2);
        if (c3) atomicAdd(&f.tally[2], c3);
    }
}

__global__ void k_tally_clear(unsigned long long *t)
{
    if (threadIdx.x < 3) t[threadIdx.x] = 0ull;
}

__global__ void k_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out,
                         int64_t count)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const U4 o = philox10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
        out[4 * i] = o.x;
        out[4 * i + 1] = o.y;
        out[4 * i + 2] = o.z;
        out[4 * i + 3] = o.w;
    }
}

// ------------------------------------------------------------ launchers ----

static unsigned grid_for(int64_t work, int block)
{
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    // 16-byte words first (p is 256-byte aligned), the last 8 bytes if any
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 > 0) {
        hipLaunchKernelGGL(k_zero16, dim3(grid_for(n16, 256)), dim3(256), 0, s, (u32x4 *)p, n16);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (bytes % 16 >= 8) return launch_fill64((uint64_t *)((char *)p + 16 * n16), 1, 0ull, s);
    return hipSuccess;
}

hipError_t launch_zero_unless(void *p, size_t bytes, const uint64_t *tag, uint64_t expect,
                              hipStream_t s)
{
    // whole 16-byte words only: callers pass regions of 256-byte multiples
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 <= 0) return hipSuccess;
    // a grid of at most 1024 blocks: when the tag is there every block only
    // reads it, and a larger grid costs more to dispatch than that
    const unsigned g = std::min<unsigned>(grid_for(n16, 256), 1024u);
    hipLaunchKernelGGL(k_zero16_unless, dim3(g), dim3(256), 0, s, (u32x4 *)p, n16, tag, expect);
    return hipGetLastError();
}

hipError_t launch_mark_rows(const uint64_t *cur, const uint64_t *old, uint32_t *ibm, uint32_t *cand,
                            int32_t ibm_words, int64_t n, int64_t W, uint32_t t, hipStream_t s)
{
    if (ibm_words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark_rows, dim3(grid_for(ibm_words, 64)), dim3(64), 0, s, cur, old, ibm,
                       cand, ibm_words, n, W, t);
    return hipGetLastError();
}

hipError_t launch_mark_gained(const uint32_t *stamp, uint32_t *ibm, uint32_t *cand, int32_t ibm_words,
                              int64_t n, uint32_t t, hipStream_t s)
{
    if (ibm_words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mark_gained, dim3(grid_for(ibm_words, 64)), dim3(64), 0, s, stamp, ibm, cand,
                       ibm_words, n, t);
    return hipGetLastError();
}

hipError_t launch_count_stamped(const uint32_t *stamp, int64_t n, uint32_t t,
                                unsigned long long *count, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill64, dim3(1), dim3(64), 0, s, (uint64_t *)count, (int64_t)1, 0ull);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n <= 0) return e;
    hipLaunchKernelGGL(k_count_stamped, dim3(std::min<unsigned>(grid_for(n, 256), 2048u)), dim3(256),
                       0, s, stamp, n, t, count);
    return hipGetLastError();
}

hipError_t launch_tail_expand(const StepArgs &a, hipStream_t s)
{
    // a wave per bitmap word, at most 1024 blocks of four waves
    const unsigned g = std::min<unsigned>(grid_for((int64_t)a.ibm_words * 64, 256), 1024u);
    hipLaunchKernelGGL(k_tail_expand, dim3(g), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_count_rows(const uint64_t *plane, int64_t n, int64_t W, unsigned long long *count,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_fill64, dim3(1), dim3(64), 0, s, (uint64_t *)count, (int64_t)1, 0ull);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n <= 0) return e;
    hipLaunchKernelGGL(k_count_rows, dim3(std::min<unsigned>(grid_for(n, 256), 2048u)), dim3(256), 0,
                       s, plane, n, W, count);
    return hipGetLastError();
}

hipError_t launch_ic_scrub(const StepArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_ic_scrub, dim3(256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ic_scrub_spec(const StepArgs &a, const SpecFin &sp, int which, uint64_t *tag,
                                uint64_t tag_value, hipStream_t s)
{
    hipLaunchKernelGGL(k_ic_scrub_spec, dim3(256), dim3(256), 0, s, a, sp, which, tag, tag_value);
    return hipGetLastError();
}

hipError_t launch_fill64(uint64_t *p, int64_t count, uint64_t value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill64, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_stamp_seeds(uint32_t *stamp, const int32_t *seeds, int64_t ns, hipStream_t s)
{
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stamp_seeds, dim3(grid_for(ns, 256)), dim3(256), 0, s, stamp, seeds, ns);
    return hipGetLastError();
}

hipError_t launch_fill32(uint32_t *p, int64_t count, uint32_t value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill32, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_lt_need(const StepArgs &a, hipStream_t s)
{
    const int64_t total = (int64_t)a.n * a.W;
    hipLaunchKernelGGL(k_lt_need, dim3(grid_for(total, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ring_clear(uint32_t *flags, int32_t ring, int32_t keep, hipStream_t s,
                             uint32_t *wflags, int32_t W, int32_t wring, int64_t t)
{
    hipLaunchKernelGGL(k_ring_clear, dim3(1), dim3(256), 0, s, flags, ring, keep, wflags, W,
                       wring, t);
    return hipGetLastError();
}

hipError_t launch_ic_front(const StepArgs &a, int grid, int block, hipStream_t s)
{
    // enough blocks for the larger of the two passes (4 arcs a thread when
    // streaming; a wave per work item when pushing), at most `grid`
    const int64_t work = std::max<int64_t>((a.nnz + 3) / 4, (int64_t)a.n * 64);
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>((work + block - 1) / block, grid));
    hipLaunchKernelGGL(k_ic_front, dim3((unsigned)g), dim3((unsigned)block), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_seed_queue(const StepArgs &a, const int32_t *seeds, int64_t ns, hipStream_t s)
{
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seed_queue, dim3(grid_for(ns, 256)), dim3(256), 0, s, a, seeds, ns);
    return hipGetLastError();
}

hipError_t launch_out_count(const int32_t *src, int64_t nnz, int32_t *cnt, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_out_count, dim3(grid_for(nnz, 256)), dim3(256), 0, s, src, nnz, cnt);
    return hipGetLastError();
}

hipError_t launch_out_fill(const int32_t *src, const int32_t *dst, int64_t nnz, int32_t *cursor,
                           int2 *oarc, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_out_fill, dim3(grid_for(nnz, 256)), dim3(256), 0, s, src, dst, nnz,
                       cursor, oarc);
    return hipGetLastError();
}

hipError_t launch_seed(uint64_t *p1, uint64_t *p2, const int32_t *seeds, int64_t ns, int32_t W,
                       int64_t B, uint32_t *flag0, uint32_t *bm, uint32_t *sum, int sum_shift,
                       hipStream_t s)
{
    if (ns <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seed, dim3(grid_for(ns * W, 256)), dim3(256), 0, s, p1, p2, seeds, ns, W,
                       B, flag0, bm, sum, sum_shift);
    return hipGetLastError();
}

int counter_planes_for(int64_t max_count)
{
    int bits = 1;
    while (bits < 32 && (max_count >> bits) != 0) ++bits;
    if (bits <= 2) return 2;
    if (bits <= 4) return 4;
    if (bits <= 8) return 8;
    if (bits <= 12) return 12;
    return 16;
}

template <int KIND, bool TAIL>
static hipError_t step_kind(const StepArgs &a, int L, dim3 grid, dim3 block, hipStream_t s)
{
    switch (L) {
    case 2: hipLaunchKernelGGL((k_step<KIND, 2, TAIL>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_step<KIND, 4, TAIL>), grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_step<KIND, 8, TAIL>), grid, block, 0, s, a); break;
    case 12: hipLaunchKernelGGL((k_step<KIND, 12, TAIL>), grid, block, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_step<KIND, 16, TAIL>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, int kind, int L, int block, hipStream_t s)
{
    const int64_t nblocks = step_blocks(a, block);
    if (nblocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)nblocks), blk((unsigned)block);
    // the tail-mode row test in its own instantiation: the other kernels
    // keep their register allocation
    if (kind == kKindIC) {
        if (a.ibm != nullptr)
            hipLaunchKernelGGL((k_step<kKindIC, 1, true>), grid, blk, 0, s, a);
        else
            hipLaunchKernelGGL((k_step<kKindIC, 1>), grid, blk, 0, s, a);
        return hipGetLastError();
    }
    if (kind == kKindEpidemic && a.ibm != nullptr)
        return step_kind<kKindEpidemic, true>(a, L, grid, blk, s);
    if (kind == kKindEpidemic) return step_kind<kKindEpidemic, false>(a, L, grid, blk, s);
    if (a.ibm != nullptr) return step_kind<kKindLT, true>(a, L, grid, blk, s);
    return step_kind<kKindLT, false>(a, L, grid, blk, s);
}

hipError_t launch_combine(const StepArgs &a, int kind, int /*block*/, hipStream_t s)
{
    if (a.n_heavy <= 0) return hipSuccess;
    const int rows_per_block = 4 * combine_rows_per_wave(a.lgG);
    const dim3 grid((unsigned)((a.n_heavy + rows_per_block - 1) / rows_per_block)), blk(256);
    if (kind == kKindIC) {
        hipLaunchKernelGGL((k_combine<kKindIC, 1>), grid, blk, 0, s, a);
        return hipGetLastError();
    }
#define FSG_COMBINE(K)                                                              \
    switch (a.Lp) {                                                                 \
    case 2: hipLaunchKernelGGL((k_combine<K, 2>), grid, blk, 0, s, a); break;       \
    case 4: hipLaunchKernelGGL((k_combine<K, 4>), grid, blk, 0, s, a); break;       \
    case 8: hipLaunchKernelGGL((k_combine<K, 8>), grid, blk, 0, s, a); break;       \
    case 12: hipLaunchKernelGGL((k_combine<K, 12>), grid, blk, 0, s, a); break;     \
    case 16: hipLaunchKernelGGL((k_combine<K, 16>), grid, blk, 0, s, a); break;     \
    default: return hipErrorInvalidValue;                                           \
    }
    if (kind == kKindEpidemic) {
        FSG_COMBINE(kKindEpidemic)
    } else {
        FSG_COMBINE(kKindLT)
    }
#undef FSG_COMBINE
    return hipGetLastError();
}

hipError_t launch_ic_stream(const StepArgs &a, int grid, int block, hipStream_t s)
{
    if (a.nnz <= 0) return hipSuccess;
    const int64_t need = (a.nnz + 4 * (int64_t)block - 1) / (4 * (int64_t)block);
    const int64_t g = std::max<int64_t>(1, std::min<int64_t>(need, grid));
    hipLaunchKernelGGL(k_ic_stream, dim3((unsigned)g), dim3((unsigned)block), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ic_clear(const StepArgs &a, hipStream_t s)
{
    const int64_t work = ((int64_t)a.n + 31) >> 5;
    hipLaunchKernelGGL(k_ic_clear, dim3(grid_for(work, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_expand_rows(const int32_t *ptr, int64_t n, int32_t *dst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, ptr, n, dst);
    return hipGetLastError();
}

int step_blocks(const StepArgs &a, int block)
{
    const int waves = block / 64;  // one heavy-row segment per wave
    return (a.n_seg + waves - 1) / waves + a.n_tiles;
}

hipError_t launch_batch_step(const BatchCtl &c, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_step, dim3((unsigned)grid), dim3(kBatchBlock), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_batch_combine(const BatchCtl &c, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_combine, dim3((unsigned)grid), dim3(kBatchBlock), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_batch_expand(const BatchCtl &c, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_expand, dim3(1024), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_batch_count(const BatchCtl &c, uint32_t t, unsigned long long *counts, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_count, dim3(2048), dim3(256), 0, s, c, t, counts);
    return hipGetLastError();
}

hipError_t launch_batch_advance(const BatchCtl &c, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinArgs &f, hipStream_t s)
{
    // a wave per 64 words, as many as that takes: the finalize mostly writes
    // (R-MAT scale 26 at B = 64: 0.771 ms with 262,144 blocks, 0.82 with
    // the 65,536 of two 64-word blocks a wave, 0.85 with 16,384)
    const int64_t waves = ((int64_t)f.n * f.G + 63) / 64;
    int64_t blocks = (waves + 3) / 4;
    if (blocks < 1) blocks = 1;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    const bool dense = f.G == f.W && f.B == 64ll * f.W &&
                       ((uintptr_t)f.states & 15u) == 0;
    if (dense)
        hipLaunchKernelGGL(k_finalize_dense, dim3((unsigned)blocks), dim3(256), 0, s, f);
    else
        hipLaunchKernelGGL(k_finalize, dim3((unsigned)blocks), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_tally(const FinArgs &f, hipStream_t s)
{
    hipLaunchKernelGGL(k_tally_clear, dim3(1), dim3(64), 0, s, f.tally);
    const int64_t words = (int64_t)f.n * f.W;
    hipLaunchKernelGGL(k_tally, dim3(grid_for(words, 256)), dim3(256), 0, s, f);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out,
                         int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_philox, dim3(grid_for(count, 256)), dim3(256), 0, s, ctr, k0, k1, out,
                       count);
    return hipGetLastError();
}

}  // namespace fsg
