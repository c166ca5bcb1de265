// fsg_abi.hip -- host side of libfsg: argument validation, FP64 threshold
// tables, the row-tile planner, workspace layout and the step loop.
// Declarations and contracts: include/fsg.h.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <fstream>
#include <sstream>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fsg.h"
#include "fsg_internal.hpp"

using namespace fsg;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        if (fsg::inject_device_fault())                                                     \
            return fail(FSG_EDEVICE, std::string(#expr) + ": injected fault");              \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(FSG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

// FSG_FAULT_INJECT: the call numbers at which a guarded allocation or a
// checked HIP call fails (0: never), parsed on first use.
struct FaultPlan {
    long alloc_at = 0, device_at = 0;
    std::atomic<long> allocs{0}, devices{0};
    FaultPlan()
    {
        const char *env = getenv("FSG_FAULT_INJECT");
        if (!env) return;
        std::string spec(env);
        size_t pos = 0;
        while (pos <= spec.size()) {
            size_t end = spec.find(',', pos);
            if (end == std::string::npos) end = spec.size();
            const std::string item = spec.substr(pos, end - pos);
            const size_t c = item.find(':');
            if (c != std::string::npos) {
                const long at = atol(item.c_str() + c + 1);
                if (item.compare(0, c, "alloc") == 0) alloc_at = at;
                if (item.compare(0, c, "device") == 0) device_at = at;
            }
            pos = end + 1;
        }
    }
};

FaultPlan &fault_plan()
{
    static FaultPlan plan;
    return plan;
}

// Probability -> uint32 threshold (the Bernoulli fires iff t == 2^32-1 or
// draw < t).  Scaling by 2^32 is exact in FP64.
uint32_t threshold_of(double p)
{
    if (!(p > 0.0)) return 0u;
    if (p >= 1.0) return 0xFFFFFFFFu;
    double x = floor(p * 4294967296.0);
    return x > 4294967294.0 ? 0xFFFFFFFEu : (uint32_t)x;
}

// Appendix A.1: with k infected in-neighbours the infection probability is
// 1 - exp(k log(1-beta)) = 1 - (1-beta)^k.  The survival power is built by
// repeated FP64 multiplication; the table stops where it saturates.
std::vector<uint32_t> infection_table(double beta, int64_t max_k)
{
    std::vector<uint32_t> t;
    t.reserve((size_t)std::min<int64_t>(max_k + 1, 1 << 16));
    volatile double surv = 1.0;
    for (int64_t k = 0; k <= max_k; ++k) {
        if (k > 0) surv = surv * (1.0 - beta);
        const uint32_t x = threshold_of(1.0 - surv);
        t.push_back(x);
        if (x == 0xFFFFFFFFu) break;  // every later entry is "always" too
    }
    return t;
}

bool bad_prob(double p) { return !(p >= 0.0 && p <= 1.0); }

int64_t next_pow2(int64_t x)
{
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

int ilog2(int64_t x)
{
    int l = 0;
    while ((1ll << l) < x) ++l;
    return l;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Largest arc count: arc indices are int32 in the kernels, which look up to
// 4 * 64 positions past an index they hold (unrolled loads of the row-group
// loops, lanes past a row's end), so every such position stays below 2^31.
constexpr int64_t kMaxNnz = ((int64_t)1 << 31) - 256;

struct Plan {
    std::vector<int32_t> tiles;      // (row_begin, row_end) pairs; no heavy rows inside
    std::vector<int32_t> heavy_rows; // rows with indeg > heavy
    std::vector<int32_t> heavy_seg;  // [n_heavy + 1] first segment of each heavy row
    std::vector<int32_t> seg_row, seg_e0, seg_e1;
    int64_t max_light = 0;           // largest light in-degree
    int64_t max_seg = 0;             // longest segment
};

}  // namespace

struct fsg_graph {
    int64_t n = 0, nnz = 0, max_indeg = 0;
    std::vector<int64_t> ptr;
    const int32_t *src_host = nullptr;
    bool bound = false;
    int32_t *d_ptr = nullptr;
    int32_t *d_src = nullptr;
    int32_t *d_dst = nullptr;  // target row of every arc (built on the device at bind)
    std::vector<int32_t> wide;  // rows with more than kWideRow in-arcs, largest first
    int32_t *d_wide = nullptr;
    // out-adjacency (fsg_graph_bind_out): arcs grouped by source
    bool has_out = false;
    int32_t *d_optr = nullptr;
    int2 *d_oarc = nullptr;
    int64_t out_items = 0;  // sum over nodes of max(1, ceil(outdeg / kOutChunk))
    std::map<std::tuple<int64_t, int64_t, int64_t>, Plan> plans;
};

namespace fsg {

int set_error(int code, const char *msg) { return fail(code, msg); }

void inject_alloc_fault()
{
    FaultPlan &f = fault_plan();
    if (f.alloc_at > 0 && f.allocs.fetch_add(1) + 1 == f.alloc_at) throw std::bad_alloc();
}

bool inject_device_fault()
{
    FaultPlan &f = fault_plan();
    return f.device_at > 0 && f.devices.fetch_add(1) + 1 == f.device_at;
}

bool graph_view(const fsg_graph *g, int64_t *n, int64_t *nnz, int64_t *max_indeg,
                const int32_t **ptr, const int32_t **src, const int32_t **wide, int64_t *n_wide)
{
    if (!g || !g->bound) return false;
    *wide = g->d_wide;
    *n_wide = (int64_t)g->wide.size();
    *n = g->n;
    *nnz = g->nnz;
    *max_indeg = g->max_indeg;
    *ptr = g->d_ptr;
    *src = g->d_src;
    return true;
}

}  // namespace fsg

// Target-node partition by prefix sums (Sec. 3.2, Definition "Target-Node-
// Based Partitioning"): node i with prefix load C_i goes to part
// ceil(d C_i / W_total); here the nodes keep their CSR order so each part is
// a contiguous row range owned by one workgroup.  Load of a row: in-degree
// (0 for heavy rows, which are processed as segments) plus row_cost.
extern "C" int fsg_plan_row_tiles(const int64_t *in_ptr, int64_t n, int64_t heavy,
                                  int64_t row_cost, int64_t n_parts, int64_t *bounds_out,
                                  int64_t *n_out)
{
    if (!in_ptr || !bounds_out || !n_out || n < 1 || n_parts < 1 || row_cost < 0)
        return fail(FSG_EINVAL, "fsg_plan_row_tiles: bad arguments");
    unsigned __int128 total = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = in_ptr[v + 1] - in_ptr[v];
        total += (unsigned __int128)((d > heavy ? 0 : d) + row_cost);
    }
    int64_t nb = 0;
    bounds_out[nb++] = 0;
    if (total == 0) {
        bounds_out[nb++] = n;
        *n_out = nb - 1;
        return FSG_OK;
    }
    unsigned __int128 c = 0;
    int64_t cur = 1;  // part of the rows seen so far
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = in_ptr[v + 1] - in_ptr[v];
        c += (unsigned __int128)((d > heavy ? 0 : d) + row_cost);
        const unsigned __int128 num = (unsigned __int128)n_parts * c;
        int64_t q = (int64_t)((num + total - 1) / total);
        if (q < 1) q = 1;
        if (q > cur) {
            // row v opens part q: close the previous one before v (if non-empty)
            if (v > bounds_out[nb - 1]) bounds_out[nb++] = v;
            cur = q;
        }
    }
    if (bounds_out[nb - 1] != n) bounds_out[nb++] = n;
    *n_out = nb - 1;
    return FSG_OK;
}

namespace {

constexpr int64_t kRowCost = 4;

const Plan &get_plan(fsg_graph *g, int64_t heavy, int64_t tile_edges)
{
    auto key = std::make_tuple(heavy, tile_edges, kRowCost);
    auto it = g->plans.find(key);
    if (it != g->plans.end()) return it->second;
    Plan p;
    const int64_t n = g->n;
    const int64_t *ptr = g->ptr.data();
    unsigned __int128 total = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = ptr[v + 1] - ptr[v];
        total += (unsigned __int128)((d > heavy ? 0 : d) + kRowCost);
        if (d > heavy) {
            p.heavy_rows.push_back((int32_t)v);
            p.heavy_seg.push_back((int32_t)p.seg_row.size());
            for (int64_t e = ptr[v]; e < ptr[v + 1]; e += heavy) {
                p.seg_row.push_back((int32_t)v);
                p.seg_e0.push_back((int32_t)e);
                p.seg_e1.push_back((int32_t)std::min(ptr[v + 1], e + heavy));
            }
            p.max_seg = std::max(p.max_seg, std::min(d, heavy));
        } else {
            p.max_light = std::max(p.max_light, d);
        }
    }
    p.heavy_seg.push_back((int32_t)p.seg_row.size());
    int64_t parts = (int64_t)((total + (unsigned __int128)tile_edges - 1) / (unsigned __int128)tile_edges);
    parts = std::max<int64_t>(1, std::min<int64_t>(parts, n));
    std::vector<int64_t> b((size_t)n + 2);
    int64_t nt = 0;
    fsg_plan_row_tiles(ptr, n, heavy, kRowCost, parts, b.data(), &nt);
    // heavy rows are cut out of the parts (their segments are separate work
    // items) and no tile holds more than kMaxTileRows rows
    for (int64_t i = 0; i < nt; ++i) {
        int64_t r = b[(size_t)i];
        const int64_t end = b[(size_t)i + 1];
        while (r < end) {
            while (r < end && ptr[r + 1] - ptr[r] > heavy) ++r;
            int64_t q = r;
            while (q < end && q - r < kMaxTileRows && ptr[q + 1] - ptr[q] <= heavy) ++q;
            if (q > r) {
                p.tiles.push_back((int32_t)r);
                p.tiles.push_back((int32_t)q);
            }
            r = q;
        }
    }
    if (p.tiles.empty()) {  // every row heavy: one empty tile keeps the grid valid
        p.tiles.push_back(0);
        p.tiles.push_back(0);
    }
    return g->plans.emplace(key, std::move(p)).first->second;
}

int model_kind(int model)
{
    if (model == kIC) return kKindIC;
    if (model == kLT) return kKindLT;
    return kKindEpidemic;
}

int check_params(const fsg_graph *g, const fsg_params *prm, int64_t B)
{
    if (!g) return fail(FSG_EINVAL, "graph is NULL");
    if (!prm) return fail(FSG_EINVAL, "params is NULL");
    if (prm->model < FSG_IC || prm->model > FSG_SWIR) return fail(FSG_EINVAL, "unknown model");
    if (B < 1) return fail(FSG_EINVAL, "B must be >= 1");
    if (B > (int64_t)1 << 31) return fail(FSG_EUNSUPPORTED, "B above 2^31");
    const bool swir = prm->model == FSG_SWIR;
    const bool latent = prm->model == FSG_SEIR || prm->model == FSG_SEIS || swir;
    const bool epi = prm->model == FSG_SI || prm->model == FSG_SIS || prm->model == FSG_SIR || latent;
    if (epi && !swir && prm->max_steps < 0)
        return fail(FSG_EINVAL, "SI/SIS/SIR/SEIR/SEIS need max_steps >= 0");
    if (prm->max_steps > 0x7FFFFFFF) return fail(FSG_EUNSUPPORTED, "max_steps above 2^31-1");
    if (prm->model == FSG_IC) {
        if (prm->ic_prob < FSG_IC_UNIFORM || prm->ic_prob > FSG_IC_PER_EDGE)
            return fail(FSG_EINVAL, "unknown ic_prob");
        if (prm->ic_prob == FSG_IC_UNIFORM && bad_prob(prm->p))
            return fail(FSG_EINVAL, "p must be in [0, 1]");
        if (prm->ic_prob == FSG_IC_PER_EDGE) {
            if (g->nnz > 0 && !prm->edge_p) return fail(FSG_EINVAL, "edge_p is NULL");
            for (int64_t e = 0; e < g->nnz; ++e)
                if (bad_prob(prm->edge_p[e])) return fail(FSG_EINVAL, "edge_p[e] outside [0, 1]");
        }
    }
    if (epi) {
        if (bad_prob(prm->beta)) return fail(FSG_EINVAL, "beta must be in [0, 1]");
        if (prm->model != FSG_SI && bad_prob(prm->gamma))
            return fail(FSG_EINVAL, "gamma must be in [0, 1]");
        if (latent && bad_prob(prm->alpha)) return fail(FSG_EINVAL, "alpha must be in [0, 1]");
        if (swir && !(prm->beta + prm->alpha <= 1.0))
            return fail(FSG_EINVAL, "SWIR needs beta + alpha <= 1 (kappa + mu)");
    }
    return FSG_OK;
}

struct Sched {
    int G, S, lgG, lgS, block, tile_edges, heavy, sync, timed;
    bool edge1;  // edge-parallel IC kernel (frontier bitmap and summary)
    bool push;   // frontier-driven IC: work queues, push over out-arcs or stream
    bool wide;   // 64-bit offsets in the row-group kernels even where 32-bit ones fit
    bool count;  // count the generator calls of the SI-family decisions
    bool reuse;  // the caller vouches for the workspace (FSG_OPT_REUSE_WORKSPACE)
    bool tail;   // SI family, LT, pull-step IC: tail mode allowed
    bool tail_always;  // ... and taken from the second chunk on (FSG_OPT_TAIL_ALWAYS)
};

void default_sched(const fsg_graph *g, const fsg_params *prm, int64_t B, fsg_schedule *o)
{
    const int64_t W = (B + 63) / 64;
    memset(o, 0, sizeof(*o));
    // lanes over words first; an edge split only for narrow batches
    o->row_lanes = (int32_t)std::max<int64_t>(16, std::min<int64_t>(next_pow2(W), 64));
    // SI-family rows of 33-48 words: three 16-lane passes fill 48 lane slots
    // where one 64-lane pass leaves up to 31 idle through the draws
    if (model_kind(prm->model) == kKindEpidemic && W > 32 && W <= 48) o->row_lanes = 16;
    o->block_threads = 256;
    o->tile_edges = 4096;
    o->heavy_threshold = 1024;
    o->steps_per_sync = 16;
    o->kernel_variant = (prm->model == FSG_IC && W == 1) ? (g && g->has_out ? 3 : 2) : 1;
    if (o->kernel_variant >= 2) {  // measured best on R-MAT scale 26 at B = 64
        o->block_threads = 512;
        o->tile_edges = 16384;
        o->heavy_threshold = 32768;
    }
    // frontier-driven steps take microseconds and go back to back; a poll
    // of the absorption flags (a host round trip with the GPU idle) costs
    // more than the early-exit launches after absorption that longer chunks
    // leave (web-scale run, 18 steps: 1.40 / 1.40 / 1.34 ms per run with
    // chunks of 8 / 16 / 32)
    if (o->kernel_variant == 3) o->steps_per_sync = 32;
}

int resolve_sched(const fsg_graph *g, const fsg_params *prm, int64_t B, const fsg_schedule *in,
                  Sched *s)
{
    fsg_schedule d;
    default_sched(g, prm, B, &d);
    fsg_schedule u = in ? *in : d;
    if (u.row_lanes == 0) u.row_lanes = d.row_lanes;
    if (u.block_threads == 0) u.block_threads = d.block_threads;
    if (u.tile_edges == 0) u.tile_edges = d.tile_edges;
    if (u.heavy_threshold == 0) u.heavy_threshold = d.heavy_threshold;
    if (u.steps_per_sync == 0) u.steps_per_sync = d.steps_per_sync;
    if (u.kernel_variant == 0) u.kernel_variant = d.kernel_variant;
    if (u.kernel_variant < 1 || u.kernel_variant > 3)
        return fail(FSG_EINVAL, "kernel_variant must be 0, 1, 2 or 3");
    if (u.kernel_variant >= 2 && !(prm->model == FSG_IC && B <= 64))
        return fail(FSG_EINVAL, "kernel_variants 2 and 3 need IC with B <= 64");
    if (u.kernel_variant == 3 && !g->has_out)
        return fail(FSG_EINVAL, "kernel_variant 3 needs the graph's out-adjacency (fsg_graph_bind_out)");
    if (u.row_lanes < 1 || u.row_lanes > 64 || (u.row_lanes & (u.row_lanes - 1)))
        return fail(FSG_EINVAL, "row_lanes must be a power of two in [1, 64]");
    if (u.block_threads < 64 || u.block_threads > 1024 || (u.block_threads & (u.block_threads - 1)))
        return fail(FSG_EINVAL, "block_threads must be a power of two in [64, 1024]");
    if (u.tile_edges < 1) return fail(FSG_EINVAL, "tile_edges must be >= 1");
    if (u.heavy_threshold < 1 || u.heavy_threshold > 65535)
        return fail(FSG_EINVAL, "heavy_threshold must be in [1, 65535]");
    if (u.steps_per_sync < 1 || u.steps_per_sync > 4096)
        return fail(FSG_EINVAL, "steps_per_sync must be in [1, 4096]");
    const int64_t W = (B + 63) / 64;
    const int64_t G = std::min<int64_t>(u.row_lanes, std::min<int64_t>(next_pow2(W), 64));
    s->G = (int)G;
    s->S = (int)(u.row_lanes / G);
    s->lgG = ilog2(s->G);
    s->lgS = ilog2(s->S);
    s->block = u.block_threads;
    s->tile_edges = u.tile_edges;
    s->heavy = u.heavy_threshold;
    s->sync = u.steps_per_sync;
    s->timed = u.time_kernels != 0;
    s->edge1 = u.kernel_variant >= 2;
    s->push = u.kernel_variant == 3;
    if (s->push) s->block = 512;
    if (u.options & ~(FSG_OPT_WIDE_OFFSETS | FSG_OPT_COUNT_DRAWS | FSG_OPT_REUSE_WORKSPACE |
                      FSG_OPT_TAIL_OFF | FSG_OPT_TAIL_ALWAYS))
        return fail(FSG_EINVAL, "unknown schedule option bits");
    if ((u.options & FSG_OPT_TAIL_OFF) && (u.options & FSG_OPT_TAIL_ALWAYS))
        return fail(FSG_EINVAL, "FSG_OPT_TAIL_OFF and FSG_OPT_TAIL_ALWAYS together");
    s->wide = (u.options & FSG_OPT_WIDE_OFFSETS) != 0;
    s->count = (u.options & FSG_OPT_COUNT_DRAWS) != 0;
    s->reuse = (u.options & FSG_OPT_REUSE_WORKSPACE) != 0;
    // the tail mode: SI, SIS, SIR (no latent plane), LT, and IC on the pull
    // step (the edge-parallel IC steps find their frontier themselves)
    s->tail = (prm->model == FSG_SI || prm->model == FSG_SIS || prm->model == FSG_SIR ||
               prm->model == FSG_LT || (prm->model == FSG_IC && !s->edge1)) &&
              !(u.options & FSG_OPT_TAIL_OFF);
    s->tail_always = s->tail && (u.options & FSG_OPT_TAIL_ALWAYS) != 0;
    return FSG_OK;
}

struct Layout {
    size_t planes[4];
    int n_planes;
    size_t flags, wflags, tiles, heavy_rows, heavy_seg, seg_row, seg_e0, seg_e1, partial, tinf, edge_t,
        seeds, bm[3], sum[3], ever, need, stamp, ibm, icount, queue[4], qctl, draws, tag, total;
    int sum_shift, sum_words;
    int64_t W, plane_words, n_tinf, n_seed_stage;
    int L;
};

constexpr int64_t kSeedStage = 65536;

// HIP events for optional per-step timing, released on scope exit.
// Events of a timed call come from a per-thread list of released ones, so a
// run does not create and destroy its events (a timed SIR run polls 25 times,
// with 16 events a poll).  Each entry remembers its device; the list is never
// torn down (its events live until the process ends).
struct CachedEvent {
    int dev;
    hipEvent_t ev;
};
constexpr size_t kEventCacheMax = 4096;
std::vector<CachedEvent> &event_cache()
{
    thread_local std::vector<CachedEvent> *c = new std::vector<CachedEvent>();
    return *c;
}

struct EventPool {
    EventPool() = default;
    EventPool(const EventPool &) = delete;
    EventPool &operator=(const EventPool &) = delete;
    std::vector<hipEvent_t> e;
    int dev = -1;
    hipError_t init(size_t count)
    {
        release();
        hipError_t r = hipGetDevice(&dev);
        if (r != hipSuccess) return r;
        std::vector<CachedEvent> &c = event_cache();
        e.assign(count, nullptr);
        for (auto &x : e) {
            for (size_t i = c.size(); i-- > 0;)
                if (c[i].dev == dev) {
                    x = c[i].ev;
                    c[i] = c.back();
                    c.pop_back();
                    break;
                }
            if (!x) {
                r = hipEventCreate(&x);
                if (r != hipSuccess) return r;
            }
        }
        return hipSuccess;
    }
    void release()
    {
        std::vector<CachedEvent> &c = event_cache();
        for (auto x : e) {
            if (!x) continue;
            if (c.size() < kEventCacheMax)
                c.push_back({dev, x});
            else
                (void)hipEventDestroy(x);
        }
        e.clear();
    }
    ~EventPool() { release(); }
};

int layout(fsg_graph *g, const fsg_params *prm, int64_t B, const Sched &s, const Plan &p,
           Layout *L)
{
    const int kind = model_kind(prm->model);
    L->W = (B + 63) / 64;
    // one extra all-zero row (index n): gathers of padding lanes read it
    L->plane_words = (g->n + 1) * L->W;
    const bool latent = prm->model == FSG_SEIR || prm->model == FSG_SEIS || prm->model == FSG_SWIR;
    // frontier-driven IC keeps a third frontier plane (index 3)
    L->n_planes = kind == kKindLT ? 2 : ((latent || s.push) ? 4 : 3);
    L->L = kind == kKindIC ? 1 : counter_planes_for(std::max(p.max_light, p.max_seg));
    // room for the longest table (it stops early once it saturates), so the
    // workspace size does not depend on beta
    // SWIR keeps three tables (S -> I, S -> I or W, W -> I) of that length
    L->n_tinf = (kind == kKindEpidemic ? g->max_indeg + 1 : 1) * (prm->model == FSG_SWIR ? 3 : 1);
    L->n_seed_stage = std::min<int64_t>(g->n, kSeedStage);
    size_t off = 0;
    for (int i = 0; i < L->n_planes; ++i) {
        L->planes[i] = off;
        off = align256(off + (size_t)L->plane_words * 8);
    }
    const int ring = s.sync + 1;
    L->flags = off; off = align256(off + (size_t)ring * 4);
    L->wflags = off;  // per-word flags [ring + 1][W] when 16 < W <= 64
    if (L->W > 16 && L->W <= 64) off = align256(off + (size_t)(ring + 1) * (size_t)L->W * 4);
    L->tiles = off; off = align256(off + p.tiles.size() * 4);
    L->heavy_rows = off; off = align256(off + (p.heavy_rows.size() + 1) * 4);
    L->heavy_seg = off; off = align256(off + p.heavy_seg.size() * 4);
    L->seg_row = off; off = align256(off + (p.seg_row.size() + 1) * 4);
    L->seg_e0 = off; off = align256(off + (p.seg_e0.size() + 1) * 4);
    L->seg_e1 = off; off = align256(off + (p.seg_e1.size() + 1) * 4);
    L->partial = off; off = align256(off + p.seg_row.size() * (size_t)L->L * (size_t)L->W * 8);
    L->tinf = off; off = align256(off + (size_t)L->n_tinf * 4);
    L->edge_t = off;
    if (prm->model == FSG_IC && prm->ic_prob == FSG_IC_PER_EDGE)
        off = align256(off + (size_t)g->nnz * 4);
    L->seeds = off; off = align256(off + (size_t)L->n_seed_stage * 4);
    L->need = off;
    if (kind == kKindLT)  // bit-sliced thresholds [n][L][W]
        off = align256(off + (size_t)g->n * (size_t)L->L * (size_t)L->W * 8);
    L->stamp = off;
    if (kind == kKindLT) off = align256(off + (size_t)g->n * 8);  // gain steps, two arrays
    L->ibm = off;  // tail mode: four infected-node (IC, LT: new-activation) and two candidate bitmaps
    if (s.tail) off = align256(off + 6 * (size_t)((g->n + 31) / 32) * 4);
    L->icount = off;  // nodes with an infected replicate (tail-mode decisions)
    if (s.tail) off = align256(off + 8);
    for (int i = 0; i < 3; ++i) L->bm[i] = L->sum[i] = 0;
    for (int i = 0; i < 4; ++i) L->queue[i] = 0;
    L->qctl = 0;
    L->sum_shift = 0;
    L->sum_words = 0;
    if (s.edge1) {
        const int nbuf = s.push ? 3 : 2;
        const size_t bmb = (size_t)((g->n + 31) / 32) * 4;
        for (int i = 0; i < nbuf; ++i) {
            L->bm[i] = off;
            off = align256(off + bmb);
        }
        // coarsest summary that fits the kernel's LDS copy, at least 256 nodes a bit
        int sh = 8;
        while ((((g->n - 1) >> sh) >> 5) + 1 > kSumWords) ++sh;
        L->sum_shift = sh;
        L->sum_words = (int)((((g->n - 1) >> sh) >> 5) + 1);
        for (int i = 0; i < nbuf; ++i) {
            L->sum[i] = off;
            off = align256(off + (size_t)L->sum_words * 4);
        }
    }
    L->ever = off;  // frontier-driven IC: bit per node ever in a frontier
    if (s.push) off = align256(off + (size_t)((g->n + 31) / 32) * 4);
    L->draws = off;  // generator-call counter (counting runs)
    off = align256(off + 8);
    if (s.push) {  // four queues of 16-byte items; counters: uint32 [4], uint64 [4]
        for (int i = 0; i < 4; ++i) {
            L->queue[i] = off;
            off = align256(off + (size_t)std::max<int64_t>(g->out_items, 1) * 16);
        }
        L->qctl = off;
        off = align256(off + 64);
    }
    L->tag = off;  // frontier-driven IC: which layout last left its buffers clear
    if (s.push) off = align256(off + 8);
    L->total = off;
    return FSG_OK;
}

}  // namespace

namespace {

int validate_run(fsg_graph *g, const fsg_params *prm, const int32_t *seeds, int64_t n_seeds,
                 int64_t B, int64_t replicate_offset)
{
    int rc = check_params(g, prm, B);
    if (rc) return rc;
    if (!g->bound) return fail(FSG_EINVAL, "graph is not bound to device memory");
    if (replicate_offset < 0 || replicate_offset + B > ((int64_t)1 << 34))
        return fail(FSG_EINVAL, "replicate_offset + B must lie in [0, 2^34]");
    if (n_seeds < 0 || (n_seeds > 0 && !seeds)) return fail(FSG_EINVAL, "bad seed array");
    for (int64_t i = 0; i < n_seeds; ++i)
        if (seeds[i] < 0 || (int64_t)seeds[i] >= g->n)
            return fail(FSG_EINVAL, "seed out of range at index " + std::to_string(i));
    return FSG_OK;
}

// Tag a frontier-driven IC run writes into its workspace once it has left
// its planes, bitmaps and summaries clear: a hash of the layout, the graph,
// the parameters and the workspace address, never 0 (the value a run in
// progress leaves there).
uint64_t clean_tag(const fsg_graph *g, const fsg_params *prm, int64_t B, const struct Layout &L,
                   const char *base)
{
    uint64_t h = 0x6A09E667F3BCC908ull;
    auto mix = [&](uint64_t x) {
        h ^= x + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 31;
    };
    mix((uint64_t)(uintptr_t)base);
    mix((uint64_t)g->n);
    mix((uint64_t)g->nnz);
    mix((uint64_t)B);
    mix((uint64_t)prm->model);
    mix((uint64_t)L.total);
    mix((uint64_t)L.planes[0]);
    mix((uint64_t)L.bm[0]);
    mix((uint64_t)L.tag);
    return h ? h : 1ull;
}

// One job on the device: its planes, tables and launch arguments.
struct Job {
    StepArgs a;
    Layout L;
    Sched s;
    int kind = 0;
    int ring = 0;
    int64_t K = 0;
    int64_t n = 0;
    int64_t B = 0;
    int model = 0;
    uint64_t *pl[4] = {nullptr, nullptr, nullptr, nullptr};
    uint32_t *bm[3] = {nullptr, nullptr, nullptr};
    uint32_t *sum[3] = {nullptr, nullptr, nullptr};
    uint4 *queue[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<uint32_t> tinf_h, edge_t_h;  // host tables the set-up uploads
    uint32_t *ever = nullptr;                // frontier-driven IC: ever-in-a-frontier bitmap
    uint32_t *ibm = nullptr;                 // tail mode: infected-node and candidate bitmaps
    bool tail = false;                       // the tail mode can be taken (out-adjacency bound)
    unsigned long long *icount = nullptr;    // tail mode: nodes infected (IC, LT: newly activated)
    uint64_t *tag = nullptr;                 // frontier-driven IC: clean-buffers tag
    uint64_t tag_value = 0;                  // the tag this job's layout writes
    // frontier plane (state 1) and its bitmap after step t: the planes
    // alternate, or rotate over three in the frontier-driven IC path
    static int mod3(int64_t t) { return (int)(((t % 3) + 3) % 3); }
    uint64_t *front(int64_t t) const
    {
        return s.push ? pl[mod3(t) == 2 ? 3 : mod3(t)] : pl[t & 1];
    }
    uint32_t *front_bm(int64_t t) const
    {
        return s.edge1 ? (s.push ? bm[mod3(t)] : bm[t & 1]) : nullptr;
    }
    uint32_t *front_sum(int64_t t) const { return s.push ? sum[mod3(t)] : sum[t & 1]; }
};

// Uploads the job's tables into `base`, clears its planes and seeds them
// (every replicate starts with the seeds in state 1).  `flags` is the job's
// absorption ring.  Returns after the stream has drained.
int setup_job(fsg_graph *g, const fsg_params *prm, const int32_t *seeds, int64_t n_seeds,
              int64_t B, int64_t replicate_offset, uint64_t rng_key, const Sched &s,
              const Plan &p, const Layout &L, char *base, uint32_t *flags, hipStream_t st,
              Job *jb)
{
    const int kind = model_kind(prm->model);
    jb->L = L;
    jb->s = s;
    jb->kind = kind;
    jb->ring = s.sync + 1;
    jb->K = prm->max_steps < 0 ? g->n : prm->max_steps;
    jb->n = g->n;
    jb->B = B;
    jb->model = prm->model;
    // plane roles: IC {F0, F1, A}; epidemic {h0, h1, r}, SEIR / SEIS also
    // the latent plane e; LT {act0, act1}
    for (int i = 0; i < 4; ++i)
        jb->pl[i] = i < L.n_planes ? (uint64_t *)(base + L.planes[i]) : nullptr;
    const int ring = jb->ring;

    // host tables stay in the job until the run ends: the copies below are
    // not waited for
    std::vector<uint32_t> &tinf = jb->tinf_h;
    tinf.assign(1, 0u);
    if (kind == kKindEpidemic) tinf = infection_table(prm->beta, g->max_indeg);
    // SWIR: kappa = beta (S -> I), mu = alpha (S -> W), nu = gamma (W -> I);
    // S -> I or W with 1 - (1 - kappa - mu)^k, the sum formed in FP64
    const bool swir = prm->model == FSG_SWIR;
    const size_t n_si = tinf.size();
    size_t n_siw = 0, n_wi = 0;
    if (swir) {
        const std::vector<uint32_t> siw = infection_table(prm->beta + prm->alpha, g->max_indeg);
        const std::vector<uint32_t> wi = infection_table(prm->gamma, g->max_indeg);
        n_siw = siw.size();
        n_wi = wi.size();
        tinf.insert(tinf.end(), siw.begin(), siw.end());
        tinf.insert(tinf.end(), wi.begin(), wi.end());
    }
    std::vector<uint32_t> &edge_t = jb->edge_t_h;
    edge_t.clear();
    if (prm->model == FSG_IC && prm->ic_prob == FSG_IC_PER_EDGE) {
        edge_t.resize((size_t)g->nnz);
        for (int64_t e = 0; e < g->nnz; ++e) edge_t[(size_t)e] = threshold_of(prm->edge_p[e]);
    }
    auto up = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, st);
    };
    if (!s.push) {  // the frontier-driven IC step reads no row tiles, segments or tables
        HIP_TRY(up(L.tiles, p.tiles.data(), p.tiles.size() * 4));
        HIP_TRY(up(L.heavy_rows, p.heavy_rows.data(), p.heavy_rows.size() * 4));
        HIP_TRY(up(L.heavy_seg, p.heavy_seg.data(), p.heavy_seg.size() * 4));
        HIP_TRY(up(L.seg_row, p.seg_row.data(), p.seg_row.size() * 4));
        HIP_TRY(up(L.seg_e0, p.seg_e0.data(), p.seg_e0.size() * 4));
        HIP_TRY(up(L.seg_e1, p.seg_e1.data(), p.seg_e1.size() * 4));
        HIP_TRY(up(L.tinf, tinf.data(), tinf.size() * 4));
    }
    HIP_TRY(up(L.edge_t, edge_t.data(), edge_t.size() * 4));

    // the planes lie back to back (256-byte aligned): one zeroing launch.
    // A frontier-driven IC run clears what it wrote before it ends; with
    // FSG_OPT_REUSE_WORKSPACE the planes, bitmaps and summaries are cleared
    // only if the tag of this layout is not in the workspace.
    const size_t plane_bytes = L.planes[L.n_planes - 1] + (size_t)L.plane_words * 8 - L.planes[0];
    if (s.push) {
        jb->tag = (uint64_t *)(base + L.tag);
        jb->ever = (uint32_t *)(base + L.ever);
        jb->tag_value = clean_tag(g, prm, B, L, base);
        const size_t bm_bytes = align256(L.ever + (size_t)((g->n + 31) / 32) * 4) - L.bm[0];
        if (s.reuse) {
            HIP_TRY(launch_zero_unless(base + L.planes[0], align256(plane_bytes), jb->tag,
                                       jb->tag_value, st));
            HIP_TRY(launch_zero_unless(base + L.bm[0], bm_bytes, jb->tag, jb->tag_value, st));
        } else {
            HIP_TRY(launch_zero(base + L.planes[0], plane_bytes, st));
            HIP_TRY(launch_zero(base + L.bm[0], bm_bytes, st));
        }
        HIP_TRY(launch_fill64(jb->tag, 1, 0ull, st));  // dirty until the run has cleared up
    } else {
        HIP_TRY(launch_zero(base + L.planes[0], plane_bytes, st));
    }
    HIP_TRY(launch_fill32(flags, ring, 0u, st));
    uint32_t *wflags = (L.W > 16 && L.W <= 64) ? (uint32_t *)(base + L.wflags) : nullptr;
    if (wflags) {  // every word is live before step 1 (slot 0); the others clear
        HIP_TRY(launch_fill32(wflags, L.W, 1u, st));
        HIP_TRY(launch_fill32(wflags + L.W, (int64_t)ring * L.W, 0u, st));
    }
    if (s.edge1) {
        for (int i = 0; i < (s.push ? 3 : 2); ++i) {
            jb->bm[i] = (uint32_t *)(base + L.bm[i]);
            jb->sum[i] = (uint32_t *)(base + L.sum[i]);
            if (s.push) continue;  // cleared above with the planes
            HIP_TRY(launch_fill32(jb->bm[i], (g->n + 31) / 32, 0u, st));
            HIP_TRY(launch_fill32(jb->sum[i], L.sum_words, 0u, st));
        }
    }
    uint32_t *qcnt = nullptr;
    unsigned long long *qarcs = nullptr;
    if (s.push) {
        for (int i = 0; i < 4; ++i) jb->queue[i] = (uint4 *)(base + L.queue[i]);
        qcnt = (uint32_t *)(base + L.qctl);
        qarcs = (unsigned long long *)(base + L.qctl + 32);
        HIP_TRY(launch_fill32(qcnt, 16, 0u, st));  // counters and arc sums of the four queues
    }
    StepArgs sq;  // seeds join the frontier of step 0 (queue 0)
    memset(&sq, 0, sizeof(sq));
    if (s.push) {
        sq.ever = jb->ever;
        sq.bm_next = jb->bm[0];
        sq.sum_next = jb->sum[0];
        sq.sum_shift = L.sum_shift;
        sq.optr = g->d_optr;
        sq.q_out = jb->queue[0];
        sq.qcnt = qcnt;
        sq.qarcs = qarcs;
        sq.qi_out = 0;
    }
    int32_t *dseeds = (int32_t *)(base + L.seeds);
    if (kind == kKindLT) HIP_TRY(launch_fill32((uint32_t *)(base + L.stamp), 2 * g->n, 0xFFFFFFFFu, st));
    if (s.tail) {
        jb->ibm = (uint32_t *)(base + L.ibm);
        jb->icount = (unsigned long long *)(base + L.icount);
    }
    jb->tail = s.tail && g->has_out;  // candidates come from the out-adjacency
    for (int64_t i0 = 0; i0 < n_seeds; i0 += L.n_seed_stage) {
        const int64_t cnt = std::min<int64_t>(L.n_seed_stage, n_seeds - i0);
        HIP_TRY(hipMemcpyAsync(dseeds, seeds + i0, (size_t)cnt * 4, hipMemcpyHostToDevice, st));
        uint64_t *second = kind == kKindIC ? jb->pl[2] : nullptr;  // IC: A too
        if (kind == kKindLT) HIP_TRY(launch_stamp_seeds((uint32_t *)(base + L.stamp), dseeds, cnt, st));
        if (s.push) HIP_TRY(launch_seed_queue(sq, dseeds, cnt, st));
        HIP_TRY(launch_seed(jb->pl[0], second, dseeds, cnt, (int32_t)L.W, B, flags, jb->bm[0],
                            jb->sum[0], L.sum_shift, st));
        // the staging array is reused by the next chunk of seeds
        if (i0 + cnt < n_seeds) HIP_TRY(hipStreamSynchronize(st));
    }

    StepArgs &a = jb->a;
    memset(&a, 0, sizeof(a));
    a.ptr = g->d_ptr;
    a.src = g->d_src;
    a.n = (int32_t)g->n;
    a.W = (int32_t)L.W;
    a.B = B;
    a.goff = (uint64_t)replicate_offset;
    a.key0 = (uint32_t)rng_key;
    a.key1 = (uint32_t)(rng_key >> 32);
    a.prev = jb->pl[0];
    a.next = jb->pl[1];
    a.aux = jb->pl[2];
    a.model = prm->model;
    a.ic_prob = prm->ic_prob;
    a.ic_t = threshold_of(prm->p);
    a.edge_t = edge_t.empty() ? nullptr : (const uint32_t *)(base + L.edge_t);
    a.tinf = (const uint32_t *)(base + L.tinf);
    a.khat = (int32_t)n_si - 1;
    a.tsiw = swir ? a.tinf + n_si : nullptr;
    a.twi = swir ? a.tinf + n_si + n_siw : nullptr;
    a.khat_siw = swir ? (int32_t)n_siw - 1 : 0;
    a.khat_wi = swir ? (int32_t)n_wi - 1 : 0;
    a.trec = prm->model == FSG_SI ? 0u : threshold_of(prm->gamma);
    const bool latent = prm->model == FSG_SEIR || prm->model == FSG_SEIS || swir;
    a.talpha = (latent && !swir) ? threshold_of(prm->alpha) : 0u;
    a.lat = latent ? jb->pl[3] : nullptr;
    a.G = s.G;
    a.S = s.S;
    a.lgG = s.lgG;
    a.lgS = s.lgS;
    a.heavy = s.heavy;
    a.fast32 = (!s.wide && g->n + 1 < (1 << 24) && L.W < (1 << 21) &&
                (g->n + 1) * L.W < (1 << 29) && g->nnz < (1 << 30)) ? 1 : 0;
    a.tiles = (const int32_t *)(base + L.tiles);
    a.n_tiles = (int32_t)(p.tiles.size() / 2);
    a.seg_row = (const int32_t *)(base + L.seg_row);
    a.seg_e0 = (const int32_t *)(base + L.seg_e0);
    a.seg_e1 = (const int32_t *)(base + L.seg_e1);
    a.n_seg = (int32_t)p.seg_row.size();
    a.heavy_rows = (const int32_t *)(base + L.heavy_rows);
    a.heavy_seg = (const int32_t *)(base + L.heavy_seg);
    a.n_heavy = (int32_t)p.heavy_rows.size();
    a.partial = (uint64_t *)(base + L.partial);
    a.Lp = L.L;
    a.flags = flags;
    a.ring = ring;
    a.wflags = wflags;
    a.wring = ring + 1;
    a.dst = g->d_dst;
    a.nnz = g->nnz;
    a.sum_shift = L.sum_shift;
    a.sum_words = L.sum_words;
    a.need = nullptr;
    a.stamp = kind == kKindLT ? (uint32_t *)(base + L.stamp) : nullptr;
    a.draws = nullptr;
    if (s.count) {
        a.draws = (unsigned long long *)(base + L.draws);
        HIP_TRY(launch_fill64((uint64_t *)a.draws, 1, 0ull, st));
    }
    if (jb->tail) {
        a.optr = g->d_optr;
        a.oarc = g->d_oarc;
    }
    if (s.push) {
        a.ever = jb->ever;
        a.optr = g->d_optr;
        a.oarc = g->d_oarc;
        a.qcnt = qcnt;
        a.qarcs = qarcs;
        // push while the frontier's out-arcs are at most 1/16 of all arcs:
        // a pushed arc costs a random read of its target's word and more
        // address traffic than a streamed source (4 bytes)
        a.push_limit = (unsigned long long)(g->nnz / 16);
    }
    if (kind == kKindLT && g->n > 0) {
        a.need = (uint64_t *)(base + L.need);
        HIP_TRY(launch_lt_need(a, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return FSG_OK;
}

// End of a frontier-driven IC run whose finalize clears the ever-active
// plane: the frontiers of the last two steps leave their buffers (every
// earlier one was cleared by the step two after it), then the tag records
// that the run left its buffers clear.  Enqueued only.
hipError_t scrub_frontiers(const Job &jb, int64_t steps_run, hipStream_t st)
{
    StepArgs a = jb.a;
    for (int64_t t = steps_run + 1; t <= steps_run + 2; ++t) {
        a.qi_clr = (int32_t)((t + 2) % 4);
        a.q_clr = jb.queue[a.qi_clr];
        a.f_clr = jb.front(t - 2);
        a.bm_clr = jb.front_bm(t - 2);
        a.sum_clr = jb.front_sum(t - 2);
        hipError_t e = launch_ic_scrub(a, st);
        if (e != hipSuccess) return e;
    }
    return launch_fill64(jb.tag, 1, jb.tag_value, st);
}

// Packed planes of the step `steps_run` -> uint8 states and counts; with
// `scrub` (frontier-driven IC, one word per node) the run's buffers are left
// clear as well.
FinArgs fin_args(const Job &jb, int64_t steps_run, uint8_t *final_states, uint32_t *counts,
                 bool scrub)
{
    FinArgs f;
    memset(&f, 0, sizeof(f));
    f.n = (int32_t)jb.n;
    f.W = (int32_t)jb.L.W;
    f.G = (int)std::min<int64_t>(next_pow2(jb.L.W), 64);
    f.lgG = ilog2(f.G);
    f.B = jb.B;
    f.model = jb.model;
    f.one = jb.front(steps_run);
    f.two = jb.kind == kKindLT ? nullptr : jb.pl[2];
    if (jb.model == FSG_SIS || jb.model == FSG_SI || jb.model == FSG_SEIS) f.two = nullptr;
    f.three = jb.kind == kKindEpidemic ? jb.pl[3] : nullptr;
    f.states = final_states;
    f.counts = counts;
    f.bm = jb.front_bm(steps_run);
    if (jb.s.push) {  // the ever-active plane is nonzero only where the bitmap says so
        f.two_bm = jb.ever;
        f.scrub = (scrub && f.W == 1) ? 1 : 0;
    }
    return f;
}

int finalize_job(const Job &jb, int64_t steps_run, uint8_t *final_states, uint32_t *counts,
                 hipStream_t st, double *ms_out = nullptr, bool scrub = false)
{
    if (!final_states && !counts) return FSG_OK;
    const FinArgs f = fin_args(jb, steps_run, final_states, counts, scrub);
    EventPool ev;
    if (ms_out) {
        HIP_TRY(ev.init(2));
        HIP_TRY(hipEventRecord(ev.e[0], st));
    }
    HIP_TRY(launch_finalize(f, st));
    if (ms_out) HIP_TRY(hipEventRecord(ev.e[1], st));
    if (f.scrub) HIP_TRY(scrub_frontiers(jb, steps_run, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (ms_out) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
        *ms_out = ms;
    }
    return FSG_OK;
}

// Frontier-driven IC through fsg_simulate: the finalize, the clearing of the
// last two frontiers and the tag are queued right after the run's first
// chunk of steps, before the host reads the absorption flags; on the device
// they act only if the chunk ended the run (SpecFin), so the finalize follows
// the last step without a host round trip.  When they do not act, the finalize
// has still dispatched its whole grid (65-75 us at web scale), so later
// chunks are not followed by one: a run that outlives its first chunk pays
// that once and is finalized after the host has seen its end.  `done` tells
// the caller the outputs are written.
struct SpecOut {
    uint8_t *states = nullptr;
    uint32_t *counts = nullptr;
    bool done = false;
    double ms = 0.0;  // finalize kernel time (timed schedules)
    EventPool ev;
};

SpecFin spec_of(const Job &jb, int64_t t0, int64_t c)
{
    SpecFin sp;
    memset(&sp, 0, sizeof(sp));
    sp.flags = jb.a.flags;
    sp.ring = jb.ring;
    sp.c = (int32_t)c;
    sp.t0 = t0;
    for (int i = 0; i < 3; ++i) {  // front(t) and its bitmap and summary depend on t mod 3
        sp.front3[i] = jb.front(i);
        sp.bm3[i] = jb.front_bm(i);
        sp.sum3[i] = jb.front_sum(i);
    }
    for (int i = 0; i < 4; ++i) sp.queue4[i] = jb.queue[i];
    return sp;
}

hipError_t queue_spec_finalize(const Job &jb, int64_t t0, int64_t c, SpecOut &so, hipStream_t st)
{
    const SpecFin sp = spec_of(jb, t0, c);
    FinArgs f = fin_args(jb, t0 + 1, so.states, so.counts, true);
    f.spec = sp;
    if (jb.s.timed) {
        hipError_t e = hipEventRecord(so.ev.e[0], st);
        if (e != hipSuccess) return e;
    }
    hipError_t e = launch_finalize(f, st);
    if (e != hipSuccess) return e;
    if (jb.s.timed) {
        e = hipEventRecord(so.ev.e[1], st);
        if (e != hipSuccess) return e;
    }
    e = launch_ic_scrub_spec(jb.a, sp, 1, nullptr, 0ull, st);
    if (e != hipSuccess) return e;
    return launch_ic_scrub_spec(jb.a, sp, 2, jb.tag, jb.tag_value, st);
}

// A run in progress: the job on the caller's workspace, its schedule, and
// how far it has got.
struct Session {
    Job jb;
    int edge_grid = 0;
    int push_grid = 0;      // frontier-driven IC: grid of a chunk that starts with a push
    bool push_next = true;  // ... whether it does (the frontier's arcs at the last poll)
    int64_t steps_run = 0;  // steps executed so far
    bool absorbed = false;
    double kernel_ms = 0.0;
    int64_t timed_steps = 0;
    bool tail_on = false;                    // the last chunk ran in the tail mode
    int64_t tail_steps = 0;                  // live steps run in the tail mode
    int64_t infected_rows = -1;              // nodes with an infected replicate at the last poll
    double setup_ms = 0.0, finalize_ms = 0.0;
    EventPool setup_ev;  // around the set-up, read once the stream has passed them
    int64_t philox_calls = 0;
};

int begin_session(fsg_graph *g, const fsg_params *prm, const int32_t *seeds, int64_t n_seeds,
                  int64_t B, int64_t replicate_offset, uint64_t rng_key, const fsg_schedule *sched,
                  void *dev_ws, size_t ws_bytes, hipStream_t st, Session *ss)
{
    int rc = validate_run(g, prm, seeds, n_seeds, B, replicate_offset);
    if (rc) return rc;
    Sched s;
    rc = resolve_sched(g, prm, B, sched, &s);
    if (rc) return rc;
    const Plan &p = get_plan(g, s.heavy, s.tile_edges);
    Layout L;
    layout(g, prm, B, s, p, &L);
    if (!dev_ws || ws_bytes < L.total) return fail(FSG_EWORKSPACE, "simulation workspace too small");
    if (((uintptr_t)dev_ws & 255) != 0) return fail(FSG_EWORKSPACE, "workspace not 256-byte aligned");
    char *base = (char *)dev_ws;
    // timing events are read after the next synchronisation (run_steps)
    EventPool &ev = ss->setup_ev;
    if (s.timed) {
        HIP_TRY(ev.init(2));
        HIP_TRY(hipEventRecord(ev.e[0], st));
    }
    rc = setup_job(g, prm, seeds, n_seeds, B, replicate_offset, rng_key, s, p, L, base,
                   (uint32_t *)(base + L.flags), st, &ss->jb);
    if (rc) return rc;
    ss->setup_ms = 0.0;
    ss->finalize_ms = 0.0;
    if (s.timed) HIP_TRY(hipEventRecord(ev.e[1], st));
    ss->edge_grid = 0;
    if (s.edge1) {
        int dev = 0, ncu = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        // streaming: four times more blocks than fit at once (32 KB of LDS
        // each), so blocks that finish early are replaced, which evens out
        // the uneven work of frontier arcs (measured best on R-MAT scale 26 at
        // B = 64).  Pushing over a small frontier, the blocks beyond one
        // resident round only add dispatch time: R-MAT scale 26, 18 pushing
        // steps and 14 steps after absorption take 0.39 ms with 16 blocks per
        // CU, 0.24 ms with 2 or 4 (the streaming step slows 8% with 4)
        ss->edge_grid = 16 * std::max(ncu, 1);
        ss->push_grid = 4 * std::max(ncu, 1);
    }
    ss->push_next = true;  // the seeds' frontier is taken to be small
    ss->steps_run = 0;
    ss->absorbed = n_seeds == 0;
    ss->kernel_ms = 0.0;
    ss->timed_steps = 0;
    return FSG_OK;
}

// Tally arguments for the state after step `step` (0: the current state,
// no absorption check).
FinArgs tally_args(const Session &ss, unsigned long long *out, uint32_t step)
{
    const Job &jb = ss.jb;
    const int64_t t = step ? (int64_t)step : ss.steps_run;
    FinArgs f;
    memset(&f, 0, sizeof(f));
    f.n = (int32_t)jb.n;
    f.W = (int32_t)jb.L.W;
    f.B = jb.B;
    f.model = jb.model;
    f.one = jb.front(t);
    f.two = jb.kind == kKindLT ? nullptr : jb.pl[2];
    if (jb.model == FSG_SIS || jb.model == FSG_SI || jb.model == FSG_SEIS) f.two = nullptr;
    f.three = jb.kind == kKindEpidemic ? jb.pl[3] : nullptr;
    f.bm = jb.front_bm(t);
    f.tally = out;
    f.flags = step ? jb.a.flags : nullptr;
    f.ring = jb.ring;
    f.step = step;
    return f;
}

// The generator-call counter of a counting run into the session.
int read_draws(Session &ss, hipStream_t st)
{
    if (!ss.jb.a.draws) return FSG_OK;
    unsigned long long calls = 0;
    HIP_TRY(hipMemcpyAsync(&calls, ss.jb.a.draws, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    ss.philox_calls = (int64_t)calls;
    return FSG_OK;
}

void fill_info(const Session &ss, fsg_run_info *info)
{
    info->steps_run = ss.steps_run;
    info->absorbed = ss.absorbed ? 1 : 0;
    info->tail_steps = (int32_t)std::min<int64_t>(ss.tail_steps, INT32_MAX);
    info->step_kernel_ms = ss.kernel_ms;
    info->step_launches = ss.timed_steps;
    info->setup_ms = ss.setup_ms;
    info->finalize_ms = ss.finalize_ms;
    info->philox_calls = ss.philox_calls;
}

// Up to n_more further steps (never past the job's step cap), in chunks of
// Tail mode of the SI family: taken for a chunk when the nodes holding an
// infected replicate, times the mean in-degree, are at most this many times n.
constexpr double kTailFactor = 1.0;

// The set-up time of a timed session, once the stream has passed its events.
hipError_t take_setup_time(Session &ss)
{
    if (ss.setup_ev.e.size() != 2) return hipSuccess;
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, ss.setup_ev.e[0], ss.setup_ev.e[1]);
    if (e != hipSuccess) return e;
    ss.setup_ms = ms;
    ss.setup_ev.release();
    return hipSuccess;
}

// `sync` steps with one poll of the absorption flags per chunk.  With
// dev_tally, row i receives the state tally after the i-th step of this call.
int run_steps(Session &ss, int64_t n_more, uint64_t *dev_tally, hipStream_t st,
              SpecOut *so = nullptr)
{
    Job &jb = ss.jb;
    const Sched &s = jb.s;
    StepArgs &a = jb.a;
    const int kind = jb.kind;
    const int ring = jb.ring;
    uint32_t *flags = a.flags;
    const int64_t t_begin = ss.steps_run;
    const int64_t K = std::min<int64_t>(jb.K, t_begin + n_more);
    std::vector<uint32_t> hflags((size_t)ring);
    unsigned long long hqarcs = 0ull;  // frontier-driven IC: the last frontier's out-arcs
    EventPool ev;  // a pair per step, or one pair per chunk for the frontier-driven IC step
    if (s.timed) HIP_TRY(ev.init(s.push ? 2 : 2 * (size_t)s.sync));
    int64_t t = t_begin;
    std::vector<uint32_t> htail(2);
    while (!ss.absorbed && t < K) {
        const int64_t c = std::min<int64_t>(s.sync, K - t);
        HIP_TRY(launch_ring_clear(flags, ring, (int32_t)(t % ring), st, a.wflags, a.W, a.wring, t));
        if (jb.tail) {
            // tail mode for this chunk: when few nodes hold an infected
            // replicate (a row can only change if it or an in-neighbour
            // does); the stamps of steps t and t-1 are written on entry
            const double n = (double)jb.n, deg = (double)a.nnz / std::max(n, 1.0);
            const bool want = t >= 1 && (s.tail_always ||
                                         (ss.infected_rows >= 0 && (double)ss.infected_rows * deg <= n * kTailFactor));
            a.ibm_words = (int32_t)((jb.n + 31) / 32);
            uint32_t *cand = jb.ibm + 4 * (size_t)a.ibm_words;
            if (want && !ss.tail_on) {
                if (kind == kKindLT)
                    HIP_TRY(launch_mark_gained(a.stamp, jb.ibm, cand, a.ibm_words, jb.n,
                                               (uint32_t)(t + 1), st));
                else
                    HIP_TRY(launch_mark_rows(jb.front(t), jb.front(t + 1), jb.ibm, cand, a.ibm_words,
                                             jb.n, jb.L.W, (uint32_t)(t + 1), st));
            }
            ss.tail_on = want;
            a.ibm = want ? jb.ibm : nullptr;
            a.cand = want ? cand : nullptr;
        }
        for (int64_t i = 1; i <= c; ++i) {
            const int64_t step = t + i;
            a.step = (uint32_t)step;
            a.prev = jb.front(step - 1);
            a.next = jb.front(step);
            // timed: the dominant kernel of the step alone (the pull step,
            // without the bitmap clear or the heavy-row combine)
            if (s.push) {
                a.bm_prev = jb.front_bm(step - 1);
                a.bm_next = jb.front_bm(step);
                a.sum_prev = jb.front_sum(step - 1);
                a.sum_next = jb.front_sum(step);
                a.f_clr = jb.front(step - 2);
                a.bm_clr = jb.front_bm(step - 2);
                a.sum_clr = jb.front_sum(step - 2);
                a.qi_in = (int32_t)((step + 3) % 4);
                a.qi_out = (int32_t)(step % 4);
                a.qi_clr = (int32_t)((step + 2) % 4);
                a.qi_rst = (int32_t)((step + 1) % 4);
                a.q_in = jb.queue[a.qi_in];
                a.q_out = jb.queue[a.qi_out];
                a.q_clr = jb.queue[a.qi_clr];
                // one kernel a step, back to back: timed per chunk (events
                // between the launches would hold each one back)
                if (s.timed && i == 1) HIP_TRY(hipEventRecord(ev.e[0], st));
                HIP_TRY(launch_ic_front(a, ss.push_next ? ss.push_grid : ss.edge_grid, s.block, st));
                if (s.timed && i == c) HIP_TRY(hipEventRecord(ev.e[1], st));
            } else if (s.edge1) {
                a.bm_prev = jb.bm[(step - 1) & 1];
                a.bm_next = jb.bm[step & 1];
                a.sum_prev = jb.sum[(step - 1) & 1];
                a.sum_next = jb.sum[step & 1];
                HIP_TRY(launch_ic_clear(a, st));
                if (s.timed) HIP_TRY(hipEventRecord(ev.e[2 * (i - 1)], st));
                HIP_TRY(launch_ic_stream(a, ss.edge_grid, s.block, st));
                if (s.timed) HIP_TRY(hipEventRecord(ev.e[2 * (i - 1) + 1], st));
            } else {
                if (s.timed) HIP_TRY(hipEventRecord(ev.e[2 * (i - 1)], st));
                if (a.ibm) HIP_TRY(launch_tail_expand(a, st));
                HIP_TRY(launch_step(a, kind, jb.L.L, s.block, st));
                if (s.timed) HIP_TRY(hipEventRecord(ev.e[2 * (i - 1) + 1], st));
                if (a.n_heavy > 0) HIP_TRY(launch_combine(a, kind, s.block, st));
            }
            if (dev_tally) {
                FinArgs f = tally_args(ss, (unsigned long long *)dev_tally + 3 * (step - t_begin - 1),
                                       (uint32_t)step);
                HIP_TRY(launch_tally(f, st));
            }
        }
        const bool spec = so != nullptr && t == t_begin;  // the run's first chunk only
        if (spec) HIP_TRY(queue_spec_finalize(jb, t, c, *so, st));
        if (s.push)  // out-arcs of the frontier the next step starts from (queue of step t+c)
            HIP_TRY(hipMemcpyAsync(&hqarcs, a.qarcs + (t + c) % 4, 8, hipMemcpyDeviceToHost, st));
        if (jb.tail) {  // nodes with an infected replicate (LT: a new activation) after the chunk
            if (kind == kKindLT)
                HIP_TRY(launch_count_stamped(a.stamp, jb.n, (uint32_t)(t + c), jb.icount, st));
            else
                HIP_TRY(launch_count_rows(jb.front(t + c), jb.n, jb.L.W, jb.icount, st));
            HIP_TRY(hipMemcpyAsync(htail.data(), jb.icount, 8, hipMemcpyDeviceToHost, st));
        }
        HIP_TRY(hipMemcpyAsync(hflags.data(), flags, (size_t)ring * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(take_setup_time(ss));
        if (jb.tail) ss.infected_rows = (int64_t)((uint64_t)htail[0] | ((uint64_t)htail[1] << 32));
        if (s.push) ss.push_next = hqarcs <= a.push_limit;
        if (s.timed && s.push) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
            ss.kernel_ms += ms;
            ss.timed_steps += c;
        } else if (s.timed) {
            for (int64_t i = 1; i <= c; ++i) {
                // steps after absorption return at once; count only live ones
                if (i > 1 && hflags[(size_t)((t + i - 1) % ring)] == 0u) break;
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev.e[2 * (i - 1)], ev.e[2 * (i - 1) + 1]));
                ss.kernel_ms += ms;
                ++ss.timed_steps;
            }
        }
        ss.steps_run = t + c;
        for (int64_t i = 1; i <= c; ++i)
            if (hflags[(size_t)((t + i) % ring)] == 0u) {
                ss.steps_run = t + i;
                ss.absorbed = true;
                break;
            }
        if (spec && ss.absorbed) {  // the queued finalize acted (the same first clear flag)
            so->done = true;
            if (s.timed) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, so->ev.e[0], so->ev.e[1]));
                so->ms = ms;
            }
        }
        if (ss.tail_on) ss.tail_steps += ss.steps_run - t;
        t += c;
    }
    return FSG_OK;
}

}  // namespace

struct fsg_session {
    Session s;
};

extern "C" {

int fsg_abi_version(void) { return FSG_ABI_VERSION; }

const char *fsg_last_error(void) { return g_err.c_str(); }

int fsg_graph_create(int64_t n, int64_t nnz, const int64_t *in_ptr, const int32_t *in_src,
                     fsg_graph **out)
{
    try {
        if (!out) return fail(FSG_EINVAL, "out is NULL");
        *out = nullptr;
        if (n < 1) return fail(FSG_EINVAL, "n must be >= 1");
        if (n > 0x7FFFFFFF - 1) return fail(FSG_EUNSUPPORTED, "n above 2^31-2");
        if (nnz < 0) return fail(FSG_EINVAL, "nnz must be >= 0");
        if (nnz > kMaxNnz) return fail(FSG_EUNSUPPORTED, "nnz above 2^31 - 256");
        if (!in_ptr) return fail(FSG_EINVAL, "in_ptr is NULL");
        if (nnz > 0 && !in_src) return fail(FSG_EINVAL, "in_src is NULL");
        if (in_ptr[0] != 0) return fail(FSG_EINVAL, "in_ptr[0] must be 0");
        if (in_ptr[n] != nnz) return fail(FSG_EINVAL, "in_ptr[n] must equal nnz");
        int64_t dmax = 0;
        for (int64_t v = 0; v < n; ++v) {
            const int64_t d = in_ptr[v + 1] - in_ptr[v];
            if (d < 0) return fail(FSG_EINVAL, "in_ptr must be non-decreasing");
            dmax = std::max(dmax, d);
        }
        for (int64_t e = 0; e < nnz; ++e)
            if (in_src[e] < 0 || (int64_t)in_src[e] >= n)
                return fail(FSG_EINVAL, "in_src entry out of range at edge " + std::to_string(e));
        fsg::inject_alloc_fault();
        fsg_graph *g = new fsg_graph;
        g->n = n;
        g->nnz = nnz;
        g->max_indeg = dmax;
        g->ptr.assign(in_ptr, in_ptr + n + 1);
        for (int64_t v = 0; v < n; ++v)
            if (in_ptr[v + 1] - in_ptr[v] > kWideRow) g->wide.push_back((int32_t)v);
        // largest rows first: kernels that give each wide row its own block
        // then start the longest ones at the head of the grid
        std::stable_sort(g->wide.begin(), g->wide.end(), [&](int32_t a, int32_t b) {
            return in_ptr[a + 1] - in_ptr[a] > in_ptr[b + 1] - in_ptr[b];
        });
        g->src_host = in_src;
        *out = g;
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(FSG_EINVAL, "unexpected host exception");
    }
}

int fsg_graph_workspace_size(const fsg_graph *g, size_t *bytes)
{
    if (!g || !bytes) return fail(FSG_EINVAL, "NULL argument");
    // sources are padded by 16 bytes: kernels read them with 16-byte loads;
    // then the target row of every arc
    *bytes = align256((size_t)(g->n + 1) * 4) + align256((size_t)std::max<int64_t>(g->nnz, 1) * 4 + 16) +
             align256((size_t)std::max<int64_t>(g->nnz, 1) * 4) + align256((g->wide.size() + 1) * 4);
    return FSG_OK;
}

int fsg_graph_bind(fsg_graph *g, void *dev_ws, size_t ws_bytes, void *stream)
{
    try {
        if (!g) return fail(FSG_EINVAL, "graph is NULL");
        size_t need = 0;
        fsg_graph_workspace_size(g, &need);
        if (!dev_ws || ws_bytes < need) return fail(FSG_EWORKSPACE, "graph workspace too small");
        if (((uintptr_t)dev_ws & 255) != 0) return fail(FSG_EWORKSPACE, "workspace not 256-byte aligned");
        if (g->nnz > 0 && !g->src_host) return fail(FSG_EINVAL, "graph already bound; sources released");
        hipStream_t s = (hipStream_t)stream;
        char *base = (char *)dev_ws;
        int32_t *dptr = (int32_t *)base;
        int32_t *dsrc = (int32_t *)(base + align256((size_t)(g->n + 1) * 4));
        int32_t *ddst = (int32_t *)((char *)dsrc + align256((size_t)std::max<int64_t>(g->nnz, 1) * 4 + 16));
        int32_t *dwide = (int32_t *)((char *)ddst + align256((size_t)std::max<int64_t>(g->nnz, 1) * 4));
        if (!g->wide.empty())
            HIP_TRY(hipMemcpyAsync(dwide, g->wide.data(), g->wide.size() * 4, hipMemcpyHostToDevice, s));
        std::vector<int32_t> p32(g->ptr.begin(), g->ptr.end());
        HIP_TRY(hipMemcpyAsync(dptr, p32.data(), p32.size() * 4, hipMemcpyHostToDevice, s));
        if (g->nnz > 0)
            HIP_TRY(hipMemcpyAsync(dsrc, g->src_host, (size_t)g->nnz * 4, hipMemcpyHostToDevice, s));
        if (g->nnz > 0) HIP_TRY(launch_expand_rows(dptr, g->n, ddst, s));
        HIP_TRY(hipStreamSynchronize(s));
        g->d_ptr = dptr;
        g->d_src = dsrc;
        g->d_dst = ddst;
        g->d_wide = dwide;
        g->bound = true;
        g->src_host = nullptr;
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

namespace {
struct OutLayout {
    size_t optr, oarc, cursor, total;
};
OutLayout out_layout(const fsg_graph *g)
{
    OutLayout o;
    size_t off = 0;
    o.optr = off; off = align256(off + (size_t)(g->n + 1) * 4);
    o.oarc = off; off = align256(off + (size_t)std::max<int64_t>(g->nnz, 1) * 8);
    o.cursor = off; off = align256(off + (size_t)g->n * 4);
    o.total = off;
    return o;
}
}  // namespace

int fsg_graph_out_workspace_size(const fsg_graph *g, size_t *bytes)
{
    if (!g || !bytes) return fail(FSG_EINVAL, "NULL argument");
    *bytes = out_layout(g).total;
    return FSG_OK;
}

int fsg_graph_bind_out(fsg_graph *g, void *dev_ws, size_t ws_bytes, void *stream)
{
    try {
        if (!g) return fail(FSG_EINVAL, "graph is NULL");
        if (!g->bound) return fail(FSG_EINVAL, "graph is not bound to device memory");
        const OutLayout o = out_layout(g);
        if (!dev_ws || ws_bytes < o.total) return fail(FSG_EWORKSPACE, "out-adjacency workspace too small");
        if (((uintptr_t)dev_ws & 255) != 0) return fail(FSG_EWORKSPACE, "workspace not 256-byte aligned");
        hipStream_t s = (hipStream_t)stream;
        char *base = (char *)dev_ws;
        int32_t *optr = (int32_t *)(base + o.optr);
        int2 *oarc = (int2 *)(base + o.oarc);
        int32_t *cursor = (int32_t *)(base + o.cursor);
        const int64_t n = g->n;
        // out-degrees on the device, prefix sums on the host
        HIP_TRY(launch_fill32((uint32_t *)cursor, n, 0u, s));
        HIP_TRY(launch_out_count(g->d_src, g->nnz, cursor, s));
        std::vector<int32_t> deg((size_t)n), p32((size_t)n + 1);
        HIP_TRY(hipMemcpyAsync(deg.data(), cursor, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        int64_t acc = 0, items = 0;
        for (int64_t u = 0; u < n; ++u) {
            p32[(size_t)u] = (int32_t)acc;
            acc += deg[(size_t)u];
            items += deg[(size_t)u] > kOutChunk ? (deg[(size_t)u] + kOutChunk - 1) / kOutChunk : 1;
        }
        p32[(size_t)n] = (int32_t)acc;
        if (acc != g->nnz) return fail(FSG_EDEVICE, "out-degree count does not add up to nnz");
        HIP_TRY(hipMemcpyAsync(optr, p32.data(), p32.size() * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(cursor, p32.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_out_fill(g->d_src, g->d_dst, g->nnz, cursor, oarc, s));
        HIP_TRY(hipStreamSynchronize(s));
        g->d_optr = optr;
        g->d_oarc = oarc;
        g->out_items = items;
        g->has_out = true;
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_graph_stats(const fsg_graph *g, int64_t *n, int64_t *nnz, int64_t *max_indeg)
{
    if (!g) return fail(FSG_EINVAL, "graph is NULL");
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (max_indeg) *max_indeg = g->max_indeg;
    return FSG_OK;
}

int fsg_graph_destroy(fsg_graph *g)
{
    delete g;
    return FSG_OK;
}

int fsg_default_schedule(const fsg_graph *g, const fsg_params *prm, int64_t B, fsg_schedule *out)
{
    if (!out) return fail(FSG_EINVAL, "out is NULL");
    int rc = check_params(g, prm, B);
    if (rc) return rc;
    default_sched(g, prm, B, out);
    return FSG_OK;
}

int fsg_sim_workspace_size(const fsg_graph *g_, const fsg_params *prm, int64_t B,
                           const fsg_schedule *sched, size_t *bytes)
{
    try {
        if (!bytes) return fail(FSG_EINVAL, "bytes is NULL");
        int rc = check_params(g_, prm, B);
        if (rc) return rc;
        fsg_graph *g = const_cast<fsg_graph *>(g_);
        Sched s;
        rc = resolve_sched(g, prm, B, sched, &s);
        if (rc) return rc;
        const Plan &p = get_plan(g, s.heavy, s.tile_edges);
        Layout L;
        layout(g, prm, B, s, p, &L);
        *bytes = L.total;
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_simulate(const fsg_graph *g_, const fsg_params *prm, const int32_t *seeds, int64_t n_seeds,
                 int64_t B, int64_t replicate_offset, uint64_t rng_key, const fsg_schedule *sched,
                 void *dev_ws, size_t ws_bytes, uint8_t *final_states, uint32_t *infected_counts,
                 fsg_run_info *info, void *stream)
{
    try {
        Session ss;
        int rc = begin_session(const_cast<fsg_graph *>(g_), prm, seeds, n_seeds, B,
                               replicate_offset, rng_key, sched, dev_ws, ws_bytes,
                               (hipStream_t)stream, &ss);
        if (rc) return rc;
        const bool scrub = ss.jb.s.push && (final_states || infected_counts);
        SpecOut so;
        if (scrub) {  // frontier-driven IC: the finalize goes in right behind the steps
            so.states = final_states;
            so.counts = infected_counts;
            if (ss.jb.s.timed) HIP_TRY(so.ev.init(2));
        }
        rc = run_steps(ss, ss.jb.K, nullptr, (hipStream_t)stream, scrub ? &so : nullptr);
        if (rc) return rc;
        if (so.done) {
            ss.finalize_ms = so.ms;
        } else {  // the run outlived its first chunk, stopped at its step cap, or has no seeds
            rc = finalize_job(ss.jb, ss.steps_run, final_states, infected_counts, (hipStream_t)stream,
                              ss.jb.s.timed ? &ss.finalize_ms : nullptr, scrub);
            if (rc) return rc;
        }
        HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
        HIP_TRY(take_setup_time(ss));
        rc = read_draws(ss, (hipStream_t)stream);
        if (rc) return rc;
        if (info) fill_info(ss, info);
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_session_begin(const fsg_graph *g, const fsg_params *prm, const int32_t *seeds,
                      int64_t n_seeds, int64_t B, int64_t replicate_offset, uint64_t rng_key,
                      const fsg_schedule *sched, void *dev_ws, size_t ws_bytes, void *stream,
                      fsg_session **out)
{
    try {
        if (!out) return fail(FSG_EINVAL, "out is NULL");
        *out = nullptr;
        std::unique_ptr<fsg_session> ss(new fsg_session);
        int rc = begin_session(const_cast<fsg_graph *>(g), prm, seeds, n_seeds, B, replicate_offset,
                               rng_key, sched, dev_ws, ws_bytes, (hipStream_t)stream, &ss->s);
        if (rc) return rc;
        *out = ss.release();
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_session_step(fsg_session *ss, int64_t n_steps, uint64_t *dev_tally, fsg_run_info *info,
                     void *stream)
{
    try {
        if (!ss) return fail(FSG_EINVAL, "session is NULL");
        if (n_steps < 0) return fail(FSG_EINVAL, "n_steps must be >= 0");
        Session &s = ss->s;
        const hipStream_t st = (hipStream_t)stream;
        const int64_t t0 = s.steps_run;
        int rc = run_steps(s, n_steps, dev_tally, st);
        if (rc) return rc;
        if (dev_tally) {
            // rows of steps that were not run (absorbed, or past max_steps)
            // repeat the final state's tally
            for (int64_t i = s.steps_run - t0; i < n_steps; ++i) {
                FinArgs f = tally_args(s, (unsigned long long *)dev_tally + 3 * i, 0u);
                HIP_TRY(launch_tally(f, st));
            }
            HIP_TRY(hipStreamSynchronize(st));
        }
        rc = read_draws(s, st);
        if (rc) return rc;
        if (info) fill_info(s, info);
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_session_read(fsg_session *ss, uint8_t *states, uint32_t *counts, uint64_t *dev_tally,
                     void *stream)
{
    if (!ss) return fail(FSG_EINVAL, "session is NULL");
    const Session &s = ss->s;
    const hipStream_t st = (hipStream_t)stream;
    int rc = finalize_job(s.jb, s.steps_run, states, counts, st);
    if (rc) return rc;
    if (dev_tally) {
        FinArgs f = tally_args(s, (unsigned long long *)dev_tally, 0u);
        HIP_TRY(launch_tally(f, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return FSG_OK;
}

int fsg_session_end(fsg_session *ss)
{
    delete ss;
    return FSG_OK;
}

}  // extern "C"

// ---- fsg_simulate without a caller workspace: the workspace is a static
// device array of kScratchBytes, one per GPU, held until the process ends.
namespace {
constexpr size_t kScratchBytes = (size_t)64 << 20;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_at;  // device -> address of that device's copy of scratch

// Device address of the current device's copy of scratch, looked up once per
// device (the host-side name of the array is not a device address).
int scratch_address(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_at.find(dev);
    if (it == g_scratch_at.end()) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255) != 0) return fail(FSG_EDEVICE, "scratch array misplaced");
        it = g_scratch_at.emplace(dev, p).first;
    }
    *out = it->second;
    return FSG_OK;
}

}  // namespace

extern "C" {

size_t fsg_simulate_noalloc_limit(void) { return kScratchBytes; }

int fsg_simulate_noalloc(const fsg_graph *g, const fsg_params *prm, const int32_t *seeds,
                         int64_t n_seeds, int64_t B, int64_t replicate_offset, uint64_t rng_key,
                         const fsg_schedule *sched, uint8_t *final_states,
                         uint32_t *infected_counts, fsg_run_info *info, void *stream)
{
    try {
        fsg_schedule s;
        if (sched) {
            s = *sched;
        } else {
            memset(&s, 0, sizeof(s));
        }
        s.time_kernels = 0;  // no HIP events
        size_t need = 0;
        int rc = fsg_sim_workspace_size(g, prm, B, &s, &need);
        if (rc) return rc;
        if (need > kScratchBytes)
            return fail(FSG_EWORKSPACE, "this run needs " + std::to_string(need) +
                                            " bytes of workspace; the static scratch holds " +
                                            std::to_string(kScratchBytes));
        void *ws = nullptr;
        rc = scratch_address(&ws);
        if (rc) return rc;
        return fsg_simulate(g, prm, seeds, n_seeds, B, replicate_offset, rng_key, &s, ws,
                            kScratchBytes, final_states, infected_counts, info, stream);
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_philox4x32_10(const uint32_t *dev_ctr, uint32_t key0, uint32_t key1, uint32_t *dev_out,
                      int64_t count, void *stream)
{
    if (count < 0 || (count > 0 && (!dev_ctr || !dev_out)))
        return fail(FSG_EINVAL, "bad philox arguments");
    HIP_TRY(launch_philox(dev_ctr, key0, key1, dev_out, count, (hipStream_t)stream));
    return FSG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

struct fsg_plan {
    std::vector<fsg_job> jobs;
    std::vector<Sched> sched;
    std::vector<const Plan *> plans;
    std::vector<Layout> layouts;
    std::vector<size_t> job_off;  // workspace offset of each job
    size_t ctl_off = 0, total = 0;
    int sync = 16;
    int blocks_per_cu = 4;  // persistent blocks of the batched kernels per compute unit
};

namespace {

// Defaults of a job in the batched launch: larger tiles and a higher heavy
// cut than a job alone, since the other jobs already fill the GPU (the batch
// autotuner chose both for every model class of the 64-job mixed batch).
constexpr int32_t kBatchTileEdges = 8192;
constexpr int32_t kBatchHeavy = 2048;

int resolve_batch_sched(const fsg_job &j, Sched *s)
{
    fsg_schedule u = j.sched;
    if (u.kernel_variant >= 2) return fail(FSG_EINVAL, "batched jobs use kernel_variant 0 or 1");
    u.kernel_variant = 1;
    u.block_threads = kBatchBlock;
    if (u.tile_edges == 0) u.tile_edges = kBatchTileEdges;
    if (u.heavy_threshold == 0) u.heavy_threshold = kBatchHeavy;
    return resolve_sched(j.g, &j.prm, j.B, &u, s);
}

}  // namespace

extern "C" {

int fsg_batch_plan(const fsg_job *jobs, int32_t n_jobs, int32_t steps_per_sync, fsg_plan **out,
                   size_t *ws_bytes)
{
    try {
        if (!out || !ws_bytes) return fail(FSG_EINVAL, "NULL output");
        *out = nullptr;
        if (!jobs || n_jobs < 1 || n_jobs > kMaxBatchJobs)
            return fail(FSG_EINVAL, "n_jobs must be in [1, 1024]");
        if (steps_per_sync < 1 || steps_per_sync > 4096)
            return fail(FSG_EINVAL, "steps_per_sync must be in [1, 4096]");
        fsg::inject_alloc_fault();
        std::unique_ptr<fsg_plan> pl(new fsg_plan);
        pl->sync = steps_per_sync;
        size_t off = 0;
        for (int32_t i = 0; i < n_jobs; ++i) {
            const fsg_job &j = jobs[i];
            fsg_graph *g = const_cast<fsg_graph *>(j.g);
            int rc = validate_run(g, &j.prm, j.seeds, j.n_seeds, j.B, j.replicate_offset);
            if (rc) return fail(rc, "job " + std::to_string(i) + ": " + g_err);
            Sched s;
            rc = resolve_batch_sched(j, &s);
            if (rc) return fail(rc, "job " + std::to_string(i) + ": " + g_err);
            s.sync = steps_per_sync;
            const Plan &p = get_plan(g, s.heavy, s.tile_edges);
            Layout L;
            layout(g, &j.prm, j.B, s, p, &L);
            pl->jobs.push_back(j);
            pl->sched.push_back(s);
            pl->plans.push_back(&p);
            pl->layouts.push_back(L);
            pl->job_off.push_back(off);
            off = align256(off + L.total);
        }
        pl->ctl_off = off;
        const size_t n = (size_t)n_jobs, ring = (size_t)steps_per_sync + 1;
        off = align256(off + n * sizeof(StepArgs));       // job table
        off = align256(off + (n + 1) * 4 * 2 + n * 4 * 2);  // item_off, comb_off, code, max_step
        off = align256(off + 16);                           // queue[2], cur_step
        off = align256(off + n * ring * 4);                 // flag rings
        off = align256(off + (n + 2 * (n + 1)) * 4);        // tail_on, word_off, row_off
        off = align256(off + n * 8);                        // per-job counts (tail mode)
        pl->total = off;
        *ws_bytes = off;
        *out = pl.release();
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_batch_set_launch(fsg_plan *plan, int32_t blocks_per_cu)
{
    if (!plan) return fail(FSG_EINVAL, "plan is NULL");
    if (blocks_per_cu < 1 || blocks_per_cu > 32)
        return fail(FSG_EINVAL, "blocks_per_cu must be in [1, 32]");
    plan->blocks_per_cu = blocks_per_cu;
    return FSG_OK;
}

int fsg_plan_destroy(fsg_plan *plan)
{
    delete plan;
    return FSG_OK;
}

int fsg_batch_run(fsg_plan *pl, void *dev_ws, size_t ws_bytes, fsg_run_info *infos,
                  double *total_ms, void *stream)
{
    try {
        if (!pl) return fail(FSG_EINVAL, "plan is NULL");
        if (!dev_ws || ws_bytes < pl->total) return fail(FSG_EWORKSPACE, "batch workspace too small");
        if (((uintptr_t)dev_ws & 255) != 0) return fail(FSG_EWORKSPACE, "workspace not 256-byte aligned");
        hipStream_t st = (hipStream_t)stream;
        char *base = (char *)dev_ws;
        const int n = (int)pl->jobs.size();
        const int ring = pl->sync + 1;
        // control area
        char *ctl = base + pl->ctl_off;
        StepArgs *d_jobs = (StepArgs *)ctl;
        char *q = ctl + align256((size_t)n * sizeof(StepArgs));
        int32_t *d_item_off = (int32_t *)q;
        int32_t *d_comb_off = d_item_off + (n + 1);
        int32_t *d_code = d_comb_off + (n + 1);
        int32_t *d_max_step = d_code + n;
        q += align256((size_t)(n + 1) * 4 * 2 + (size_t)n * 4 * 2);
        uint32_t *d_queue = (uint32_t *)q;
        uint32_t *d_step = d_queue + 2;
        q += align256(16);
        uint32_t *d_flags = (uint32_t *)q;
        q += align256((size_t)n * ring * 4);
        int32_t *d_tail_on = (int32_t *)q;
        int32_t *d_word_off = d_tail_on + n;
        int32_t *d_row_off = d_word_off + (n + 1);
        q += align256((size_t)(n + 2 * (n + 1)) * 4);
        unsigned long long *d_counts = (unsigned long long *)q;

        std::vector<Job> jb((size_t)n);
        std::vector<StepArgs> h_jobs((size_t)n);
        std::vector<int32_t> item_off((size_t)n + 1, 0), comb_off((size_t)n + 1, 0),
            code((size_t)n), max_step((size_t)n), word_off((size_t)n + 1, 0),
            row_off((size_t)n + 1, 0), tail_on((size_t)n, 0);
        bool any_heavy = false, any_tail = false;
        for (int i = 0; i < n; ++i) {
            const fsg_job &j = pl->jobs[(size_t)i];
            fsg_graph *g = const_cast<fsg_graph *>(j.g);
            int rc = setup_job(g, &j.prm, j.seeds, j.n_seeds, j.B, j.replicate_offset, j.rng_key,
                               pl->sched[(size_t)i], *pl->plans[(size_t)i], pl->layouts[(size_t)i],
                               base + pl->job_off[(size_t)i], d_flags + (size_t)i * ring, st,
                               &jb[(size_t)i]);
            if (rc) return rc;
            StepArgs &a = jb[(size_t)i].a;
            if (jb[(size_t)i].tail) {  // the tail mode's bitmaps (used while tail_on)
                a.ibm_words = (int32_t)((a.n + 31) / 32);
                a.ibm = jb[(size_t)i].ibm;
                a.cand = jb[(size_t)i].ibm + 4 * (size_t)a.ibm_words;
                any_tail = true;
            }
            word_off[(size_t)i + 1] = word_off[(size_t)i] + (jb[(size_t)i].tail ? a.ibm_words : 0);
            row_off[(size_t)i + 1] = row_off[(size_t)i] + (jb[(size_t)i].tail ? a.n : 0);
            h_jobs[(size_t)i] = a;  // prev/next hold planes 0 and 1
            item_off[(size_t)i + 1] = item_off[(size_t)i] + step_blocks(a, kBatchBlock);
            const int rows_per_combine = (kBatchBlock / 64) * combine_rows_per_wave(a.lgG);
            comb_off[(size_t)i + 1] =
                comb_off[(size_t)i] + (a.n_heavy + rows_per_combine - 1) / rows_per_combine;
            any_heavy |= a.n_heavy > 0;
            code[(size_t)i] = jb[(size_t)i].kind * 32 + (jb[(size_t)i].kind == kKindIC ? 1 : a.Lp);
            max_step[(size_t)i] = (int32_t)std::min<int64_t>(jb[(size_t)i].K, 0x7FFFFFFF);
        }
        HIP_TRY(hipMemcpyAsync(d_jobs, h_jobs.data(), (size_t)n * sizeof(StepArgs), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_item_off, item_off.data(), item_off.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_comb_off, comb_off.data(), comb_off.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_code, code.data(), code.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_max_step, max_step.data(), max_step.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_word_off, word_off.data(), word_off.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_row_off, row_off.data(), row_off.size() * 4, hipMemcpyHostToDevice, st));
        HIP_TRY(launch_fill32((uint32_t *)d_tail_on, n, 0u, st));
        HIP_TRY(launch_fill32(d_queue, 2, 0u, st));
        HIP_TRY(launch_fill32(d_step, 1, 1u, st));
        HIP_TRY(hipStreamSynchronize(st));

        BatchCtl c;
        c.jobs = d_jobs;
        c.item_off = d_item_off;
        c.comb_off = d_comb_off;
        c.code = d_code;
        c.max_step = d_max_step;
        c.n_jobs = n;
        c.ring = ring;
        c.queue = d_queue;
        c.cur_step = d_step;
        c.tail_on = d_tail_on;
        c.word_off = d_word_off;
        c.row_off = d_row_off;
        int dev = 0, ncu = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        const int grid =
            std::max(1, std::min(pl->blocks_per_cu * std::max(ncu, 1), item_off[(size_t)n]));
        const int cgrid = std::max(1, std::min(2 * std::max(ncu, 1), comb_off[(size_t)n]));

        // capture one chunk of steps in a graph on a private stream
        struct Cap {
            hipStream_t s = nullptr;
            hipGraph_t g = nullptr;
            hipGraphExec_t e = nullptr;
            ~Cap()
            {
                if (e) (void)hipGraphExecDestroy(e);
                if (g) (void)hipGraphDestroy(g);
                if (s) (void)hipStreamDestroy(s);
            }
        } cap;
        HIP_TRY(hipStreamCreateWithFlags(&cap.s, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(cap.s, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < pl->sync; ++i) {
            if (any_tail) {
                hipError_t e0 = launch_batch_expand(c, cap.s);
                if (e0 != hipSuccess) {
                    hipGraph_t dummy = nullptr;
                    (void)hipStreamEndCapture(cap.s, &dummy);
                    if (dummy) (void)hipGraphDestroy(dummy);
                    return fail(FSG_EDEVICE, std::string("batched launch capture failed: ") +
                                                 hipGetErrorString(e0));
                }
            }
            hipError_t e1 = launch_batch_step(c, grid, cap.s);
            hipError_t e2 = any_heavy ? launch_batch_combine(c, cgrid, cap.s) : hipSuccess;
            hipError_t e3 = launch_batch_advance(c, cap.s);
            if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
                hipGraph_t dummy = nullptr;
                (void)hipStreamEndCapture(cap.s, &dummy);
                if (dummy) (void)hipGraphDestroy(dummy);
                return fail(FSG_EDEVICE, std::string("batched launch capture failed: ") +
                                             hipGetErrorString(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3)));
            }
        }
        HIP_TRY(hipStreamEndCapture(cap.s, &cap.g));
        HIP_TRY(hipGraphInstantiate(&cap.e, cap.g, nullptr, nullptr, 0));

        std::vector<uint32_t> hf((size_t)n * ring);
        std::vector<int64_t> steps_run((size_t)n, 0);
        std::vector<int> done((size_t)n, 0), absorbed((size_t)n, 0);
        int remaining = 0;
        for (int i = 0; i < n; ++i) {
            const fsg_job &j = pl->jobs[(size_t)i];
            if (j.n_seeds == 0 || jb[(size_t)i].K == 0) {
                done[(size_t)i] = 1;
                absorbed[(size_t)i] = j.n_seeds == 0;
            } else {
                ++remaining;
            }
        }
        EventPool ev;
        HIP_TRY(ev.init(2));
        double kernel_ms = 0.0;
        int64_t t0 = 0;
        // tail mode per job: nodes with an infected replicate (LT: a new
        // activation) at the last poll, -1 before the first
        std::vector<int64_t> icount((size_t)n, -1), tail_steps((size_t)n, 0);
        std::vector<unsigned long long> hcount((size_t)n, 0);
        while (remaining > 0) {
            if (any_tail) {
                bool changed = false;
                for (int i = 0; i < n; ++i) {
                    const Job &J = jb[(size_t)i];
                    if (!J.tail || done[(size_t)i]) continue;
                    const double nn = (double)J.n, deg = (double)J.a.nnz / std::max(nn, 1.0);
                    const bool want = t0 >= 1 && (pl->sched[(size_t)i].tail_always ||
                                                  (icount[(size_t)i] >= 0 &&
                                                   (double)icount[(size_t)i] * deg <= nn * kTailFactor));
                    if (want && !tail_on[(size_t)i]) {  // the bitmaps of steps t0 and t0-1
                        const StepArgs &a = h_jobs[(size_t)i];
                        const uint32_t t = (uint32_t)(t0 + 1);
                        if (J.kind == kKindLT) {
                            HIP_TRY(launch_mark_gained(a.stamp, a.ibm, a.cand, a.ibm_words, a.n, t, st));
                        } else {
                            // base planes: prev holds odd steps' inputs (state of even steps)
                            const uint64_t *p0 = a.prev, *p1 = a.next;
                            const uint64_t *cur = (t & 1u) ? p0 : p1, *old = (t & 1u) ? p1 : p0;
                            HIP_TRY(launch_mark_rows(cur, old, a.ibm, a.cand, a.ibm_words, a.n, a.W, t,
                                                     st));
                        }
                    }
                    if (want != (tail_on[(size_t)i] != 0)) changed = true;
                    tail_on[(size_t)i] = want ? 1 : 0;
                }
                if (changed)
                    HIP_TRY(hipMemcpyAsync(d_tail_on, tail_on.data(), (size_t)n * 4,
                                           hipMemcpyHostToDevice, st));
            }
            HIP_TRY(hipEventRecord(ev.e[0], st));
            HIP_TRY(hipGraphLaunch(cap.e, st));
            HIP_TRY(hipEventRecord(ev.e[1], st));
            if (any_tail) {
                HIP_TRY(launch_fill64((uint64_t *)d_counts, n, 0ull, st));
                HIP_TRY(launch_batch_count(c, (uint32_t)(t0 + pl->sync), d_counts, st));
                HIP_TRY(hipMemcpyAsync(hcount.data(), d_counts, (size_t)n * 8, hipMemcpyDeviceToHost, st));
            }
            HIP_TRY(hipMemcpyAsync(hf.data(), d_flags, hf.size() * 4, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (any_tail)
                for (int i = 0; i < n; ++i) icount[(size_t)i] = (int64_t)hcount[(size_t)i];
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev.e[0], ev.e[1]));
            kernel_ms += ms;
            for (int i = 0; i < n; ++i) {
                if (done[(size_t)i]) continue;
                const uint32_t *f = hf.data() + (size_t)i * ring;
                for (int k = 1; k <= pl->sync; ++k) {
                    const int64_t t = t0 + k;
                    if (f[t % ring] == 0u) {
                        done[(size_t)i] = 1;
                        absorbed[(size_t)i] = 1;
                        steps_run[(size_t)i] = t;
                        break;
                    }
                    if (t == jb[(size_t)i].K) {
                        done[(size_t)i] = 1;
                        steps_run[(size_t)i] = t;
                        break;
                    }
                }
                if (tail_on[(size_t)i])
                    tail_steps[(size_t)i] += (done[(size_t)i] ? steps_run[(size_t)i] : t0 + pl->sync) - t0;
                if (done[(size_t)i]) --remaining;
            }
            t0 += pl->sync;
        }
        for (int i = 0; i < n; ++i) {
            const fsg_job &j = pl->jobs[(size_t)i];
            int rc = finalize_job(jb[(size_t)i], steps_run[(size_t)i], j.final_states,
                                  j.infected_counts, st);
            if (rc) return rc;
            if (infos) {
                infos[i].steps_run = steps_run[(size_t)i];
                infos[i].absorbed = absorbed[(size_t)i];
                infos[i].tail_steps = (int32_t)std::min<int64_t>(tail_steps[(size_t)i], INT32_MAX);
                infos[i].step_kernel_ms = 0.0;
                infos[i].step_launches = 0;
                infos[i].setup_ms = 0.0;
                infos[i].finalize_ms = 0.0;
                infos[i].philox_calls = 0;
            }
        }
        if (total_ms) *total_ms = kernel_ms;
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

}  // extern "C"

// --------------------------------------------------------------- autotuner

namespace {

std::vector<fsg_schedule> candidates(const fsg_graph *g, const fsg_params *prm, int64_t B,
                                     bool batch_only)
{
    std::vector<fsg_schedule> out;
    const int64_t W = (B + 63) / 64;
    const int gmax = (int)std::min<int64_t>(next_pow2(W), 64);
    auto add = [&](int lanes, int block, int tile, int heavy, int variant) {
        fsg_schedule s;
        memset(&s, 0, sizeof(s));
        s.row_lanes = lanes;
        s.block_threads = block;
        s.tile_edges = tile;
        s.heavy_threshold = heavy;
        s.steps_per_sync = 16;
        s.kernel_variant = variant;
        out.push_back(s);
    };
    if (!batch_only && prm->model == FSG_IC && W == 1) {
        if (g->has_out) add(16, 512, 16384, 32768, 3);
        for (int block : {256, 512, 1024})
            for (int tile : {8192, 16384, 32768})
                for (int heavy : {8192, 32768}) add(16, block, tile, heavy, 2);
    }
    std::vector<int> lanes;
    for (int l = gmax; l <= 64; l *= 2) lanes.push_back(l);
    if (gmax < 16 && std::find(lanes.begin(), lanes.end(), 16) == lanes.end()) lanes.push_back(16);
    for (int l : lanes)
        for (int block : batch_only ? std::vector<int>{kBatchBlock} : std::vector<int>{256, 512})
            for (int tile : {2048, 4096, 16384})
                for (int heavy : {512, 1024, 4096}) add(l, block, tile, heavy, 1);
    return out;
}

std::string tune_key(const fsg_graph *g, const fsg_params *prm, int64_t B, bool batch_only)
{
    std::ostringstream k;
    k << "n=" << g->n << ",nnz=" << g->nnz << ",dmax=" << g->max_indeg << ",model=" << prm->model
      << ",icp=" << prm->ic_prob << ",B=" << B << ",batch=" << (batch_only ? 1 : 0)
      << ",out=" << (g->has_out ? 1 : 0);
    return k.str();
}

bool cache_lookup(const char *path, const std::string &key, fsg_schedule *out, double *ms)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        fsg_schedule s;
        memset(&s, 0, sizeof(s));
        double m = 0;
        if (!(is >> k >> s.row_lanes >> s.block_threads >> s.tile_edges >> s.heavy_threshold >>
              s.steps_per_sync >> s.kernel_variant >> m))
            continue;
        if (k == key) {  // the last entry for a key wins
            *out = s;
            *ms = m;
            found = true;
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, const fsg_schedule &s, double ms)
{
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << s.row_lanes << " " << s.block_threads << " " << s.tile_edges << " "
      << s.heavy_threshold << " " << s.steps_per_sync << " " << s.kernel_variant << " " << ms
      << "\n";
}

}  // namespace

extern "C" {

int fsg_autotune_workspace_size(const fsg_graph *g_, const fsg_params *prm, int64_t B,
                                int32_t batch_only, size_t *bytes)
{
    try {
        if (!bytes) return fail(FSG_EINVAL, "bytes is NULL");
        int rc = check_params(g_, prm, B);
        if (rc) return rc;
        size_t best = 0;
        fsg_schedule d;
        default_sched(g_, prm, B, &d);
        std::vector<fsg_schedule> cs = candidates(g_, prm, B, batch_only != 0);
        cs.push_back(d);
        for (fsg_schedule s : cs) {
            s.steps_per_sync = 64;  // the longest poll interval fsg_autotune uses
            size_t b = 0;
            rc = fsg_sim_workspace_size(g_, prm, B, &s, &b);
            if (rc) return rc;
            best = std::max(best, b);
        }
        *bytes = best;
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_autotune(const fsg_graph *g, const fsg_params *prm, const int32_t *seeds, int64_t n_seeds,
                 int64_t B, uint64_t rng_key, int32_t tune_steps, int32_t batch_only,
                 const char *cache_path, void *dev_ws, size_t ws_bytes, fsg_schedule *best,
                 double *best_ms, double *default_ms, void *stream)
{
    try {
        if (!best) return fail(FSG_EINVAL, "best is NULL");
        if (tune_steps < 1) return fail(FSG_EINVAL, "tune_steps must be >= 1");
        int rc = check_params(g, prm, B);
        if (rc) return rc;
        const std::string key = tune_key(g, prm, B, batch_only != 0);
        double cached_ms = 0;
        if (cache_lookup(cache_path, key, best, &cached_ms)) {
            if (best_ms) *best_ms = cached_ms;
            if (default_ms) *default_ms = -1.0;
            return FSG_OK;
        }
        // Objective: device time of whole steps (pull step, heavy-row merge
        // and frontier clear), from runs of K and 2K steps timed with HIP
        // events on the stream; their difference leaves out the set-up.
        hipStream_t st = (hipStream_t)stream;
        EventPool ev;
        HIP_TRY(ev.init(2));
        auto run_for = [&](const fsg_schedule &s, int64_t k, double *ms, int64_t *steps) -> int {
            fsg_params tp = *prm;
            tp.max_steps = prm->max_steps < 0 ? k : std::min<int64_t>(prm->max_steps, k);
            fsg_run_info info;
            HIP_TRY(hipEventRecord(ev.e[0], st));
            int r = fsg_simulate(g, &tp, seeds, n_seeds, B, 0, rng_key, &s, dev_ws, ws_bytes,
                                 nullptr, nullptr, &info, stream);
            if (r) return r;
            HIP_TRY(hipEventRecord(ev.e[1], st));
            HIP_TRY(hipEventSynchronize(ev.e[1]));
            float f = 0.f;
            HIP_TRY(hipEventElapsedTime(&f, ev.e[0], ev.e[1]));
            *ms = f;
            *steps = info.steps_run;
            return FSG_OK;
        };
        auto time_one = [&](const fsg_schedule &s0, double *ms) -> int {
            fsg_schedule s = s0;
            s.time_kernels = 0;
            s.steps_per_sync = std::max(1, std::min(tune_steps, 64));
            double t1 = 0, t2 = 0;
            int64_t s1 = 0, s2 = 0;
            int r = run_for(s, tune_steps, &t1, &s1);
            if (r) return r;
            r = run_for(s, 2 * (int64_t)tune_steps, &t2, &s2);
            if (r) return r;
            *ms = s2 > s1 ? std::max(0.0, t2 - t1) / (double)(s2 - s1)
                          : (s2 > 0 ? t2 / (double)s2 : 1e30);
            return FSG_OK;
        };
        fsg_schedule d;
        default_sched(g, prm, B, &d);
        if (batch_only) {
            d.kernel_variant = 1;
            d.block_threads = kBatchBlock;
        }
        double dms = 0;
        rc = time_one(d, &dms);  // also a warm-up of the code objects
        if (rc) return rc;
        rc = time_one(d, &dms);
        if (rc) return rc;
        fsg_schedule win = d;
        double wms = dms;
        for (const fsg_schedule &s : candidates(g, prm, B, batch_only != 0)) {
            double ms = 0;
            rc = time_one(s, &ms);
            if (rc) return rc;
            if (ms < wms) {
                wms = ms;
                win = s;
            }
        }
        win.time_kernels = 0;
        *best = win;
        if (best_ms) *best_ms = wms;
        if (default_ms) *default_ms = dms;
        cache_store(cache_path, key, win, wms);
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

}  // extern "C"

// ------------------------------------------------------ batch autotuner ----
// The batch is tuned as a batch: every trial plans and runs the whole batch
// (all jobs to absorption or their caps) and is scored by its device time,
// so a schedule that helps one job alone but costs the batch is not taken.
namespace {

struct BatchTrial {
    std::vector<fsg_schedule> sched;  // per job
    int sync = 16, blocks_per_cu = 4;
};

// Knob values tried per model class (0 keeps the library default).
const int kTryLanes[] = {0, 16, 32, 64};
const int kTryTile[] = {0, 4096, 16384};
const int kTryHeavy[] = {0, 512, 1024};
const int kTrySync[] = {16, 8, 32, 64};
const int kTryBlocks[] = {4, 2, 8};

int model_class(int model)
{
    const int k = model_kind(model);
    return k == kKindIC ? 0 : (k == kKindLT ? 2 : 1);
}

}  // namespace

extern "C" {

int fsg_batch_autotune_workspace_size(const fsg_job *jobs, int32_t n_jobs, size_t *bytes)
{
    try {
        if (!jobs || !bytes || n_jobs < 1 || n_jobs > kMaxBatchJobs)
            return fail(FSG_EINVAL, "bad arguments");
        size_t best = 0;
        std::vector<fsg_job> js(jobs, jobs + n_jobs);
        for (int tile : kTryTile)
            for (int heavy : kTryHeavy) {
                for (auto &j : js) {
                    j.sched.tile_edges = tile;
                    j.sched.heavy_threshold = heavy;
                }
                fsg_plan *pl = nullptr;
                size_t need = 0;
                int rc = fsg_batch_plan(js.data(), n_jobs, 64, &pl, &need);
                if (rc) return rc;
                fsg_plan_destroy(pl);
                best = std::max(best, need);
            }
        *bytes = best;
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

int fsg_batch_autotune(const fsg_job *jobs, int32_t n_jobs, int32_t max_trials, void *dev_ws,
                       size_t ws_bytes, fsg_job *tuned, int32_t *steps_per_sync,
                       int32_t *blocks_per_cu, double *best_ms, double *default_ms,
                       int32_t *trials_run, void *stream)
{
    try {
        if (!jobs || !tuned || !steps_per_sync || !blocks_per_cu || n_jobs < 1 ||
            n_jobs > kMaxBatchJobs)
            return fail(FSG_EINVAL, "bad arguments");
        if (max_trials < 1) return fail(FSG_EINVAL, "max_trials must be >= 1");
        const std::vector<fsg_job> base(jobs, jobs + n_jobs);
        int trials = 0;
        auto run = [&](const BatchTrial &t, double *ms) -> int {
            std::vector<fsg_job> js = base;
            for (int i = 0; i < n_jobs; ++i) js[(size_t)i].sched = t.sched[(size_t)i];
            fsg_plan *pl = nullptr;
            size_t need = 0;
            int rc = fsg_batch_plan(js.data(), n_jobs, t.sync, &pl, &need);
            if (rc) return rc;
            std::unique_ptr<fsg_plan, int (*)(fsg_plan *)> guard(pl, fsg_plan_destroy);
            if (need > ws_bytes) return fail(FSG_EWORKSPACE, "batch autotune workspace too small");
            pl->blocks_per_cu = t.blocks_per_cu;
            double total = 0;
            rc = fsg_batch_run(pl, dev_ws, ws_bytes, nullptr, &total, stream);
            if (rc) return rc;
            *ms = total;
            ++trials;
            return FSG_OK;
        };
        BatchTrial cur;
        for (const auto &j : base) {
            fsg_schedule s = j.sched;
            s.time_kernels = 0;
            cur.sched.push_back(s);
        }
        double cms = 0;
        int rc = run(cur, &cms);  // warm-up
        if (rc) return rc;
        rc = run(cur, &cms);
        if (rc) return rc;
        const double dms = cms;
        auto consider = [&](const BatchTrial &t) -> int {
            if (trials >= max_trials) return FSG_OK;
            double ms = 0;
            int r = run(t, &ms);
            if (r) return r;
            if (ms < cms) {
                cms = ms;
                cur = t;
            }
            return FSG_OK;
        };
        // launch-level knobs, then per model class lanes, tiles, heavy cut
        for (int v : kTrySync) {
            if (v == cur.sync) continue;
            BatchTrial t = cur;
            t.sync = v;
            rc = consider(t);
            if (rc) return rc;
        }
        for (int v : kTryBlocks) {
            if (v == cur.blocks_per_cu) continue;
            BatchTrial t = cur;
            t.blocks_per_cu = v;
            rc = consider(t);
            if (rc) return rc;
        }
        for (int cls = 0; cls < 3; ++cls) {
            bool present = false;
            for (const auto &j : base) present |= model_class(j.prm.model) == cls;
            if (!present) continue;
            for (int knob = 0; knob < 3; ++knob) {
                const int *vals = knob == 0 ? kTryLanes : (knob == 1 ? kTryTile : kTryHeavy);
                const int nv = knob == 0 ? 4 : 3;
                const BatchTrial start = cur;
                for (int k = 0; k < nv; ++k) {
                    BatchTrial t = start;
                    bool changed = false;
                    for (int i = 0; i < n_jobs; ++i) {
                        if (model_class(base[(size_t)i].prm.model) != cls) continue;
                        fsg_schedule &sc = t.sched[(size_t)i];
                        int32_t &field = knob == 0 ? sc.row_lanes
                                                   : (knob == 1 ? sc.tile_edges : sc.heavy_threshold);
                        if (field != vals[k]) {
                            field = vals[k];
                            changed = true;
                        }
                    }
                    if (!changed) continue;
                    rc = consider(t);
                    if (rc) return rc;
                }
            }
        }
        for (int i = 0; i < n_jobs; ++i) {
            tuned[i] = base[(size_t)i];
            tuned[i].sched = cur.sched[(size_t)i];
        }
        *steps_per_sync = cur.sync;
        *blocks_per_cu = cur.blocks_per_cu;
        if (best_ms) *best_ms = cms;
        if (default_ms) *default_ms = dms;
        if (trials_run) *trials_run = trials;
        return FSG_OK;
    } catch (const std::bad_alloc &) {
        return fail(FSG_ENOMEM, "host allocation failed");
    }
}

}  // extern "C"
