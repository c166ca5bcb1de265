// fsg_internal.hpp -- structures shared by the host side of libfsg and its
// kernel launchers.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct fsg_graph;

namespace fsg {

// Host helpers shared by the translation units (fsg_abi.hip).
int set_error(int code, const char *msg);  // records the message, returns code

// Fault injection for tests of the error paths, armed by the environment
// variable FSG_FAULT_INJECT (read once per process): "alloc:N" makes the
// N-th guarded host allocation fail (std::bad_alloc -> FSG_ENOMEM),
// "device:N" makes the N-th checked HIP call report an error without
// calling HIP (-> FSG_EDEVICE); both may be given, comma-separated.  Each
// fires once.  Unset, both checks are a load and a compare.
void inject_alloc_fault();  // throws std::bad_alloc when this allocation is to fail
bool inject_device_fault(); // true when this checked HIP call is to fail
// Device view of a graph; false if it is not bound.
bool graph_view(const fsg_graph *g, int64_t *n, int64_t *nnz, int64_t *max_indeg,
                const int32_t **ptr, const int32_t **src, const int32_t **wide, int64_t *n_wide);

// Rows with more in-arcs than this are aggregated by a whole block (their
// list is built when a graph is bound).
constexpr int kWideRow = 256;

enum Kind { kKindIC = 0, kKindEpidemic = 1, kKindLT = 2 };

// Rows a tile may hold.
constexpr int kMaxTileRows = 2048;
// Words of the frontier summary the edge-parallel kernel keeps in LDS.
constexpr int kSumWords = 8192;
enum Model { kIC = 0, kSI = 1, kSIS = 2, kSIR = 3, kLT = 4, kSEIR = 5, kSEIS = 6, kSWIR = 7 };
enum IcProb { kIcUniform = 0, kIcWeightedCascade = 1, kIcPerEdge = 2 };

// Everything one synchronous step needs.  Planes are uint64 [n][W]:
//   IC:       prev/next = frontier F (double-buffered), aux = ever-active A
//   SI/SIS/SIR: prev/next = infected h (double-buffered), aux = removed r
//   LT:       prev/next = active (double-buffered), aux unused
struct StepArgs {
    const int32_t *ptr;  // [n+1]
    const int32_t *src;  // [nnz]
    const int32_t *dst;  // [nnz] target row of every arc (edge-parallel IC kernel)
    int64_t nnz;
    int32_t n;
    int32_t W;            // words per node: ceil(B / 64)
    int64_t B;
    uint64_t goff;        // replicate_offset
    uint32_t key0, key1;
    const uint64_t *prev;
    uint64_t *next;
    uint64_t *aux;
    int32_t model;
    int32_t ic_prob;
    uint32_t ic_t;          // uniform IC threshold
    const uint32_t *edge_t; // per-edge IC thresholds [nnz] or null
    const uint32_t *tinf;   // infection thresholds by infected-neighbour count
    int32_t khat;           // last index of tinf
    uint32_t trec;          // recovery threshold
    uint32_t talpha;        // SEIR / SEIS: E -> I threshold
    uint64_t *lat;          // SEIR / SEIS: latent (E) plane, SWIR: weakened (W) plane [n][W],
                            // updated in place; else null
    // SWIR: thresholds of S -> I or W and of W -> I by infected-neighbour
    // count (tinf holds S -> I); each table stops where it saturates
    const uint32_t *tsiw, *twi;
    int32_t khat_siw, khat_wi;
    // schedule
    int32_t G, S, lgG, lgS; // lanes per row: G over words, S over edges
    int32_t heavy;          // rows with more in-edges are processed as segments
    int32_t fast32;         // n+1 < 2^24, W < 2^21, (n+1)*W < 2^29, nnz < 2^30: 32-bit offsets
    const int32_t *tiles;   // [n_tiles + 1] row boundaries
    int32_t n_tiles;
    // heavy rows cut into segments
    const int32_t *seg_row, *seg_e0, *seg_e1;
    int32_t n_seg;
    const int32_t *heavy_rows, *heavy_seg;  // [n_heavy], [n_heavy + 1]
    int32_t n_heavy;
    uint64_t *partial;      // [n_seg][Lp][W]
    int32_t Lp;             // counter planes per partial (1 for IC)
    // LT: each replicate's activation threshold max(1, ceil(U indeg / 2^32)),
    // bit-sliced: plane p of node v at need[(v Lp + p) W + w], written for
    // p < bitlen(indeg(v)) <= Lp once per run; null for the other models
    uint64_t *need;
    // LT: [2][n], array t & 1 holds t for the nodes that gained an
    // activation (any replicate) at step t; step t reads array (t-1) & 1,
    // which no one writes during step t.  Seeds: 0 in array 0.  Null for
    // the other models.
    uint32_t *stamp;
    // SI / SIS / SIR and LT late in a run (the tail mode): four bitmaps of
    // ibm_words words, bitmap t % 4 marking the nodes with an infected
    // replicate after step t (LT: with a new activation at step t), and two
    // candidate bitmaps: before step t the nodes of bitmap
    // t-1 and their out-neighbours (optr / oarc) are marked in candidate
    // bitmap t % 2.  Step t reads bitmap t-2 and candidate bitmap t % 2, sets
    // bits in bitmap t and clears bitmap t+1 and candidate bitmap (t+1) % 2;
    // a light row that is not a candidate is left out of step t (no count can
    // be nonzero, no replicate can recover).  Null otherwise.
    uint32_t *ibm;
    uint32_t *cand;
    int32_t ibm_words;
    // frontier bitmaps of the edge-parallel IC kernel: bit u of bm_prev is set
    // iff node u has a newly active replicate after step t-1 (prev is only
    // meaningful where it is set); bm_next is cleared before step t
    const uint32_t *bm_prev;
    uint32_t *bm_next;
    // summaries of the bitmaps: bit i set iff some node u with u >> sum_shift
    // == i has its bitmap bit set (staged in LDS by the edge-parallel kernel)
    const uint32_t *sum_prev;
    uint32_t *sum_next;
    int32_t sum_shift;
    int32_t sum_words;
    // absorption flags: flags[t % ring] = 1 iff some replicate still has a
    // state-1 node after step t
    uint32_t *flags;
    int32_t ring;
    uint32_t step;
    // the same flags per word of 64 replicates, [wring][W]: word w of slot
    // t % wring is set iff the replicates of that word alone would set the
    // flag above after step t.  Step t reads the slots of t-1 and t-2 and
    // leaves out words clear in both.  Null unless 16 < W <= 64 (with fewer
    // words a row's words take one pass of lanes anyway).
    uint32_t *wflags;
    int32_t wring;  // ring + 1 slots (step t must not clear t-1 or t-2)
    // frontier-driven IC (one word per node): the out-adjacency of the graph
    // (oarc[optr[u] .. optr[u+1]) = (target row v, edge id e) of the arcs
    // u -> v) and four queues of (node, chunk) work items, one per step mod 4.
    // Every node that joins the frontier of step t is queued once, as
    // max(1, ceil(outdeg / kOutChunk)) items.  Step t reads the queue of t-1,
    // fills the queue of t, takes the nodes of the queue of t-2 out of their
    // plane, bitmap and summary (f_clr, bm_clr, sum_clr: the buffers step
    // t+1 writes), and resets the counters of the queue step t+1 fills.
    // Frontier planes, bitmaps and summaries rotate over three buffers.
    const int32_t *optr;
    const int2 *oarc;
    uint4 *q_in, *q_out, *q_clr;  // items (node, chunk, first arc, end of arcs)
    uint32_t *qcnt;              // [4] items in each queue
    unsigned long long *qarcs;   // [4] out-arcs of each queue's nodes
    int32_t qi_in, qi_out, qi_clr, qi_rst;
    uint64_t *f_clr;
    uint32_t *bm_clr, *sum_clr;
    // bit per node set when the node first joins a frontier (any replicate):
    // the nodes whose ever-active word can be nonzero
    uint32_t *ever;
    // step t pushes over the out-arcs of the frontier of t-1 when they are at
    // most this many, else it streams the sources of every arc
    unsigned long long push_limit;
    // when set, the SI-family decision code adds its Philox4x32-10 calls here
    // (a counting run; normal runs leave it null)
    unsigned long long *draws;
};

// Out-arcs per work item of the frontier-driven IC step (one per lane of
// the item's wave).
constexpr int kOutChunk = 64;

// A finalize queued right after a chunk of frontier-driven IC steps, before
// the host has read whether the chunk ended the run: its kernels act only if
// one of steps t0+1 .. t0+c left its absorption flag clear, and take the
// first such step T as the run's last (the frontier buffers of a step t are
// those of t mod 3, its work queue that of t mod 4).
struct SpecFin {
    const uint32_t *flags;  // absorption ring, or null: not speculative
    int32_t ring;
    int32_t c;
    int64_t t0;
    uint64_t *front3[3];  // frontier plane after a step t, t mod 3 = i
    uint32_t *bm3[3];     // its bitmap
    uint32_t *sum3[3];    // its summary
    uint4 *queue4[4];     // the work queue step t fills, t mod 4 = i
};

struct FinArgs {
    int32_t n, W, G, lgG;
    int64_t B;
    int32_t model;
    const uint64_t *one;  // state-1 plane (F, h, active)
    uint64_t *two;        // state-2 plane (A for IC, r for SIR and SEIR) or null
    // when set (one word per node), `two` is read only for nodes whose bit is
    // set and is zero elsewhere; with `scrub` the words read and the bitmap
    // are cleared after reading (the run leaves that plane all zero)
    uint32_t *two_bm;
    int32_t scrub;
    const uint64_t *three;  // latent plane (SEIR / SEIS) or null
    const uint32_t *bm;   // when set, `one` is valid only for nodes whose bit is set
    uint8_t *states;      // [n][B] or null
    uint32_t *counts;     // [n] or null
    // tally of the state after a step: out[s-1] = #(node, replicate) in
    // state s, s = 1, 2, 3; when the step did no work (the job was already
    // absorbed; flag of step - 1 clear) the previous row out[-3..-1] is
    // copied instead
    unsigned long long *tally;
    const uint32_t *flags;  // absorption ring, or null (always a live step)
    int32_t ring;
    uint32_t step;
    SpecFin spec;  // finalize queued before the run's end was known (spec.flags set)
};

// Many jobs in one launch per synchronous step.  Each job keeps its own
// StepArgs (prev/next hold its planes 0 and 1; step is filled in by the
// kernel from *cur_step).  Work items are the step blocks of every job
// (prefix item_off) and the heavy-row combine groups (prefix comb_off).
constexpr int kMaxBatchJobs = 1024;

struct BatchCtl {
    const StepArgs *jobs;     // [n_jobs]
    const int32_t *item_off;  // [n_jobs + 1]
    const int32_t *comb_off;  // [n_jobs + 1]
    const int32_t *code;      // [n_jobs]: kind * 32 + counter planes
    const int32_t *max_step;  // [n_jobs]
    int32_t n_jobs;
    int32_t ring;
    uint32_t *queue;          // [2] dequeue counters (step items, combine items)
    uint32_t *cur_step;       // the step the next launch executes
    // tail mode (SI family, LT, IC; jobs whose graph has its out-adjacency):
    // tail_on[j] != 0 while job j runs in it (set by the host per chunk; the
    // job's StepArgs carry its bitmaps, which job_at_step drops otherwise);
    // word_off: prefix over the jobs of their bitmap words (0 for jobs that
    // cannot take the mode), row_off: prefix of their node counts
    const int32_t *tail_on;   // [n_jobs]
    const int32_t *word_off;  // [n_jobs + 1]
    const int32_t *row_off;   // [n_jobs + 1]
};

// launchers (fsg_kernels.hip); return the hipError_t of the launch
hipError_t launch_fill64(uint64_t *p, int64_t count, uint64_t value, hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);  // p 256-byte aligned
// the same unless *tag == expect when the kernel runs (the region is then
// known to be zero already)
hipError_t launch_zero_unless(void *p, size_t bytes, const uint64_t *tag, uint64_t expect,
                              hipStream_t s);
hipError_t launch_fill32(uint32_t *p, int64_t count, uint32_t value, hipStream_t s);
hipError_t launch_stamp_seeds(uint32_t *stamp, const int32_t *seeds, int64_t ns, hipStream_t s);
// Tail mode of the SI family: the bitmaps step t reads (state t-1 in `cur`,
// state t-2 in `old`) and the cleared one it writes, and the number of nodes
// with a nonzero word in a plane.
hipError_t launch_mark_rows(const uint64_t *cur, const uint64_t *old, uint32_t *ibm, uint32_t *cand,
                            int32_t ibm_words, int64_t n, int64_t W, uint32_t t, hipStream_t s);
// LT: the bitmaps from the activation stamps, and the nodes with a new
// activation at step t.
hipError_t launch_mark_gained(const uint32_t *stamp, uint32_t *ibm, uint32_t *cand, int32_t ibm_words,
                              int64_t n, uint32_t t, hipStream_t s);
hipError_t launch_count_stamped(const uint32_t *stamp, int64_t n, uint32_t t,
                                unsigned long long *count, hipStream_t s);
// Candidate rows of tail-mode step a.step (one wave per infected node).
hipError_t launch_tail_expand(const StepArgs &a, hipStream_t s);
hipError_t launch_count_rows(const uint64_t *plane, int64_t n, int64_t W, unsigned long long *count,
                             hipStream_t s);
hipError_t launch_ring_clear(uint32_t *flags, int32_t ring, int32_t keep, hipStream_t s,
                             uint32_t *wflags = nullptr, int32_t W = 0, int32_t wring = 0,
                             int64_t t = 0);
hipError_t launch_seed(uint64_t *p1, uint64_t *p2, const int32_t *seeds, int64_t ns, int32_t W,
                       int64_t B, uint32_t *flag0, uint32_t *bm, uint32_t *sum, int sum_shift,
                       hipStream_t s);
hipError_t launch_ic_stream(const StepArgs &a, int grid, int block, hipStream_t s);
hipError_t launch_ic_front(const StepArgs &a, int grid, int block, hipStream_t s);
// the clear duty of k_ic_front alone (the queue of a.qi_clr leaves f_clr,
// bm_clr, sum_clr), whatever the absorption flags say
hipError_t launch_ic_scrub(const StepArgs &a, hipStream_t s);
// the same for a finalize queued before the run's end was known: the
// frontier of step T - 2 + which, T the run's last step (1 or 2), and the
// run's tag written after the second
hipError_t launch_ic_scrub_spec(const StepArgs &a, const SpecFin &sp, int which, uint64_t *tag,
                                uint64_t tag_value, hipStream_t s);
hipError_t launch_seed_queue(const StepArgs &a, const int32_t *seeds, int64_t ns, hipStream_t s);
hipError_t launch_out_count(const int32_t *src, int64_t nnz, int32_t *cnt, hipStream_t s);
hipError_t launch_out_fill(const int32_t *src, const int32_t *dst, int64_t nnz, int32_t *cursor,
                           int2 *oarc, hipStream_t s);
hipError_t launch_expand_rows(const int32_t *ptr, int64_t n, int32_t *dst, hipStream_t s);
hipError_t launch_ic_clear(const StepArgs &a, hipStream_t s);
hipError_t launch_lt_need(const StepArgs &a, hipStream_t s);
hipError_t launch_step(const StepArgs &a, int kind, int L, int block, hipStream_t s);
hipError_t launch_combine(const StepArgs &a, int kind, int block, hipStream_t s);
hipError_t launch_finalize(const FinArgs &f, hipStream_t s);
hipError_t launch_tally(const FinArgs &f, hipStream_t s);
hipError_t launch_philox(const uint32_t *ctr, uint32_t k0, uint32_t k1, uint32_t *out,
                         int64_t count, hipStream_t s);
int counter_planes_for(int64_t max_count);  // compile-time counter width to use
int step_blocks(const StepArgs &a, int block);  // blocks of one job's pull step
hipError_t launch_batch_step(const BatchCtl &c, int grid, hipStream_t s);
hipError_t launch_batch_combine(const BatchCtl &c, int grid, hipStream_t s);
hipError_t launch_batch_advance(const BatchCtl &c, hipStream_t s);
// tail mode of the batched launch: candidates of the next step of every job
// in the mode (before each batched step), and per job the nodes with an
// infected replicate / a new activation after step t into counts[j]
hipError_t launch_batch_expand(const BatchCtl &c, hipStream_t s);
hipError_t launch_batch_count(const BatchCtl &c, uint32_t t, unsigned long long *counts, hipStream_t s);
constexpr int kBatchBlock = 256;  // block size of the batched kernels
// Waves per SIMD the batched step kernel is compiled for.  One kernel holds every
// (model, counter width) case, so unbounded it takes the register count of the
// widest case plus what the case switch adds (229 VGPRs: two waves per SIMD);
// three waves keep the LT and SI cases up to 12 counter planes unspilled,
// four spill them.
constexpr int kBatchWavesPerSimd = 3;

// Heavy rows merged per wave by the combine kernels: each row takes G word
// lanes times min(64 / G, 16) segment lanes.
__host__ __device__ inline int combine_rows_per_wave(int lgG)
{
    const int lanes = 64 >> lgG;
    return lanes < 16 ? 1 : lanes / 16;
}

}  // namespace fsg
