/*
 * fsg.h -- C-ABI of libfsg, batched Monte Carlo graph propagation on MI355X.
 *
 * The library runs the synchronous message-passing step of FS_GPlib
 * (arxiv 2603.14895): for every node and every Monte Carlo replicate, gather
 * the previous-round states of the in-neighbours, aggregate, and update the
 * node's state (Sec. 3.1, Eq. ms, Eq. agg, Eq. updata), for all replicates of
 * a batch at once (Definition "Batched Monte Carlo Method", Eq. batch), until
 * no replicate can change any more or a step cap is reached.  The calls
 * follow the problem statement of the paper's model interface (Sec. 4,
 * Eq. model: graph, seed set, parameters, device; run_epochs returns the
 * final states of all runs), plus the replicate count, the replicate offset
 * of the batch and the RNG key.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns FSG_OK (0) or a negative status; no C++ exception
 *   crosses this boundary.  fsg_last_error() describes the last failure on
 *   the calling thread.  On failure, outputs are unspecified and nothing has
 *   been written to caller memory except possibly the outputs themselves.
 * - Arguments are validated on the host before anything is launched.
 * - The caller owns every buffer.  All device memory comes from the caller
 *   (a workspace sized by the *_workspace_size queries); the library never
 *   allocates or frees device memory.  It may allocate host memory.
 * - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 * - Randomness: Philox4x32-10 (Salmon et al., SC'11) keyed by rng_key.  A
 *   draw for (domain, unit, replicate g, step) uses counter
 *   (lo32 unit, g >> 2, step, domain << 24 | hi32 unit) and keeps word g & 3;
 *   g = replicate_offset + r is the global replicate index, so results do
 *   not depend on how a Monte Carlo run is split into batches.  Domains:
 *   1 = IC edge trial (unit = edge id, step 0), 2 = per-node step draw
 *   (unit = node, step = t), 3 = LT threshold (unit = node, step 0).
 *   A Bernoulli(p) fires iff t == 0xFFFFFFFF or draw < t, with
 *   t = thr(p) = 0 for p <= 0, 0xFFFFFFFF for p >= 1, otherwise
 *   min(floor(p * 2^32), 0xFFFFFFFE), computed in FP64 on the host.
 */
#ifndef FSG_H
#define FSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSG_ABI_VERSION 3

/* status codes */
#define FSG_OK 0
#define FSG_EINVAL (-1)       /* an argument is out of its documented range    */
#define FSG_ENOMEM (-2)       /* host allocation failed                        */
#define FSG_EDEVICE (-3)      /* a HIP call failed; the message names it       */
#define FSG_EUNSUPPORTED (-4) /* valid but outside what this build handles     */
#define FSG_EWORKSPACE (-5)   /* workspace missing, too small or misaligned    */

/* models (Table tab:29s; SIR rule of Appendix A.1) */
#define FSG_IC 0  /* independent cascade: 0 inactive, 1 newly active, 2 active  */
#define FSG_SI 1  /* SI: SIR without recovery                                   */
#define FSG_SIS 2 /* SIS: recovery returns the node to S                        */
#define FSG_SIR 3 /* SIR: 0 S, 1 I, 2 R                                         */
#define FSG_LT 4  /* linear threshold, in-weights 1/indeg, thresholds U(0,1)    */
#define FSG_SEIR 5 /* SEIR(DT): 0 S, 1 E (latent), 2 I, 3 R                     */
#define FSG_SEIS 6 /* SEIS(DT): SEIR with recovery back to S                    */
#define FSG_SWIR 7 /* SWIR: 0 S, 1 W (weakened), 2 I, 3 R                      */

/* IC edge probability */
#define FSG_IC_UNIFORM 0          /* p for every arc                         */
#define FSG_IC_WEIGHTED_CASCADE 1 /* p = 1/indeg(target)                     */
#define FSG_IC_PER_EDGE 2         /* edge_p[e], host array of nnz doubles    */

typedef struct fsg_graph fsg_graph;

/* Model and parameters.
 * max_steps: step cap K >= 0.  For IC and LT a negative value means "until
 * absorption" (at most n steps can change anything).  SI, SIS, SIR require
 * K >= 0.  p, beta, gamma, edge_p[] must lie in [0, 1] and not be NaN.
 * For SI, gamma is ignored (no recovery).
 * SEIR / SEIS (named in Table tab:29s; the paper gives no equations, so
 * this is the discrete-time SIR rule with a latent state): a susceptible
 * node with k infectious in-neighbours becomes E with probability
 * 1 - (1-beta)^k, E becomes I with probability alpha, I becomes R (SEIS: S)
 * with probability gamma, one draw per node, replicate and step; seeds
 * start infectious; they require K >= 0.  alpha must lie in [0, 1] and is
 * ignored by the other models.
 * SWIR (named in Table tab:29s and compared in Table tab:result with three
 * parameters; the paper gives no rule, so this is a reading): kappa = beta,
 * mu = alpha, nu = gamma, kappa + mu <= 1.  With k infected in-neighbours a
 * susceptible node becomes I with probability 1 - (1-kappa)^k, else W with
 * probability (1-kappa)^k - (1-kappa-mu)^k (one draw decides both), a
 * weakened node becomes I with probability 1 - (1-nu)^k, and an infected
 * node is removed after one step; seeds start infected; a negative K means
 * "until no node is infected". */
typedef struct {
    int32_t model;
    int32_t ic_prob;
    double p;
    const double *edge_p; /* host, [nnz], only for FSG_IC_PER_EDGE */
    double beta;
    double gamma;
    int64_t max_steps;
    double alpha; /* SEIR / SEIS: per-step probability of E -> I */
} fsg_params;

/* steps_run: number of synchronous steps executed (the batch shares one
 * loop that stops once no replicate has a state-1 node -- for SEIR / SEIS
 * no node in E or I -- or at max_steps).
 * absorbed: 1 iff no replicate ends with such a node.
 * step_kernel_ms, step_launches: when the schedule asks for kernel timing,
 * the summed device time of the pull-step kernel (HIP events recorded on the
 * call's stream right around its launch in every step that did work; the
 * heavy-row combine and the frontier clear are not included) and the number
 * of steps timed; the frontier-driven IC step (one kernel a step, launched
 * back to back) is timed per chunk of steps_per_sync launches instead, the
 * launches after absorption, which return at once, included in both; else 0.
 * setup_ms: with kernel timing, the device time from the first to the last
 * set-up operation (table uploads, plane fills, seeding; host work between
 * them included); finalize_ms: the device time of the kernel that writes
 * final_states and infected_counts (fsg_simulate only); else 0.
 * tail_steps: steps run in the tail mode (see FSG_OPT_TAIL_OFF), which
 * leave out the rows that cannot change; else 0.
 * philox_calls: with FSG_OPT_COUNT_DRAWS, the Philox4x32-10 calls of the
 * SI-family decisions over the steps run (each call gives the draws of four
 * consecutive replicates of one node and step); else 0. */
typedef struct {
    int64_t steps_run;
    int32_t absorbed;
    int32_t tail_steps;
    double step_kernel_ms;
    int64_t step_launches;
    double setup_ms;
    double finalize_ms;
    int64_t philox_calls;
} fsg_run_info;

/* Launch schedule of the pull step (what the autotuner searches).  A value
 * of 0 in any field means "library default".
 *   row_lanes      lanes that share one row, a power of two in [1, 64].
 *                  The lanes split first over the row's state words
 *                  (min(row_lanes, next_pow2(ceil(B/64))) of them), the
 *                  rest split the row's in-edge list.
 *   block_threads  workgroup size: 64, 128, 256, 512 or 1024.
 *   tile_edges     target in-edges per workgroup tile (contiguous rows).
 *   heavy_threshold rows with more in-edges than this are cut into
 *                  segments of at most this many edges, processed in
 *                  parallel and merged (OR / integer add, order-free).
 *   steps_per_sync synchronous steps launched between host polls of the
 *                  absorption flags.
 *   time_kernels   1: time every pull step with HIP events (reported in
 *                  fsg_run_info); 0: no timing.
 *   kernel_variant 0: the library picks (3 for IC with B <= 64 on a graph
 *                  with its out-adjacency bound, else 2 for IC with
 *                  B <= 64, else 1); 1: row-group pull kernel (any model
 *                  and B); 2: edge-parallel IC kernel with a frontier
 *                  bitmap (IC with B <= 64 only, else FSG_EINVAL); 3:
 *                  frontier-driven IC (IC with B <= 64 on a graph bound
 *                  with fsg_graph_bind_out): each step pushes the trials of
 *                  the previous step's frontier over its out-arcs while
 *                  those are at most nnz / 16, and otherwise streams every
 *                  arc as variant 2 does; same draws, same results.  With
 *                  variants 2 and 3, row_lanes is not used, and variant 3
 *                  launches blocks of 512 threads.
 *   options        bit flags, 0 by default.  FSG_OPT_WIDE_OFFSETS: the
 *                  row-group kernels address sources and state planes with
 *                  64-bit offsets even where 32-bit ones suffice (they are
 *                  used by themselves when n + 1 >= 2^24, ceil(B/64) >=
 *                  2^21, (n + 1) ceil(B/64) >= 2^29 or nnz >= 2^30); the
 *                  results are the same either way.  FSG_OPT_COUNT_DRAWS:
 *                  count the generator calls of the SI / SIS / SIR / SEIR /
 *                  SEIS decisions (reported in fsg_run_info.philox_calls;
 *                  one wave-reduced atomic add per row pass, so it is for
 *                  measurement runs, not timed ones).
 *                  FSG_OPT_REUSE_WORKSPACE (fsg_simulate): the caller
 *                  states that dev_ws was last written by a completed
 *                  fsg_simulate call with the same graph, parameters, B and
 *                  schedule, and not modified since.  A frontier-driven IC
 *                  run (variant 3) that wrote outputs leaves its frontier
 *                  planes, bitmaps and ever-active plane all zero (the
 *                  finalize clears the ever-active words it reads, a last
 *                  pass clears the two frontiers no step cleared) and
 *                  records that with a tag in dev_ws; with this option the
 *                  next such run clears those buffers only if the tag is not
 *                  there (checked on the device, so a run that stopped on an
 *                  error, or another layout in the same memory, still gets
 *                  them cleared).  Other runs ignore the option; results are
 *                  the same either way.
 *                  Tail mode (SI, SIS, SIR, LT, and IC on the pull step,
 *                  kernel_variant 1; any B; fsg_simulate, sessions and
 *                  batches; on a graph with its out-adjacency bound): once
 *                  few nodes hold an infected replicate (IC, LT: a new
 *                  activation), a row whose in-neighbours and itself hold
 *                  none after step t-1 cannot change at step t and is left
 *                  out of it; before each step the out-arcs of those nodes
 *                  mark the rows that are not (one more small kernel a step,
 *                  timed with the step kernel).  The library counts such
 *                  nodes at every poll of the absorption flags and takes the
 *                  mode for the next chunk of steps when that count times
 *                  the mean in-degree is at most n.  FSG_OPT_TAIL_OFF never
 *                  takes it; FSG_OPT_TAIL_ALWAYS takes it for every chunk
 *                  after the first (for tests).  Results are the same either
 *                  way. */
#define FSG_OPT_WIDE_OFFSETS 1
#define FSG_OPT_COUNT_DRAWS 2
#define FSG_OPT_REUSE_WORKSPACE 4
#define FSG_OPT_TAIL_OFF 8
#define FSG_OPT_TAIL_ALWAYS 16
typedef struct {
    int32_t row_lanes;
    int32_t block_threads;
    int32_t tile_edges;
    int32_t heavy_threshold;
    int32_t steps_per_sync;
    int32_t time_kernels;
    int32_t kernel_variant;
    int32_t options;
} fsg_schedule;

/* Library version of this header (FSG_ABI_VERSION). */
int fsg_abi_version(void);

/* Message for the last failing call on this thread; valid until the next
 * fsg_* call on the same thread.  Never NULL. */
const char *fsg_last_error(void);

/* Graph (Sec. 2, Definitions "Graph" and "CSR"; update rule Eq. nodestate
 * pulls over in-neighbours N^-(v)).
 * n >= 1 nodes, nnz >= 0 arcs, nnz <= 2^31 - 256 (arc indices and the
 * few arcs kernels look past a row's end stay in int32).  in_ptr: host int64 [n+1],
 * in_ptr[0] = 0, non-decreasing, in_ptr[n] = nnz.  in_src: host int32
 * [nnz]; in_src[in_ptr[v] .. in_ptr[v+1]) are the sources u of the arcs
 * u -> v.  The edge id of an arc is its position in in_src.  Undirected
 * graphs store both arcs.  Self-loops and repeated arcs are allowed.
 * in_ptr is copied; in_src is borrowed until fsg_graph_bind returns.
 * Errors: FSG_EINVAL (NULL pointers, n < 1, a malformed CSR, a source out
 * of range), FSG_EUNSUPPORTED (nnz > 2^31 - 256, n > 2^31 - 2), FSG_ENOMEM. */
int fsg_graph_create(int64_t n, int64_t nnz, const int64_t *in_ptr, const int32_t *in_src,
                     fsg_graph **out);

/* Device bytes the graph needs (row pointers and sources on the device). */
int fsg_graph_workspace_size(const fsg_graph *g, size_t *bytes);

/* Copies the graph into caller device memory dev_ws (at least
 * fsg_graph_workspace_size bytes, 256-byte aligned), which must stay valid
 * and untouched while the graph is used.  Synchronous on `stream`.
 * Errors: FSG_EWORKSPACE, FSG_EDEVICE. */
int fsg_graph_bind(fsg_graph *g, void *dev_ws, size_t ws_bytes, void *stream);

/* Out-adjacency of a bound graph, for the frontier-driven IC steps
 * (kernel_variant 3): the arcs grouped by source, each with its target row
 * and its edge id (its position in in_src), so a step can reach the out-arcs
 * of the nodes that just became active without scanning every arc.  Built on
 * the device from the bound sources (out-degrees, prefix sums on the host,
 * placement); the order of arcs inside a source's group is unspecified and
 * does not change any result.  dev_ws: at least fsg_graph_out_workspace_size
 * bytes (4 (n + 1) + 8 nnz + 4 n, rounded up), 256-byte aligned, kept valid
 * and untouched while the graph is used.  Synchronous on `stream`.
 * Errors: FSG_EINVAL (graph NULL or not bound), FSG_EWORKSPACE,
 * FSG_EDEVICE, FSG_ENOMEM. */
int fsg_graph_out_workspace_size(const fsg_graph *g, size_t *bytes);
int fsg_graph_bind_out(fsg_graph *g, void *dev_ws, size_t ws_bytes, void *stream);

/* n, nnz and the largest in-degree; any output may be NULL. */
int fsg_graph_stats(const fsg_graph *g, int64_t *n, int64_t *nnz, int64_t *max_indeg);

/* Frees the host-side graph object (never the caller's device memory). */
int fsg_graph_destroy(fsg_graph *g);

/* Schedule the library picks for this graph, model and B without tuning. */
int fsg_default_schedule(const fsg_graph *g, const fsg_params *prm, int64_t B,
                         fsg_schedule *out);

/* Device bytes fsg_simulate needs for (graph, params, B, schedule); sched
 * may be NULL (default schedule). */
int fsg_sim_workspace_size(const fsg_graph *g, const fsg_params *prm, int64_t B,
                           const fsg_schedule *sched, size_t *bytes);

/* Batched Monte Carlo propagation (Algorithm 1 run as Eq. batch): B >= 1
 * replicates with global indices replicate_offset + r, r < B
 * (replicate_offset >= 0, replicate_offset + B <= 2^34), every replicate
 * starting with the seed set in state 1 (SEIR / SEIS: state 2, I) and
 * everything else in state 0.
 * seeds: host int32 [n_seeds], each in [0, n); duplicates are ignored and an
 * empty set is valid (nothing happens).
 * Outputs (device, either may be NULL):
 *   final_states [n][B] uint8, final_states[v*B + r] = state of node v in
 *     replicate r (IC 0/1/2, SIR 0/1/2, SI and SIS 0/1, LT 0/1,
 *     SEIR 0/1/2/3, SEIS 0/1/2, SWIR 0/1/2/3);
 *   infected_counts [n] uint32, the number of replicates in which v is
 *     counted: ever active (IC), ever infected (SI, SIR), infected at the
 *     end (SIS), active (LT), ever exposed (SEIR), exposed or infectious at
 *     the end (SEIS), ever weakened or infected (SWIR).
 * info (host, may be NULL) receives steps_run and absorbed.
 * The graph must be bound.  dev_ws: at least fsg_sim_workspace_size bytes,
 * 256-byte aligned; its contents on entry do not matter.  The call returns
 * after the work on `stream` has completed.
 * Errors: FSG_EINVAL, FSG_EWORKSPACE, FSG_EDEVICE, FSG_EUNSUPPORTED. */
int fsg_simulate(const fsg_graph *g, const fsg_params *prm, const int32_t *seeds, int64_t n_seeds,
                 int64_t B, int64_t replicate_offset, uint64_t rng_key, const fsg_schedule *sched,
                 void *dev_ws, size_t ws_bytes, uint8_t *final_states, uint32_t *infected_counts,
                 fsg_run_info *info, void *stream);

/* fsg_simulate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same run, with the workspace taken from a static device array of
 * fsg_simulate_noalloc_limit() bytes (64 MiB) that each GPU the library runs
 * on holds until the process ends.  The call itself allocates no device
 * memory (no hipMalloc, hipFree or allocating library routine); the caller
 * still owns the bound graph and the outputs.  Kernel timing is not done
 * (sched->time_kernels is ignored).  Every call on one GPU uses that GPU's
 * one array, so calls that overlap on a GPU (other threads or streams)
 * race; the array keeps the last call's contents, and a call clears what it
 * needs.  Errors: as fsg_simulate, and FSG_EWORKSPACE when the run needs more
 * workspace than the array holds (fsg_sim_workspace_size tells). */
size_t fsg_simulate_noalloc_limit(void);
int fsg_simulate_noalloc(const fsg_graph *g, const fsg_params *prm, const int32_t *seeds,
                         int64_t n_seeds, int64_t B, int64_t replicate_offset, uint64_t rng_key,
                         const fsg_schedule *sched, uint8_t *final_states,
                         uint32_t *infected_counts, fsg_run_info *info, void *stream);

/* Stateful stepping (the paper's run_iteration / run_iterations: steps that
 * continue from the current state, Sec. 3.3 "Basic Workflow").  Because
 * every draw is keyed by (unit, replicate, step), a run cut into any number
 * of session steps gives bit for bit what one fsg_simulate call gives.
 * fsg_session_begin validates and seeds like fsg_simulate (same workspace,
 * fsg_sim_workspace_size) and keeps pointers into dev_ws, which must stay
 * valid until fsg_session_end; synchronous.  Calls on one session must not
 * overlap. */
typedef struct fsg_session fsg_session;
int fsg_session_begin(const fsg_graph *g, const fsg_params *prm, const int32_t *seeds,
                      int64_t n_seeds, int64_t B, int64_t replicate_offset, uint64_t rng_key,
                      const fsg_schedule *sched, void *dev_ws, size_t ws_bytes, void *stream,
                      fsg_session **out);
/* Runs up to n_steps further steps (fewer once the run is absorbed or
 * reaches prm->max_steps).  dev_tally (device uint64 [n_steps][3], or NULL):
 * row i receives, for the state after the i-th step of this call, the number
 * of (node, replicate) pairs in states 1, 2 and 3 (state 0 is the rest of
 * n * B); rows of steps not run repeat the final state's tally.  info:
 * steps_run = steps executed since begin, absorbed.  Synchronous. */
int fsg_session_step(fsg_session *s, int64_t n_steps, uint64_t *dev_tally, fsg_run_info *info,
                     void *stream);
/* The current state: states (device uint8 [n][B] or NULL), counts (device
 * uint32 [n] or NULL, as fsg_simulate) and its tally (device uint64 [3] or
 * NULL).  Synchronous. */
int fsg_session_read(fsg_session *s, uint8_t *states, uint32_t *counts, uint64_t *dev_tally,
                     void *stream);
int fsg_session_end(fsg_session *s);

/* ---- Hegselmann-Krause opinion dynamics (Appendix A.2, "Micro-accelerated
 * implementation of HK model").  Each of B replicates holds one FP32
 * opinion per node; a synchronous step sends over every arc j -> i the pair
 * (h_j, 1) if |h_i - h_j| < eps (strict) and (0, 0) otherwise; node i takes
 * the sum of the first components divided by the sum of the second, and
 * keeps h_i when that count is 0.  No randomness.
 * Arithmetic: per (node, replicate) the passing opinions are added in IEEE
 * single precision in in_src order (one rounding per addition, from +0.0),
 * then divided once, rounding to nearest even, by the count; results are
 * bit-reproducible.
 *
 * fsg_hk_workspace_size: device bytes fsg_hk needs for (graph, B, sched);
 * sched may be NULL.
 * fsg_hk: dev_h (device float [n][B], replicate fastest, 16-byte aligned)
 * holds the initial opinions on entry and the final ones on return.  The
 * run stops after max_steps >= 0 steps, or after the first step that
 * changes no opinion in any replicate (the batch shares one loop).  eps
 * must be finite and >= 0 (0: nothing ever moves).  sched (may be NULL):
 * steps_per_sync (steps queued between host polls of the change flags,
 * default 16, at most 256) and time_kernels are used, the other fields are
 * ignored.  dev_counts (device uint32 [B], or NULL) receives, per
 * replicate, the number of nodes whose final opinion exceeds act.  info
 * (may be NULL): steps_run = steps executed (the unchanged last step
 * included), absorbed = 1 iff the run stopped on a step with no change,
 * step_kernel_ms / step_launches as fsg_simulate.  dev_ws: at least
 * fsg_hk_workspace_size bytes, 256-byte aligned.  Synchronous on stream.
 * Errors: FSG_EINVAL (graph not bound, B < 1, max_steps < 0, eps negative,
 * NaN or infinite, act NaN), FSG_EWORKSPACE, FSG_EUNSUPPORTED
 * (n * B / v >= 2^31 - 256, v = 4 if B % 4 == 0 else 1, or B >= 2^28),
 * FSG_EDEVICE. */
int fsg_hk_workspace_size(const fsg_graph *g, int64_t B, const fsg_schedule *sched, size_t *bytes);
int fsg_hk(const fsg_graph *g, float eps, int64_t max_steps, int64_t B, float *dev_h,
           const fsg_schedule *sched, void *dev_ws, size_t ws_bytes, float act,
           uint32_t *dev_counts, fsg_run_info *info, void *stream);
/* Weighted HK (named "WHK" in Table tab:29s, compared with the parameters
 * (0.32, 0.2) in Table tab:result; the paper gives no rule, so this is a
 * reading): each node moves the fraction mu in [0, 1] of the way from its
 * opinion h to the HK mean m of its eps-neighbourhood, h' = (1 - mu) h +
 * mu m (two products and a sum, each rounded to FP32, no contraction), and
 * keeps h when no in-neighbour is within eps.  mu = 1 is fsg_hk; otherwise
 * as fsg_hk (same workspace, flags, counts and errors, FSG_EINVAL for mu
 * outside [0, 1]). */
int fsg_whk(const fsg_graph *g, float eps, float mu, int64_t max_steps, int64_t B, float *dev_h,
            const fsg_schedule *sched, void *dev_ws, size_t ws_bytes, float act,
            uint32_t *dev_counts, fsg_run_info *info, void *stream);

/* ---- Batches: many jobs (graphs, models, seed sets, B) in one launch per
 * synchronous step (Definition "Batched Monte Carlo Method" applied across
 * jobs as well as replicates).  Every launch is a persistent work-queue
 * kernel whose blocks dequeue the tiles and heavy-row segments of all live
 * jobs; a chunk of steps is captured once in a hipGraph and replayed until
 * every job is absorbed or at its step cap.  Each job's results are
 * bit-identical to fsg_simulate on the same arguments. */
typedef struct fsg_plan fsg_plan;

typedef struct {
    const fsg_graph *g;         /* bound graph                                      */
    fsg_params prm;
    const int32_t *seeds;       /* host, read by fsg_batch_run                      */
    int64_t n_seeds;
    int64_t B;
    int64_t replicate_offset;
    uint64_t rng_key;
    fsg_schedule sched;         /* zeros = defaults; kernel_variant must be 0 or 1   */
    uint8_t *final_states;      /* device [n][B] or NULL                            */
    uint32_t *infected_counts;  /* device [n] or NULL                               */
} fsg_job;

/* Plans a batch of 1 <= n_jobs <= 1024 jobs (each validated as by
 * fsg_simulate) and reports the device workspace it needs.  steps_per_sync
 * (>= 1) is the number of steps per captured graph.  The jobs array is
 * copied; the seed arrays it points to must stay valid until
 * fsg_batch_run returns.  Errors: FSG_EINVAL, FSG_EUNSUPPORTED, FSG_ENOMEM. */
int fsg_batch_plan(const fsg_job *jobs, int32_t n_jobs, int32_t steps_per_sync, fsg_plan **out,
                   size_t *ws_bytes);

/* Runs the batch with caller workspace dev_ws (256-byte aligned, at least
 * ws_bytes of fsg_batch_plan).  infos: host [n_jobs] or NULL; total_ms:
 * host, device time of all captured step chunks (HIP events on `stream`),
 * or NULL.  Returns after the work has completed.
 * Errors: FSG_EINVAL, FSG_EWORKSPACE, FSG_EDEVICE. */
int fsg_batch_run(fsg_plan *plan, void *dev_ws, size_t ws_bytes, fsg_run_info *infos,
                  double *total_ms, void *stream);

/* Persistent blocks per compute unit of the batched step and merge kernels
 * (default 4; at most 32).  Errors: FSG_EINVAL. */
int fsg_batch_set_launch(fsg_plan *plan, int32_t blocks_per_cu);

int fsg_plan_destroy(fsg_plan *plan);

/* ---- Batch autotuner (the batch-size methodology of Tables tab:IC_batchsize
 * and tab:SIR_batchsize applied to a whole batch): every trial plans and
 * runs the whole batch and is scored by its device time (fsg_batch_run's
 * total_ms), so a schedule that helps a job alone but costs the batch is
 * not taken.  Coordinate descent from the jobs' own schedules over:
 * steps_per_sync (16, 8, 32, 64), blocks per compute unit (4, 2, 8), then
 * for each model class present (IC, SI family, LT) the lanes per row
 * (default, 16, 32, 64), tile size (default, 2048, 8192 arcs) and heavy-row
 * cut (default, 512, 2048), each applied to every job of the class.  The
 * default is run twice (the first is a warm-up); at most max_trials trials.
 * The jobs' outputs are written by every trial (the same bits each time).
 * tuned: host [n_jobs] receives the jobs with their tuned schedules;
 * steps_per_sync / blocks_per_cu: the tuned launch (give them to
 * fsg_batch_plan / fsg_batch_set_launch); best_ms / default_ms: device ms
 * of one batch run; trials_run: trials run.  dev_ws: at least
 * fsg_batch_autotune_workspace_size bytes.  Synchronous.
 * Errors: as fsg_batch_plan and fsg_batch_run. */
int fsg_batch_autotune_workspace_size(const fsg_job *jobs, int32_t n_jobs, size_t *bytes);
int fsg_batch_autotune(const fsg_job *jobs, int32_t n_jobs, int32_t max_trials, void *dev_ws,
                       size_t ws_bytes, fsg_job *tuned, int32_t *steps_per_sync,
                       int32_t *blocks_per_cu, double *best_ms, double *default_ms,
                       int32_t *trials_run, void *stream);

/* ---- Autotuner: times short runs of candidate schedules (from the seeds,
 * runs of tune_steps and 2 tune_steps steps with HIP events around each on
 * `stream`; the cost per step is their difference over the extra steps, so
 * the set-up is left out and every kernel of a step counts) -- lanes per row,
 * tile size, heavy-row cut, block size, kernel variant -- and returns the
 * fastest.  batch_only = 1 restricts the search to schedules the batched
 * launch accepts.  cache_path (nullable): a text file of earlier results
 * keyed by graph size, in-degree maximum, model and B; a hit returns without
 * running anything.  dev_ws: at least fsg_autotune_workspace_size bytes.
 * best_ms / default_ms (nullable): measured ms per step of the winner and of
 * the library default. */
int fsg_autotune_workspace_size(const fsg_graph *g, const fsg_params *prm, int64_t B,
                                int32_t batch_only, size_t *bytes);
int fsg_autotune(const fsg_graph *g, const fsg_params *prm, const int32_t *seeds, int64_t n_seeds,
                 int64_t B, uint64_t rng_key, int32_t tune_steps, int32_t batch_only,
                 const char *cache_path, void *dev_ws, size_t ws_bytes, fsg_schedule *best,
                 double *best_ms, double *default_ms, void *stream);

/* ---- Learned surrogate of the SIR spread (message passing with learned
 * message, aggregation = mean over in-neighbours, learned update; the
 * structure of Eq. ms, Eq. agg, Eq. updata).  Per node v of seed set s:
 *   x_v = [seed_v, 20 beta, log1p(indeg_v) / 8, 1, 0 x 12]
 *   h1 = ReLU(W1 [x_v | mean x_u] + b1), h2, h3 likewise from h1, h2 (width 64)
 *   p_v = sigmoid(wo . h3_v + bo), the predicted infection frequency of v.
 * BF16 weights and activations, FP32 accumulation (MFMA), FP32 master
 * weights and Adam moments.  Parameters: a flat FP32 vector of 18689 values
 * in the order W1 [32][64], b1, W2 [128][64], b2, W3 [128][64], b3, wo [64],
 * bo.  A network lives on the host until bound to caller device memory of
 * fsg_gnn_state_size bytes; activations use a per-call workspace of
 * fsg_gnn_workspace_size bytes.  All device pointers are caller-owned. */
typedef struct fsg_gnn fsg_gnn;

/* hidden must be 64 and layers 3 (FSG_EUNSUPPORTED otherwise); init_seed
 * fixes the uniform Glorot initialisation of the weights (biases 0). */
int fsg_gnn_create(int32_t hidden, int32_t layers, uint64_t init_seed, fsg_gnn **out);
int fsg_gnn_destroy(fsg_gnn *g);
int fsg_gnn_param_count(const fsg_gnn *g, int64_t *count);
int fsg_gnn_state_size(const fsg_gnn *g, size_t *bytes);
/* Uploads the initial parameters into dev_state (256-byte aligned) and
 * zeroes the Adam moments.  Synchronous. */
int fsg_gnn_bind(fsg_gnn *g, void *dev_state, size_t bytes, void *stream);
/* Workspace of one forward or training call on `graph` for n_sets seed sets. */
int fsg_gnn_workspace_size(const fsg_gnn *g, const fsg_graph *graph, int32_t n_sets,
                           size_t *bytes);
/* dev_mask: device uint8 [n_sets][n] (1 = seed); beta: host float [n_sets]
 * in [0, 1]; dev_prob: device float [n_sets][n] receives p_v.  Synchronous. */
int fsg_gnn_forward(fsg_gnn *g, const fsg_graph *graph, int32_t n_sets, const uint8_t *dev_mask,
                    const float *beta, float *dev_prob, void *ws, size_t ws_bytes, void *stream);
/* One step of mean binary cross-entropy against dev_target (device float
 * [n_sets][n], per-node infection frequencies from Monte Carlo): forward,
 * backward (the mean aggregation is transposed by pulling over `reverse`,
 * the bound graph with every arc reversed), then, if apply_update, Adam with
 * learning rate lr (beta1 0.9, beta2 0.999, eps 1e-8).  The gradient stays
 * readable through fsg_gnn_get_grads; *loss (host, nullable) receives the
 * mean loss.  Synchronous. */
int fsg_gnn_train_step(fsg_gnn *g, const fsg_graph *graph, const fsg_graph *reverse,
                       int32_t n_sets, const uint8_t *dev_mask, const float *beta,
                       const float *dev_target, float lr, int32_t apply_update, float *loss,
                       void *ws, size_t ws_bytes, void *stream);
/* Host copies of the FP32 parameters / last gradient (n = parameter count).
 * fsg_gnn_set_params also zeroes the Adam moments and the step count. */
int fsg_gnn_get_params(const fsg_gnn *g, float *out, int64_t n, void *stream);
int fsg_gnn_set_params(fsg_gnn *g, const float *in, int64_t n, void *stream);
int fsg_gnn_get_grads(const fsg_gnn *g, float *out, int64_t n, void *stream);
/* The optimiser step of fsg_gnn_train_step on its own: Adam (Kingma and Ba,
 * ICLR 2015, Algorithm 1; beta1 0.9, beta2 0.999, eps 1e-8, learning rate
 * lr >= 0) with step count t = previous t + 1, in FP32 on the master
 * parameters:  m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 * p = p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), each operation
 * rounded to FP32; then the BF16 weight copies are refreshed.  dev_grad:
 * device float [parameter count], e.g. a gradient summed over several
 * processes, or NULL for the gradient of the last training step.
 * Synchronous.  Errors: FSG_EINVAL, FSG_EDEVICE. */
int fsg_gnn_apply_update(fsg_gnn *g, const float *dev_grad, float lr, void *stream);
/* Host copies of the optimiser state: Adam moments m and v (FP32 [n] each,
 * n = parameter count), the BF16 weight copies the products read (uint16
 * bit patterns of W1, W2, W3 in that order, row-major, 18432 values) and
 * the step count t; every output may be NULL.  Synchronous. */
int fsg_gnn_get_state(const fsg_gnn *g, float *m, float *v, uint16_t *wb, int64_t *step,
                      int64_t n, void *stream);
/* Acceptance gate and spread calibration of the surrogate (fitted by the
 * caller on simulator labels of training queries and on a held-out split). */
#define FSG_CALIB_TERMS 9
typedef struct {
    double tau;         /* fall back when the members' relative std exceeds tau */
    int64_t min_seeds;  /* fall back for seed sets with fewer distinct nodes */
    int32_t calibrated; /* 1: the ensemble mean is multiplied by exp(sum_i calib[i] f_i) */
    int32_t reserved;   /* 0 */
    /* f = [1, x, x^2, x^3, 1/k, x/k, 1/k^2, ln k, x ln k] with x = 20 beta and
     * k the number of distinct seeds */
    double calib[FSG_CALIB_TERMS];
} fsg_spread_gate;

/* Spread estimate of one SIR query with Monte Carlo fallback: the ensemble
 * members predict sum_v p_v; uncertainty = (sample std / mean) over
 * members.  The estimate is the members' mean, calibrated if the gate says
 * so.  If uncertainty > gate->tau or the seed set has fewer than
 * gate->min_seeds distinct nodes, the plain simulator runs B_fallback
 * replicates (max_steps, rng_key) instead and its mean count is returned
 * with *used_fallback = 1.  An empty seed set gives spread 0.  ws:
 * fsg_gnn_workspace_size for n_sets = 1; sim_ws: fsg_sim_workspace_size for
 * SIR with B_fallback; dev_counts: device uint32 [n]; 1 <= n_members <= 64.
 * Synchronous. */
int fsg_estimate_spread(fsg_gnn *const *members, int32_t n_members, const fsg_graph *graph,
                        const int32_t *seeds, int64_t n_seeds, double beta, double gamma,
                        int64_t max_steps, const fsg_spread_gate *gate, int64_t B_fallback,
                        uint64_t rng_key, void *ws, size_t ws_bytes, void *sim_ws,
                        size_t sim_ws_bytes, uint32_t *dev_counts, double *spread,
                        double *uncertainty, int32_t *used_fallback, void *stream);

/* Row-tile planner (host only; Sec. 3.2, Definition "Target-Node-Based
 * Partitioning via Longest Processing Time Heuristic", kept in CSR order so
 * every part is a contiguous row range).  Row v weighs
 * (indeg(v) > heavy ? 0 : indeg(v)) + row_cost; with prefix weight C_v and
 * total W, row v goes to part ceil(n_parts * C_v / W).  Empty parts are
 * dropped.  bounds_out (host, n + 2 int64) receives the row boundaries
 * 0 = b_0 < b_1 < ... < b_k = n of the k <= n_parts non-empty parts and
 * *n_out = k.  Each part's weight differs from W / n_parts by less than the
 * largest row weight (Proposition "Load Balance Guarantee").
 * Errors: FSG_EINVAL. */
int fsg_plan_row_tiles(const int64_t *in_ptr, int64_t n, int64_t heavy, int64_t row_cost,
                       int64_t n_parts, int64_t *bounds_out, int64_t *n_out);

/* The generator itself: out[4i .. 4i+3] = Philox4x32-10(ctr[4i .. 4i+3],
 * key) for i < count, computed on the device.  dev_ctr and dev_out are
 * device arrays of 4*count uint32.  Asynchronous on `stream`. */
int fsg_philox4x32_10(const uint32_t *dev_ctr, uint32_t key0, uint32_t key1, uint32_t *dev_out,
                      int64_t count, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FSG_H */
