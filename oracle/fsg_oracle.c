/*
 * fsg_oracle.c -- plain CPU oracle for batched Monte Carlo graph propagation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP library.
 *
 * What it computes (FS_GPlib, arxiv 2603.14895):
 *   - the traditional mechanism-based propagation loop nest (Algorithm 1):
 *     for every Monte Carlo run, for every step, for every node, look at the
 *     previous-round states of the in-neighbours and update (Eq. nodestate,
 *     Sec. 2, "Paradigm of mechanism-based propagation model");
 *   - SIR exactly as the micro-implementation of Appendix A.1: a susceptible
 *     node with k infected in-neighbours is infected with probability
 *     1 - (1-beta)^k (the log-sum message of A.1 summed over k neighbours),
 *     an infected node recovers with probability gamma;
 *   - SIS / SI (Table tab:29s names them; semantics are the SIR rule with
 *     recovery back to S, resp. no recovery);
 *   - SEIR(DT) / SEIS(DT) (named in Table tab:29s, validated in the
 *     comparison tables of the appendix, not defined by equations there):
 *     the SIR rule with a latent state E between S and I.  A susceptible node
 *     with k infectious in-neighbours becomes E with probability
 *     1 - (1-beta)^k, E becomes I with probability alpha, I becomes R (SEIS:
 *     S) with probability gamma; one draw per node, replicate and step decides
 *     whichever transition the node's state allows, as for SIR;
 *   - independent cascade (Table tab:29s; Kempe et al. cited in Sec. 2): every
 *     newly active node gets one chance per out-arc to activate its target;
 *   - linear threshold with in-weights 1/indeg and U(0,1) thresholds;
 *   - the Hegselmann-Krause opinion model as the micro-implementation of
 *     Appendix A.2 (strict |h_i - h_j| < eps; a node with no eps-neighbour
 *     keeps its opinion), in FP32 with the in-arcs summed in CSR order.
 *
 * Randomness is passed in as a fixed counter-based generator so the result is
 * a deterministic function of the inputs:
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 *   easy as 1, 2, 3", SC'11), written here from that paper's definition.
 *   draw(dom, unit, g, step) = Philox(key = (lo32 key, hi32 key),
 *                                     ctr = (lo32 unit, g >> 2, step,
 *                                            dom << 24 | hi32 unit))[g & 3]
 *   with g the global replicate index.  A Bernoulli(p) trial succeeds iff
 *   t == 0xFFFFFFFF or draw < t, where t = thr(p) is computed in FP64.
 *
 * Everything below is the plain definition: per replicate, per step, per
 * node, per in-edge loops over uint8 states.  No blocking, bit packing or
 * reordering.  OpenMP parallelism is over independent replicates only.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ALWAYS 0xFFFFFFFFu

/* When set, the live-edge BFS reports each finished replicate on stderr. */
static int orc_verbose = 0;
void orc_set_verbose(int on) { orc_verbose = on; }

enum { ORC_IC = 0, ORC_SI = 1, ORC_SIS = 2, ORC_SIR = 3, ORC_LT = 4, ORC_SEIR = 5, ORC_SEIS = 6,
       ORC_SWIR = 7 };
enum { ORC_IC_UNIFORM = 0, ORC_IC_WEIGHTED_CASCADE = 1, ORC_IC_PER_EDGE = 2 };
enum { ORC_DOM_IC_EDGE = 1, ORC_DOM_NODE_STEP = 2, ORC_DOM_LT_THRESH = 3 };

/* ---------------------------------------------------------------- Philox -- */

/* One Philox4x32 round: two 32x32->64 products on words 0 and 2, the high
 * halves xor-ed with the other two words and the key (SC'11, Sec. 4.2). */
static void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

/* Philox4x32 with 10 rounds; the key is bumped by the Weyl constants
 * (golden ratio, sqrt(3)-1) between consecutive rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        philox_round(c, k0, k1);
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

uint32_t orc_draw(uint64_t rng_key, uint32_t dom, uint64_t unit, uint64_t g, uint32_t step)
{
    uint32_t ctr[4] = {(uint32_t)unit, (uint32_t)(g >> 2), step,
                       (dom << 24) | (uint32_t)(unit >> 32)};
    uint32_t key[2] = {(uint32_t)rng_key, (uint32_t)(rng_key >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[g & 3];
}

/* ---------------------------------------------------------- thresholds -- */

/* Probability p -> uint32 threshold: "never" 0, "always" 0xFFFFFFFF,
 * otherwise floor(p * 2^32) kept below the sentinel. */
uint32_t orc_thr(double p)
{
    if (!(p > 0.0)) return 0u;
    if (p >= 1.0) return ORC_ALWAYS;
    double s = floor(p * 4294967296.0);
    if (s > 4294967294.0) s = 4294967294.0;
    return (uint32_t)s;
}

static int fires(uint32_t u, uint32_t t) { return t == ORC_ALWAYS || u < t; }

/* Infection table of Appendix A.1: P(infect | k infected in-neighbours) =
 * 1 - exp(k log(1-beta)) = 1 - (1-beta)^k.  The power is formed by repeated
 * FP64 multiplication (q_0 = 1, q_k = q_{k-1} (1-beta)), then thresholded. */
void orc_sir_table(double beta, int64_t len, uint32_t *table)
{
    double q = 1.0;
    for (int64_t k = 0; k < len; ++k) {
        if (k > 0) {
            volatile double next = q * (1.0 - beta); /* no contraction */
            q = next;
        }
        table[k] = orc_thr(1.0 - q);
    }
}

/* ------------------------------------------------------------ simulator -- */

typedef struct {
    int model, ic_prob;
    double p, beta, gamma;
    const double *edge_p;
    int64_t max_steps; /* < 0: until absorption (IC, LT only) */
    int64_t n;
    const int64_t *ptr;
    const int32_t *src;
    uint64_t rng_key;
    const uint32_t *tinf; /* [max_indeg + 1] */
    uint32_t trec;
    uint32_t talpha; /* SEIR / SEIS: E -> I */
    /* SWIR: S -> I or W with k infectious in-neighbours, W -> I */
    const uint32_t *t_si, *t_siw, *t_wi;
} orc_problem;

/* Models whose states are 0 S, 1 E or W, 2 I, 3 R, with seeds starting in I. */
static int is_latent_model(int model)
{
    return model == ORC_SEIR || model == ORC_SEIS || model == ORC_SWIR;
}

/* Threshold of in-edge e of node v for IC. */
static uint32_t ic_edge_threshold(const orc_problem *P, int64_t v, int64_t e)
{
    if (P->ic_prob == ORC_IC_UNIFORM) return orc_thr(P->p);
    if (P->ic_prob == ORC_IC_PER_EDGE) return orc_thr(P->edge_p[e]);
    /* weighted cascade: p_uv = 1 / indeg(v) */
    int64_t indeg = P->ptr[v + 1] - P->ptr[v];
    return orc_thr(1.0 / (double)indeg);
}

/* States: IC, SI, SIS, SIR, LT: 0 = S / inactive, 1 = I / newly active,
 * 2 = R / active since an earlier step (LT reports 1 for both 1 and 2).
 * SEIR, SEIS: 0 = S, 1 = E, 2 = I, 3 = R.  A run goes on while some node is
 * in a state that can still change others or itself: 1, or for SEIR / SEIS
 * E or I. */
static int has_one(const orc_problem *P, const uint8_t *x, int64_t n)
{
    const int latent = is_latent_model(P->model);
    for (int64_t v = 0; v < n; ++v) {
        if (P->model == ORC_SWIR) {  /* a weakened node alone changes nothing */
            if (x[v] == 2) return 1;
        } else if (x[v] == 1 || (latent && x[v] == 2)) {
            return 1;
        }
    }
    return 0;
}

/* One synchronous step t (t >= 1) of replicate g: y = F(x). */
static void one_step(const orc_problem *P, uint64_t g, uint32_t t, const uint8_t *x, uint8_t *y)
{
    const int64_t n = P->n;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t e0 = P->ptr[v], e1 = P->ptr[v + 1];
        uint8_t xv = x[v], yv = xv;
        if (P->model == ORC_IC) {
            if (xv == 1) {
                yv = 2;
            } else if (xv == 0) {
                for (int64_t e = e0; e < e1; ++e) {
                    if (x[P->src[e]] != 1) continue;
                    uint32_t u = orc_draw(P->rng_key, ORC_DOM_IC_EDGE, (uint64_t)e, g, 0);
                    if (fires(u, ic_edge_threshold(P, v, e))) {
                        yv = 1;
                        break;
                    }
                }
            }
        } else if (P->model == ORC_LT) {
            if (xv != 0) {
                yv = 2;
            } else {
                int64_t c = 0;
                for (int64_t e = e0; e < e1; ++e)
                    if (x[P->src[e]] != 0) ++c;
                int64_t indeg = e1 - e0;
                uint64_t U = orc_draw(P->rng_key, ORC_DOM_LT_THRESH, (uint64_t)v, g, 0);
                /* active-weight c / indeg reaches the threshold U / 2^32 */
                if (c >= 1 && ((uint64_t)c << 32) >= U * (uint64_t)indeg) yv = 1;
            }
        } else if (P->model == ORC_SWIR) {
            /* an infectious node is removed after one step; a susceptible
             * node with k infectious in-neighbours becomes I with probability
             * 1-(1-kappa)^k, else W with probability (1-kappa)^k -
             * (1-kappa-mu)^k (one draw decides both); a weakened one becomes
             * I with probability 1-(1-nu)^k */
            if (xv == 2) {
                yv = 3;
            } else if (xv == 0 || xv == 1) {
                int64_t k = 0;
                for (int64_t e = e0; e < e1; ++e)
                    if (x[P->src[e]] == 2) ++k;
                if (k > 0) {
                    uint32_t U = orc_draw(P->rng_key, ORC_DOM_NODE_STEP, (uint64_t)v, g, t);
                    if (xv == 0) {
                        if (fires(U, P->t_si[k]))
                            yv = 2;
                        else if (fires(U, P->t_siw[k]))
                            yv = 1;
                    } else if (fires(U, P->t_wi[k])) {
                        yv = 2;
                    }
                }
            }
        } else if (is_latent_model(P->model)) { /* SEIR, SEIS */
            uint32_t U = orc_draw(P->rng_key, ORC_DOM_NODE_STEP, (uint64_t)v, g, t);
            if (xv == 0) {
                int64_t k = 0;
                for (int64_t e = e0; e < e1; ++e)
                    if (x[P->src[e]] == 2) ++k;
                if (k > 0 && fires(U, P->tinf[k])) yv = 1;
            } else if (xv == 1) {
                if (fires(U, P->talpha)) yv = 2;
            } else if (xv == 2) {
                if (fires(U, P->trec)) yv = (P->model == ORC_SEIS) ? 0 : 3;
            }
        } else { /* SI, SIS, SIR */
            uint32_t U = orc_draw(P->rng_key, ORC_DOM_NODE_STEP, (uint64_t)v, g, t);
            if (xv == 0) {
                int64_t k = 0;
                for (int64_t e = e0; e < e1; ++e)
                    if (x[P->src[e]] == 1) ++k;
                if (k > 0 && fires(U, P->tinf[k])) yv = 1;
            } else if (xv == 1) {
                if (fires(U, P->trec)) yv = (P->model == ORC_SIS) ? 0 : 2;
            }
        }
        y[v] = yv;
    }
}

/* Runs replicate g from the seeds; returns the number of steps executed. */
static int64_t run_replicate(const orc_problem *P, uint64_t g, const int32_t *seeds, int64_t n_seeds,
                             uint8_t *x, uint8_t *y)
{
    memset(x, 0, (size_t)P->n);
    /* seeds start infectious: state 1, for SEIR / SEIS state 2 (I) */
    for (int64_t i = 0; i < n_seeds; ++i) x[seeds[i]] = is_latent_model(P->model) ? 2 : 1;
    int64_t t = 0;
    while ((P->max_steps < 0 || t < P->max_steps) && has_one(P, x, P->n)) {
        ++t;
        one_step(P, g, (uint32_t)t, x, y);
        memcpy(x, y, (size_t)P->n);
    }
    return t;
}

static int64_t max_indegree(int64_t n, const int64_t *ptr)
{
    int64_t m = 0;
    for (int64_t v = 0; v < n; ++v)
        if (ptr[v + 1] - ptr[v] > m) m = ptr[v + 1] - ptr[v];
    return m;
}

/*
 * Batched Monte Carlo: B replicates with global indices replicate_offset + r.
 * states: [n][B] row-major (states[v*B + r]) or NULL; counts: [n] or NULL.
 * steps_run: the largest step count over replicates (the shared loop of a
 * batch stops when no replicate has a state-1 node, or at max_steps).
 * absorbed: 1 iff no replicate ends with a state-1 node.
 * Returns 0, or -1 on invalid arguments.
 */
int orc_simulate(int model, int ic_prob, double p, const double *edge_p, double beta, double gamma,
                 double alpha, int64_t max_steps, int64_t n, const int64_t *ptr, const int32_t *src,
                 const int32_t *seeds, int64_t n_seeds, int64_t B, int64_t replicate_offset,
                 uint64_t rng_key, uint8_t *states, uint32_t *counts, int64_t *steps_run,
                 int32_t *absorbed, int nthreads)
{
    if (n < 1 || B < 0 || model < ORC_IC || model > ORC_SWIR) return -1;
    if (model != ORC_IC && model != ORC_LT && model != ORC_SWIR && max_steps < 0) return -1;
    if (model == ORC_SWIR && !(beta + alpha <= 1.0)) return -1;
    for (int64_t i = 0; i < n_seeds; ++i)
        if (seeds[i] < 0 || seeds[i] >= n) return -1;

    int64_t dmax = max_indegree(n, ptr);
    uint32_t *tinf = (uint32_t *)calloc((size_t)(dmax + 1), sizeof(uint32_t));
    orc_sir_table(beta, dmax + 1, tinf);
    orc_problem P = {model, ic_prob, p, beta, (model == ORC_SI) ? 0.0 : gamma, edge_p, max_steps,
                     n, ptr, src, rng_key, tinf, 0, 0, NULL, NULL, NULL};
    P.trec = orc_thr(P.gamma);
    P.talpha = orc_thr(alpha);
    /* SWIR: kappa = beta (S -> I), mu = alpha (S -> W), nu = gamma (W -> I) */
    uint32_t *t_siw = (uint32_t *)calloc((size_t)(dmax + 1), sizeof(uint32_t));
    uint32_t *t_wi = (uint32_t *)calloc((size_t)(dmax + 1), sizeof(uint32_t));
    if (model == ORC_SWIR) {
        orc_sir_table(beta + alpha, dmax + 1, t_siw);
        orc_sir_table(gamma, dmax + 1, t_wi);
    }
    P.t_si = tinf;
    P.t_siw = t_siw;
    P.t_wi = t_wi;

    int64_t smax = 0;
    int any_one = 0;
    if (counts) memset(counts, 0, (size_t)n * sizeof(uint32_t));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel reduction(max : smax) reduction(| : any_one)
#endif
    {
        uint8_t *x = (uint8_t *)malloc((size_t)n);
        uint8_t *y = (uint8_t *)malloc((size_t)n);
        uint32_t *cnt = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t r = 0; r < B; ++r) {
            int64_t t = run_replicate(&P, (uint64_t)(replicate_offset + r), seeds, n_seeds, x, y);
            if (t > smax) smax = t;
            if (has_one(&P, x, n)) any_one = 1;
            for (int64_t v = 0; v < n; ++v) {
                uint8_t s = x[v];
                uint8_t out = (model == ORC_LT) ? (uint8_t)(s != 0) : s;
                if (states) states[v * B + r] = out;
                /* counted: IC ever active; SIR/SI ever infected; SIS infected
                 * at the end; LT active; SEIR ever exposed; SEIS exposed or
                 * infectious at the end; SWIR ever weakened or infected */
                int counted = (model == ORC_SIS)    ? (s == 1)
                              : (model == ORC_SEIS) ? (s == 1 || s == 2)
                                                    : (s != 0);
                cnt[v] += (uint32_t)counted;
            }
        }
        if (counts) {
#ifdef _OPENMP
#pragma omp critical
#endif
            for (int64_t v = 0; v < n; ++v) counts[v] += cnt[v];
        }
        free(cnt);
        free(y);
        free(x);
    }
    free(tinf);
    free(t_siw);
    free(t_wi);
    if (steps_run) *steps_run = smax;
    if (absorbed) *absorbed = !any_one;
    return 0;
}

/*
 * IC by breadth-first search in the live-edge graph.  Because an edge draw
 * does not depend on the step and an arc is consulted only in the one step
 * after its source became newly active, synchronous IC activates node v at
 * exactly its hop distance from the seed set in the graph of live arcs
 * {e : fires(draw(IC_EDGE, e, g, 0), t_e)}.  This is a second, independent
 * algorithm for the same final states (and it is work-efficient, so it also
 * serves at sizes the plain loop nest cannot reach).
 * dist: optional [n][B] int32, -1 for unreached.
 */
int orc_ic_live_edge(int ic_prob, double p, const double *edge_p, int64_t max_steps, int64_t n,
                     const int64_t *ptr, const int32_t *src, const int32_t *seeds, int64_t n_seeds,
                     int64_t B, int64_t replicate_offset, uint64_t rng_key, uint8_t *states,
                     uint32_t *counts, int32_t *dist_out, int64_t *steps_run, int32_t *absorbed,
                     int nthreads)
{
    if (n < 1 || B < 0) return -1;
    for (int64_t i = 0; i < n_seeds; ++i)
        if (seeds[i] < 0 || seeds[i] >= n) return -1;
    int64_t nnz = ptr[n];
    /* out-arc lists with the in-CSR position of each arc (its edge id) */
    int64_t *optr = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int32_t *odst = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int64_t *oeid = (int64_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
    for (int64_t e = 0; e < nnz; ++e) optr[src[e] + 1]++;
    for (int64_t v = 0; v < n; ++v) optr[v + 1] += optr[v];
    int64_t *fill = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    memcpy(fill, optr, (size_t)(n + 1) * sizeof(int64_t));
    for (int64_t v = 0; v < n; ++v)
        for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) {
            int64_t pos = fill[src[e]]++;
            odst[pos] = (int32_t)v;
            oeid[pos] = e;
        }
    free(fill);
    orc_problem P = {ORC_IC, ic_prob, p, 0.0, 0.0, edge_p, max_steps, n, ptr, src, rng_key, NULL, 0, 0,
                     NULL, NULL, NULL};

    int64_t smax = 0;
    int any_one = 0;
    if (counts) memset(counts, 0, (size_t)n * sizeof(uint32_t));
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel reduction(max : smax) reduction(| : any_one)
#endif
    {
        int32_t *dist = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        uint32_t *cnt = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
        for (int64_t v = 0; v < n; ++v) dist[v] = -1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int64_t r = 0; r < B; ++r) {
            uint64_t g = (uint64_t)(replicate_offset + r);
            int64_t head = 0, tail = 0;
            for (int64_t i = 0; i < n_seeds; ++i)
                if (dist[seeds[i]] < 0) {
                    dist[seeds[i]] = 0;
                    queue[tail++] = seeds[i];
                }
            int64_t dmax = -1;
            while (head < tail) {
                int32_t u = queue[head++];
                if (dist[u] > dmax) dmax = dist[u];
                /* arcs past the step cap are never consulted */
                if (max_steps >= 0 && dist[u] >= max_steps) continue;
                for (int64_t k = optr[u]; k < optr[u + 1]; ++k) {
                    int32_t v = odst[k];
                    if (dist[v] >= 0) continue;
                    uint32_t dr = orc_draw(rng_key, ORC_DOM_IC_EDGE, (uint64_t)oeid[k], g, 0);
                    if (fires(dr, ic_edge_threshold(&P, v, oeid[k]))) {
                        dist[v] = dist[u] + 1;
                        queue[tail++] = v;
                    }
                }
            }
            /* steps this replicate runs: one past its deepest level, capped */
            int64_t T = (tail == 0) ? 0 : dmax + 1;
            if (max_steps >= 0 && T > max_steps) T = max_steps;
            if (T > smax) smax = T;
            for (int64_t i = 0; i < tail; ++i) {
                int32_t v = queue[i];
                uint8_t s = (dist[v] < T) ? 2 : (dist[v] == T ? 1 : 0);
                if (s == 1) any_one = 1;
                if (s != 0) cnt[v] += 1;
                if (states) states[(int64_t)v * B + r] = s;
                if (dist_out) dist_out[(int64_t)v * B + r] = dist[v];
            }
            /* unreached nodes (and nodes cut off by the cap) */
            if (states || dist_out) {
                for (int64_t v = 0; v < n; ++v)
                    if (dist[v] < 0) {
                        if (states) states[v * B + r] = 0;
                        if (dist_out) dist_out[v * B + r] = -1;
                    }
            }
            for (int64_t i = 0; i < tail; ++i) dist[queue[i]] = -1;
            if (orc_verbose) {
                fprintf(stderr, "[oracle] live-edge replicate %lld: %lld reached, depth %lld\n",
                        (long long)g, (long long)tail, (long long)dmax);
                fflush(stderr);
            }
        }
        if (counts) {
#ifdef _OPENMP
#pragma omp critical
#endif
            for (int64_t v = 0; v < n; ++v) counts[v] += cnt[v];
        }
        free(cnt);
        free(queue);
        free(dist);
    }
    free(oeid);
    free(odst);
    free(optr);
    if (steps_run) *steps_run = smax;
    if (absorbed) *absorbed = !any_one;
    return 0;
}

/* Bulk draws for statistical tests of the generator. */
void orc_draw_many(uint64_t rng_key, uint32_t dom, const uint64_t *unit, const uint64_t *g,
                   const uint32_t *step, int64_t count, uint32_t *out)
{
    for (int64_t i = 0; i < count; ++i) out[i] = orc_draw(rng_key, dom, unit[i], g[i], step[i]);
}


/*
 * Hegselmann-Krause (Appendix A.2): per replicate r and step, every node i
 * sums the opinions h_j of the in-neighbours j (arcs j -> i, CSR order, with
 * multiplicity) with |h_i - h_j| < eps and counts them; the new opinion is
 * the sum divided by the count, or the old opinion when the count is 0.
 * FP32 throughout (IEEE single, round to nearest), no contraction.
 * h: [n][B] row-major, initial opinions on entry, final ones on return.
 * The loop stops after max_steps steps or after a step that changed no
 * opinion in any replicate; *steps_run counts the steps executed (the last,
 * unchanged one included), *converged = 1 iff it stopped on no change.
 */
/* New opinion of node v in replicate r from the opinions x [n][B]. */
static float hk_node(float eps, const int64_t *ptr, const int32_t *src, int64_t B, const float *x,
                     int64_t v, int64_t r);

/* Weighted HK: node v moves the fraction mu of the way from its opinion h
 * to the HK mean m of its eps-neighbourhood: (1 - mu) h + mu m, each product
 * and the sum rounded to single precision; h itself when no in-neighbour is
 * within eps.  mu = 1 is plain HK. */
static float whk_node(float eps, float mu, const int64_t *ptr, const int32_t *src, int64_t B,
                      const float *x, int64_t v, int64_t r)
{
    const float hv = x[v * B + r];
    const float m = hk_node(eps, ptr, src, B, x, v, r);
    if (mu == 1.0f) return m;
    int any = 0;
    for (int64_t e = ptr[v]; e < ptr[v + 1] && !any; ++e)
        if (fabsf(hv - x[(int64_t)src[e] * B + r]) < eps) any = 1;
    if (!any) return hv;
    const float one_minus = 1.0f - mu;
    volatile float a = one_minus * hv; /* no contraction */
    volatile float b = mu * m;
    return a + b;
}

static float hk_node(float eps, const int64_t *ptr, const int32_t *src, int64_t B, const float *x,
                     int64_t v, int64_t r)
{
    const float hv = x[v * B + r];
    float mc = 0.0f;
    int64_t mv = 0;
    for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e) {
        const float hj = x[(int64_t)src[e] * B + r];
        if (fabsf(hv - hj) < eps) {
            mc += hj;
            ++mv;
        }
    }
    return mv > 0 ? mc / (float)mv : hv;
}

/* One step for the listed rows only: out[i][r] = new opinion of rows[i]. */
int orc_hk_rows(float eps, int64_t n, const int64_t *ptr, const int32_t *src, int64_t B,
                const float *x, const int64_t *rows, int64_t n_rows, float *out)
{
    if (n < 1 || B < 0) return -1;
    for (int64_t i = 0; i < n_rows; ++i) {
        if (rows[i] < 0 || rows[i] >= n) return -1;
        for (int64_t r = 0; r < B; ++r) out[i * B + r] = hk_node(eps, ptr, src, B, x, rows[i], r);
    }
    return 0;
}

int orc_whk(float eps, float mu, int64_t max_steps, int64_t n, const int64_t *ptr,
            const int32_t *src, int64_t B, float *h, int64_t *steps_run, int32_t *converged,
            int nthreads)
{
    if (n < 1 || B < 0 || max_steps < 0 || !(mu >= 0.0f && mu <= 1.0f)) return -1;
    float *x = (float *)malloc((size_t)n * (size_t)B * sizeof(float));
    float *y = (float *)malloc((size_t)n * (size_t)B * sizeof(float));
    memcpy(x, h, (size_t)n * (size_t)B * sizeof(float));
    int64_t t = 0;
    int changed = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    while (t < max_steps && changed) {
        ++t;
        changed = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(| : changed)
#endif
        for (int64_t r = 0; r < B; ++r) {
            for (int64_t v = 0; v < n; ++v) {
                const float nv = whk_node(eps, mu, ptr, src, B, x, v, r);
                y[v * B + r] = nv;
                if (nv != x[v * B + r]) changed = 1;
            }
        }
        float *tmp = x;
        x = y;
        y = tmp;
    }
    memcpy(h, x, (size_t)n * (size_t)B * sizeof(float));
    free(x);
    free(y);
    if (steps_run) *steps_run = t;
    if (converged) *converged = !changed;
    return 0;
}

int orc_hk(float eps, int64_t max_steps, int64_t n, const int64_t *ptr, const int32_t *src,
           int64_t B, float *h, int64_t *steps_run, int32_t *converged, int nthreads)
{
    return orc_whk(eps, 1.0f, max_steps, n, ptr, src, B, h, steps_run, converged, nthreads);
}
