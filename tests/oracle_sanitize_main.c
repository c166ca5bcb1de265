/* Driver of the CPU oracle for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure, compiled and run by
 * tests/test_oracle_sanitizers.py).  It runs every entry point of
 * oracle/fsg_oracle.c on a small graph with the awkward cases -- self-loops,
 * repeated arcs, an isolated node, a hub, a replicate count that is not a
 * multiple of 64, a nonzero replicate offset, a step cap -- and checks a few
 * results that must agree, so a wrong index surfaces as a sanitizer report or
 * a failed check. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_simulate(int model, int ic_prob, double p, const double *edge_p, double beta, double gamma,
                 double alpha, int64_t max_steps, int64_t n, const int64_t *ptr, const int32_t *src,
                 const int32_t *seeds, int64_t n_seeds, int64_t B, int64_t replicate_offset,
                 uint64_t rng_key, uint8_t *states, uint32_t *counts, int64_t *steps_run,
                 int32_t *absorbed, int nthreads);
int orc_ic_live_edge(int ic_prob, double p, const double *edge_p, int64_t max_steps, int64_t n,
                     const int64_t *ptr, const int32_t *src, const int32_t *seeds, int64_t n_seeds,
                     int64_t B, int64_t replicate_offset, uint64_t rng_key, uint8_t *states,
                     uint32_t *counts, int32_t *dist_out, int64_t *steps_run, int32_t *absorbed,
                     int nthreads);
int orc_hk(float eps, int64_t max_steps, int64_t n, const int64_t *ptr, const int32_t *src,
           int64_t B, float *h, int64_t *steps_run, int32_t *converged, int nthreads);
int orc_hk_rows(float eps, int64_t n, const int64_t *ptr, const int32_t *src, int64_t B,
                const float *x, const int64_t *rows, int64_t n_rows, float *out);
uint32_t orc_thr(double p);
void orc_sir_table(double beta, int64_t len, uint32_t *table);
void orc_draw_many(uint64_t rng_key, uint32_t dom, const uint64_t *unit, const uint64_t *g,
                   const uint32_t *step, int64_t count, uint32_t *out);

#define N 40
#define B 70

static int fails = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                  \
        }                                                             \
    } while (0)

int main(void)
{
    /* arcs u -> v: a ring, chords, self-loops, a repeated arc, a hub (node 0
     * pulls from everyone), node 39 isolated */
    int32_t eu[400], ev[400];
    int m = 0;
    for (int i = 0; i < 38; ++i) { eu[m] = i; ev[m++] = (i + 1) % 38; }
    for (int i = 0; i < 38; i += 3) { eu[m] = i; ev[m++] = (i * 7 + 5) % 38; }
    eu[m] = 4; ev[m++] = 4;
    eu[m] = 5; ev[m++] = 6;
    eu[m] = 5; ev[m++] = 6;
    for (int i = 1; i < 38; ++i) { eu[m] = i; ev[m++] = 0; }
    int64_t ptr[N + 1];
    memset(ptr, 0, sizeof(ptr));
    for (int e = 0; e < m; ++e) ptr[ev[e] + 1]++;
    for (int v = 0; v < N; ++v) ptr[v + 1] += ptr[v];
    int32_t *src = malloc(sizeof(int32_t) * m);
    int64_t fill[N];
    memcpy(fill, ptr, sizeof(fill));
    for (int e = 0; e < m; ++e) src[fill[ev[e]]++] = eu[e];
    double *ep = malloc(sizeof(double) * m);
    for (int e = 0; e < m; ++e) ep[e] = (e % 5) / 5.0;
    const int32_t seeds[] = {3, 3, 17, 39};

    uint8_t *st = malloc((size_t)N * B), *st2 = malloc((size_t)N * B);
    uint32_t cnt[N], cnt2[N];
    int64_t steps, steps2;
    int32_t abs1, abs2;
    for (int model = 0; model <= 6; ++model) {
        const int64_t K = (model == 0 || model == 4) ? -1 : 25;
        CHECK(orc_simulate(model, 0, 0.3, NULL, 0.2, 0.15, 0.4, K, N, ptr, src, seeds, 4, B, 3,
                           0x1234ABCDull + (uint64_t)model, st, cnt, &steps, &abs1, 1) == 0);
        for (int v = 0; v < N; ++v) {
            uint32_t c = 0;
            for (int r = 0; r < B; ++r) {
                const uint8_t x = st[v * B + r];
                CHECK(x <= 3);
                c += x != 0;
            }
            if (model == 0 || model == 1 || model == 3 || model == 4 || model == 5) CHECK(c == cnt[v]);
        }
        if (model != 2 && model != 6)  /* a seed keeps a mark unless it can return to S */
            for (int r = 0; r < B; ++r) CHECK(st[39 * B + r] != 0);
    }
    /* IC: the live-edge BFS gives the synchronous loop's states */
    for (int icp = 0; icp <= 2; ++icp) {
        CHECK(orc_simulate(0, icp, 0.35, ep, 0, 0, 0, -1, N, ptr, src, seeds, 4, B, 5, 99, st, cnt,
                           &steps, &abs1, 1) == 0);
        int32_t *dist = malloc(sizeof(int32_t) * N * B);
        CHECK(orc_ic_live_edge(icp, 0.35, ep, -1, N, ptr, src, seeds, 4, B, 5, 99, st2, cnt2, dist,
                               &steps2, &abs2, 1) == 0);
        CHECK(memcmp(st, st2, (size_t)N * B) == 0);
        CHECK(memcmp(cnt, cnt2, sizeof(cnt)) == 0);
        CHECK(steps == steps2 && abs1 == abs2);
        free(dist);
    }
    /* HK: whole steps and the per-row step agree */
    float *h = malloc(sizeof(float) * N * 6), *h1 = malloc(sizeof(float) * N * 6);
    for (int i = 0; i < N * 6; ++i) h[i] = (float)((i * 37) % 101) / 50.0f - 1.0f;
    memcpy(h1, h, sizeof(float) * N * 6);
    int64_t rows[N];
    for (int v = 0; v < N; ++v) rows[v] = v;
    float *row_out = malloc(sizeof(float) * N * 6);
    CHECK(orc_hk_rows(0.5f, N, ptr, src, 6, h, rows, N, row_out) == 0);
    int32_t conv;
    CHECK(orc_hk(0.5f, 1, N, ptr, src, 6, h1, &steps, &conv, 1) == 0);
    CHECK(memcmp(row_out, h1, sizeof(float) * N * 6) == 0);
    CHECK(orc_hk(0.5f, 30, N, ptr, src, 6, h, &steps, &conv, 1) == 0);
    /* tables and draws */
    uint32_t tab[2000];
    orc_sir_table(0.02, 2000, tab);
    for (int k = 1; k < 2000; ++k) CHECK(tab[k] >= tab[k - 1]);
    CHECK(orc_thr(0.0) == 0u && orc_thr(1.0) == 0xFFFFFFFFu && orc_thr(0.5) == 0x80000000u);
    uint64_t unit[9], gg[9];
    uint32_t stp[9], out[9];
    for (int i = 0; i < 9; ++i) { unit[i] = (uint64_t)i << 31; gg[i] = (uint64_t)i * 3; stp[i] = (uint32_t)i; }
    orc_draw_many(7, 2, unit, gg, stp, 9, out);
    CHECK(out[0] != out[1] || out[1] != out[2]);
    /* invalid arguments are refused */
    CHECK(orc_simulate(3, 0, 0, NULL, 0.1, 0.1, 0, -1, N, ptr, src, seeds, 4, B, 0, 1, st, cnt,
                       &steps, &abs1, 1) == -1);
    const int32_t bad[] = {N};
    CHECK(orc_simulate(0, 0, 0.1, NULL, 0, 0, 0, -1, N, ptr, src, bad, 1, B, 0, 1, st, cnt, &steps,
                       &abs1, 1) == -1);
    free(src); free(ep); free(st); free(st2); free(h); free(h1); free(row_out);
    if (fails) return 1;
    printf("oracle sanitizer run ok\n");
    return 0;
}
