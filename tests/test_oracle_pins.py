"""Pins of the CPU oracle against things fixed outside the oracle itself:
published Philox test vectors, exact integer identities of the threshold
rule, closed forms of the propagation models, exhaustive enumeration of
live-edge worlds and exact Markov chains on tiny graphs.

Monte Carlo checks use fixed keys, so they are deterministic; the bound
|z| < 5 is on binomial z-scores against exact probabilities.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import twin
from paper_2603_14895_amd import workloads as W
from tests import oracle_exact as X

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ZMAX = 5.0


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            h = [int(x, 16) for x in line.split()]
            rows.append((h[0:4], h[4:6], h[6:10]))
    return rows


# ------------------------------------------------------------------ Philox --

def test_philox_kat_c_and_twin():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle.philox4x32_10(ctr, key) == out
        assert twin.philox4x32_10(ctr, key) == out


def test_draw_counter_layout():
    """draw() picks word g&3 of the block with counter (lo unit, g>>2, step,
    dom<<24 | hi unit) -- checked against the raw generator."""
    key = 0x0123456789ABCDEF
    for dom, unit, g, step in [(1, 5, 0, 0), (2, 2**33 + 7, 13, 9), (3, 99, 2**20 + 3, 0)]:
        blk = oracle.philox4x32_10(
            [unit & 0xFFFFFFFF, g >> 2, step, (dom << 24) | (unit >> 32)],
            [key & 0xFFFFFFFF, key >> 32])
        assert oracle.draw(key, dom, unit, g, step) == blk[g & 3]
        assert twin.draw(key, dom, unit, g, step) == blk[g & 3]


def test_draw_uniformity_and_independence():
    """Chi-square on 256 bins per output lane and lag-1 correlation across
    adjacent counters (a wrong multiplier or a missing round fails this)."""
    n = 1 << 18
    unit = np.arange(n, dtype=np.uint64)
    for g in range(4):
        u = oracle.draw_many(0xDEADBEEF12345678, 2, unit, g, 7).astype(np.float64)
        hist = np.bincount((u / 2**24).astype(np.int64), minlength=256)
        exp = n / 256
        chi2 = ((hist - exp) ** 2 / exp).sum()
        assert chi2 < 255 + 6 * math.sqrt(2 * 255)
        x = u / 2**32 - 0.5
        corr = (x[1:] * x[:-1]).mean() / x.var()
        assert abs(corr) < 5 / math.sqrt(n)
        assert abs(u.mean() / 2**32 - 0.5) < 5 * math.sqrt(1 / 12 / n)


# ---------------------------------------------------------------- thresholds --

def test_thr_values():
    A = 0xFFFFFFFF
    assert oracle.thr(0.0) == 0 and oracle.thr(-1.0) == 0
    assert oracle.thr(1.0) == A and oracle.thr(2.0) == A
    assert oracle.thr(0.5) == 2**31
    assert oracle.thr(0.25) == 2**30
    # p just below one keeps clear of the "always" sentinel
    assert oracle.thr(1.0 - 2**-53) == 0xFFFFFFFE
    # thr(p) = floor(p * 2^32) exactly, from the exact rational value of p
    for p in [0.1, 0.05, 0.02, 0.03, 0.3333, 1e-9, 0.999999]:
        assert oracle.thr(p) == math.floor(Fraction(p) * 2**32)
        assert twin.thr(p) == oracle.thr(p)


def test_weighted_cascade_threshold_is_integer_division():
    """thr(1/d) in FP64 equals the exact floor(2^32 / d) for every d >= 2 (the
    reciprocal's rounding error is far below the distance to the next
    integer), and d = 1 is the always sentinel."""
    assert oracle.thr(1.0 / 1) == 0xFFFFFFFF
    ds = list(range(2, 5000)) + [2**k + j for k in range(12, 31) for j in (-1, 0, 1)]
    for d in ds:
        assert oracle.thr(1.0 / d) == (2**32) // d, d


def test_sir_table_against_exact_powers():
    """T[k] = thr(1 - (1-beta)^k) (Appendix A.1 with k infected neighbours);
    the FP64 power is within one unit of the exact rational threshold."""
    for beta in [0.02, 0.03, 0.01, 0.5, 0.05]:
        L = 400
        t = oracle.sir_table(beta, L)
        assert list(t[:60]) == twin.sir_table(beta, 60)
        assert t[0] == 0
        assert (np.diff(t.astype(np.int64)) >= 0).all()
        b = Fraction(beta)
        q = Fraction(1)
        for k in range(L):
            if k:
                q *= 1 - b
            exact = math.floor((1 - q) * 2**32)
            exact = min(exact, 0xFFFFFFFE)
            assert abs(int(t[k]) - exact) <= 1, (beta, k)
    # beta = 1: a single infected neighbour always infects
    t = oracle.sir_table(1.0, 4)
    assert list(t) == [0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]
    t = oracle.sir_table(0.0, 4)
    assert list(t) == [0, 0, 0, 0]


# ------------------------------------------------------------- twin vs C --

def _tiny_graphs():
    rng = np.random.default_rng(7)
    out = []
    for n, m in [(1, 0), (2, 1), (5, 7), (8, 20), (12, 30)]:
        edges = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(m)]
        out.append(W.from_edges(n, edges))
    # self-loop, multi-edge and an isolated node
    out.append(W.from_edges(5, [(0, 1), (0, 1), (1, 1), (1, 2), (2, 3), (3, 1)]))
    return out


@pytest.mark.parametrize("model", ["ic", "sir", "sis", "si", "lt"])
def test_twin_matches_c_oracle(model):
    for gi, gr in enumerate(_tiny_graphs()):
        ptr, src = gr.numpy()
        seeds = np.array([0, gr.n - 1, 0], dtype=np.int32)
        kw = dict(p=0.4, beta=0.3, gamma=0.25,
                  max_steps=-1 if model in ("ic", "lt") else 6, replicate_offset=5 + gi)
        if model == "ic" and gi % 2:
            kw.update(ic_prob=oracle.IC_WEIGHTED_CASCADE)
        s1, c1, st1, a1 = oracle.simulate(model, ptr, src, seeds, 9, 0xABCDEF0123 + gi, **kw)
        s2, c2, st2, a2 = twin.simulate(oracle.native.MODEL_NAMES[model], ptr, src, seeds, 9,
                                        0xABCDEF0123 + gi, **kw)
        assert (s1 == np.array(s2, dtype=np.uint8)).all()
        assert list(c1) == c2 and st1 == st2 and a1 == a2


# -------------------------------------------------------------- IC pins --

def test_ic_directed_path_closed_form():
    """Directed path 0->1->...->L from seed 0: P[node k active] = p^k and its
    activation step is exactly k."""
    L, p, B = 7, 0.7, 40000
    gr = W.from_edges(L + 1, [(i, i + 1) for i in range(L)])
    ptr, src = gr.numpy()
    st, cnt, steps, absorbed = oracle.simulate("ic", ptr, src, [0], B, 0x1111, p=p)
    assert absorbed == 1 and steps <= L + 1
    for k in range(L + 1):
        z = X.zscore(cnt[k] / B, p ** k, B)
        assert abs(z) < ZMAX, (k, cnt[k] / B, p ** k)
    # activation step: with the step cap K = k, node k is newly active (1)
    # exactly when reached, never earlier
    for K in (1, 3):
        sK, _, _, _ = oracle.simulate("ic", ptr, src, [0], 2000, 0x1111, p=p, max_steps=K)
        reached = st[K] != 0
        assert ((sK[K] == 1) == reached[:2000]).all()
        assert (sK[K + 1:] == 0).all()


def test_ic_in_star_and_out_star():
    s, p, B = 6, 0.3, 40000
    # in-star: leaves 1..s -> centre 0, all leaves seeded
    gr = W.from_edges(s + 1, [(i, 0) for i in range(1, s + 1)])
    ptr, src = gr.numpy()
    _, cnt, steps, _ = oracle.simulate("ic", ptr, src, list(range(1, s + 1)), B, 0x2222, p=p)
    assert abs(X.zscore(cnt[0] / B, 1 - (1 - p) ** s, B)) < ZMAX
    assert steps == 2
    # out-star from a seeded centre: the number of active leaves is Binomial(s, p)
    gr = W.from_edges(s + 1, [(0, i) for i in range(1, s + 1)])
    ptr, src = gr.numpy()
    st, _, _, _ = oracle.simulate("ic", ptr, src, [0], B, 0x3333, p=p)
    k = (st[1:] != 0).sum(axis=0)
    hist = np.bincount(k, minlength=s + 1)
    exp = np.array([math.comb(s, j) * p ** j * (1 - p) ** (s - j) for j in range(s + 1)]) * B
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < s + 6 * math.sqrt(2 * s)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ic_brute_force_live_edge_worlds(seed):
    """All 2^|E| live-edge worlds of a random graph with <= 14 arcs give exact
    activation probabilities and exact activation-step distributions."""
    rng = np.random.default_rng(100 + seed)
    n, m = 7, 13
    edges = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(m)]
    gr = W.from_edges(n, edges)
    ptr, src = gr.numpy()
    eprob = rng.uniform(0.1, 0.9, size=m)
    seeds = [0, 3]
    p_act, p_dist = X.ic_exact_marginals(n, ptr, src, seeds, eprob)
    B = 40000
    st, cnt, _, _ = oracle.simulate("ic", ptr, src, seeds, B, 0x4444 + seed,
                                    ic_prob=oracle.IC_PER_EDGE, edge_p=eprob)
    for v in range(n):
        assert abs(X.zscore(cnt[v] / B, p_act[v], B)) < ZMAX, (v, cnt[v] / B, p_act[v])
    # activation step distribution from the live-edge BFS's distances
    _, _, dist, _, _ = oracle.ic_live_edge(ptr, src, seeds, B, 0x4444 + seed,
                                           ic_prob=oracle.IC_PER_EDGE, edge_p=eprob,
                                           want_dist=True)
    for v in range(n):
        for d in range(n):
            f = (dist[v] == d).mean()
            assert abs(X.zscore(f, p_dist[v, d], B)) < ZMAX, (v, d)


@pytest.mark.parametrize("ic_prob", [oracle.IC_UNIFORM, oracle.IC_WEIGHTED_CASCADE, oracle.IC_PER_EDGE])
@pytest.mark.parametrize("K", [-1, 0, 1, 2, 4])
def test_ic_live_edge_bfs_equals_synchronous_loop(ic_prob, K):
    """Second algorithm, same answer: states, counts, steps and absorption of
    the plain synchronous loop equal BFS in the live-edge graph, bit for bit."""
    gr = W.chung_lu(400, 6.0, 2.5, 11)
    ptr, src = gr.numpy()
    ep = np.random.default_rng(3).uniform(0, 0.5, size=gr.nnz)
    seeds = W.uniform_seeds(gr.n, 5, 12)
    kw = dict(p=0.15, ic_prob=ic_prob, edge_p=ep, max_steps=K, replicate_offset=77)
    a = oracle.simulate("ic", ptr, src, seeds, 70, 0x5555, **kw)
    b = oracle.ic_live_edge(ptr, src, seeds, 70, 0x5555, **kw)
    assert (a[0] == b[0]).all()
    assert (a[1] == b[1]).all()
    assert a[2] == b[3] and a[3] == b[4]


def test_ic_weighted_cascade_in_arc_weights_and_chains():
    """Weighted cascade: on an in-degree-1 chain every arc is certain; at a
    node of in-degree d with all d sources seeded, P = 1 - (1 - 1/d)^d."""
    gr = W.from_edges(6, [(i, i + 1) for i in range(5)])
    ptr, src = gr.numpy()
    st, cnt, steps, _ = oracle.simulate("ic", ptr, src, [0], 50, 9,
                                        ic_prob=oracle.IC_WEIGHTED_CASCADE)
    assert (cnt == 50).all() and steps == 6
    d, B = 5, 40000
    gr = W.from_edges(d + 1, [(i, 0) for i in range(1, d + 1)])
    ptr, src = gr.numpy()
    _, cnt, _, _ = oracle.simulate("ic", ptr, src, list(range(1, d + 1)), B, 10,
                                   ic_prob=oracle.IC_WEIGHTED_CASCADE)
    assert abs(X.zscore(cnt[0] / B, 1 - (1 - 1 / d) ** d, B)) < ZMAX


# ------------------------------------------------------------- SIR pins --

@pytest.mark.parametrize("K", [1, 3, 8, 25])
def test_sir_single_edge_closed_form(K):
    """u -> v, u infected at step 0: v is infected at step t iff u stayed
    infectious through t-1 and v escaped the first t-1 contacts, so
    P[v ever infected by K] = beta * (1 - ((1-beta)(1-gamma))^K) / (1 - (1-beta)(1-gamma))."""
    beta, gamma, B = 0.2, 0.15, 40000
    gr = W.from_edges(2, [(0, 1)])
    ptr, src = gr.numpy()
    _, cnt, _, _ = oracle.simulate("sir", ptr, src, [0], B, 0x6666, beta=beta, gamma=gamma,
                                   max_steps=K)
    a = (1 - beta) * (1 - gamma)
    pk = beta * (1 - a ** K) / (1 - a)
    assert abs(X.zscore(cnt[1] / B, pk, B)) < ZMAX


def test_sir_no_transmission_recovery_is_geometric():
    """beta = 0: the seed stays infected through t steps with probability (1-gamma)^t."""
    gamma, B = 0.1, 40000
    gr = W.from_edges(3, [(0, 1), (1, 2), (2, 0)])
    ptr, src = gr.numpy()
    for K in (1, 5, 12):
        st, _, _, _ = oracle.simulate("sir", ptr, src, [0], B, 0x7777, beta=0.0, gamma=gamma,
                                      max_steps=K)
        assert abs(X.zscore((st[0] == 1).mean(), (1 - gamma) ** K, B)) < ZMAX
        assert (st[1:] == 0).all()


def test_si_deterministic_layers():
    """SI with beta = 1: infection spreads one hop per step along arcs."""
    gr = W.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)])
    ptr, src = gr.numpy()
    for K in range(6):
        st, _, _, _ = oracle.simulate("si", ptr, src, [0], 4, 1, beta=1.0, gamma=0.5, max_steps=K)
        assert (st[: K + 1] == 1).all() and (st[K + 1:] == 0).all()


@pytest.mark.parametrize("model", ["sir", "sis"])
@pytest.mark.parametrize("case", [0, 1])
def test_epidemic_exact_markov_chain(model, case):
    """Per-node state marginals after K steps equal those of the exact
    synchronous Markov chain over all joint states."""
    rng = np.random.default_rng(50 + case)
    n = 5
    edges = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(9)] + [(0, 1), (1, 0)]
    gr = W.from_edges(n, edges)
    ptr, src = gr.numpy()
    beta, gamma, K, B = 0.35, 0.3, 4, 40000
    marg = X.epidemic_exact_marginals(n, ptr, src, [0], beta, gamma, K, sis=(model == "sis"))
    st, _, _, _ = oracle.simulate(model, ptr, src, [0], B, 0x8888 + case, beta=beta,
                                  gamma=gamma, max_steps=K)
    for v in range(n):
        for s in range(3):
            f = (st[v] == s).mean()
            assert abs(X.zscore(f, marg[v, s], B)) < ZMAX, (v, s, f, marg[v, s])


# ---------------------------------------------------- SEIR / SEIS pins --

@pytest.mark.parametrize("model", ["seir", "seis"])
@pytest.mark.parametrize("case", [0, 1])
def test_latent_exact_markov_chain(model, case):
    """Per-node marginals of the four states after K steps equal those of the
    exact synchronous SEIR / SEIS chain over all 4^n joint states."""
    rng = np.random.default_rng(150 + case)
    n = 5
    edges = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(9)] + [(0, 1), (1, 0)]
    gr = W.from_edges(n, edges)
    ptr, src = gr.numpy()
    beta, alpha, gamma, K, B = 0.4, 0.5, 0.3, 5, 40000
    marg = X.latent_exact_marginals(n, ptr, src, [0], beta, alpha, gamma, K,
                                    seis=(model == "seis"))
    st, _, _, _ = oracle.simulate(model, ptr, src, [0], B, 0x5E1 + case, beta=beta,
                                  alpha=alpha, gamma=gamma, max_steps=K)
    for v in range(n):
        for s in range(4):
            f = (st[v] == s).mean()
            assert abs(X.zscore(f, marg[v, s], B)) < ZMAX, (v, s, f, marg[v, s])


def test_seir_single_edge_closed_form():
    """Arc 0 -> 1, seed 0 infectious: node 1 is ever exposed with probability
    beta / (1 - (1-beta)(1-gamma)) (the seed transmits with probability beta
    in every step it is still infectious); with K large every exposed node
    ends recovered."""
    gr = W.from_edges(2, [(0, 1)])
    ptr, src = gr.numpy()
    beta, alpha, gamma, B = 0.3, 0.4, 0.2, 100000
    T = beta / (1.0 - (1.0 - beta) * (1.0 - gamma))
    st, cnt, steps, absorbed = oracle.simulate("seir", ptr, src, [0], B, 0x5E2, beta=beta,
                                               alpha=alpha, gamma=gamma, max_steps=400)
    assert absorbed == 1
    assert abs(X.zscore(cnt[1] / B, T, B)) < ZMAX
    assert set(np.unique(st[1]).tolist()) <= {0, 3} and (st[0] == 3).all()
    assert (cnt[1] == (st[1] == 3).sum())


def test_seir_no_infection_decay():
    """beta = 0: nobody is exposed; a seed is still infectious after K steps
    with probability (1-gamma)^K."""
    gr = W.from_edges(3, [(0, 1), (1, 2), (0, 2)])
    ptr, src = gr.numpy()
    gamma, K, B = 0.15, 6, 100000
    st, _, _, _ = oracle.simulate("seir", ptr, src, [0], B, 0x5E3, beta=0.0, alpha=0.5,
                                  gamma=gamma, max_steps=K)
    assert abs(X.zscore((st[0] == 2).mean(), (1 - gamma) ** K, B)) < ZMAX
    assert (st[1:] == 0).all()


def test_seir_deterministic_latency():
    """beta = alpha = 1, gamma = 0 on a path: hop d is exposed at step 2d - 1
    and infectious from step 2d on (one step in E)."""
    gr = W.from_edges(5, [(0, 1), (1, 2), (2, 3), (3, 4)])
    ptr, src = gr.numpy()
    for K in range(9):
        st, _, _, _ = oracle.simulate("seir", ptr, src, [0], 3, 7, beta=1.0, alpha=1.0,
                                      gamma=0.0, max_steps=K)
        for d in range(5):
            want = 2 if (d == 0 or K >= 2 * d) else (1 if K == 2 * d - 1 else 0)
            assert (st[d] == want).all(), (K, d, st[d], want)


# ----------------------------------------------------------- SWIR pins --

@pytest.mark.parametrize("case", [0, 1])
def test_swir_exact_markov_chain(case):
    """Per-node marginals of S, W, I, R after K steps equal those of the
    exact synchronous SWIR chain over all 4^n joint states (the weakened
    state needs two infectious contacts in different steps, so a node reached
    by two paths carries the nu term)."""
    rng = np.random.default_rng(250 + case)
    n = 5
    edges = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(9)] + \
        [(0, 1), (0, 2), (2, 1), (1, 3)]
    gr = W.from_edges(n, edges)
    ptr, src = gr.numpy()
    kappa, mu, nu, K, B = 0.3, 0.35, 0.5, 4, 40000
    marg = X.swir_exact_marginals(n, ptr, src, [0], kappa, mu, nu, K)
    st, _, _, _ = oracle.simulate("swir", ptr, src, [0], B, 0x5A1 + case, beta=kappa, alpha=mu,
                                  gamma=nu, max_steps=K)
    for v in range(n):
        for s in range(4):
            f = (st[v] == s).mean()
            assert abs(X.zscore(f, marg[v, s], B)) < ZMAX, (v, s, f, marg[v, s])


def test_swir_without_weakening_is_sir_with_one_step_recovery():
    """mu = 0: no node is ever weakened, and SWIR(kappa, 0, nu) is SIR with
    beta = kappa and gamma = 1 (recovery after exactly one step) under the
    same draws, bit for bit (SWIR's I and R are SIR's 1 and 2)."""
    gr = W.chung_lu(400, 8.0, 2.5, 251)
    ptr, src = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 6, 252)
    a, ac, asteps, aab = oracle.simulate("swir", ptr, src, seeds, 96, 0x5A2, beta=0.2, alpha=0.0,
                                         gamma=0.7, max_steps=-1)
    b, bc, bsteps, bab = oracle.simulate("sir", ptr, src, seeds, 96, 0x5A2, beta=0.2, gamma=1.0,
                                         max_steps=400)
    assert (a != 1).all()
    relabel = np.array([0, 2, 3], dtype=np.uint8)
    assert (a == relabel[b]).all()
    assert (ac == bc).all() and asteps == bsteps and aab == bab == 1


def test_swir_single_edge_closed_form():
    """Arc 0 -> 1, seed 0: the seed is removed after one step, so node 1 gets
    one contact: it ends weakened with probability mu, removed (infected at
    step 1) with probability kappa, susceptible otherwise; the run absorbs at
    step 2 (or 1 when node 1 is not infected)."""
    gr = W.from_edges(2, [(0, 1)])
    ptr, src = gr.numpy()
    kappa, mu, nu, B = 0.25, 0.4, 0.9, 100000
    st, cnt, steps, absorbed = oracle.simulate("swir", ptr, src, [0], B, 0x5A3, beta=kappa,
                                               alpha=mu, gamma=nu, max_steps=-1)
    assert absorbed == 1 and steps == 2 and (st[0] == 3).all()
    assert abs(X.zscore((st[1] == 1).mean(), mu, B)) < ZMAX
    assert abs(X.zscore((st[1] == 3).mean(), kappa, B)) < ZMAX
    assert cnt[1] == (st[1] != 0).sum()


def test_swir_weakened_then_infected_closed_form():
    """Seed 0 -> 1 and 0 -> 2 -> 1: node 1 is infected either at step 1
    (kappa), or, if weakened at step 1 (mu) and node 2 infected at step 1
    (kappa), at step 2 with nu; if still susceptible and node 2 infected, at
    step 2 with kappa.  P[1 ever infected] = kappa + kappa (mu nu + (1 -
    kappa - mu) kappa)."""
    gr = W.from_edges(3, [(0, 1), (0, 2), (2, 1)])
    ptr, src = gr.numpy()
    kappa, mu, nu, B = 0.3, 0.3, 0.6, 200000
    st, _, _, _ = oracle.simulate("swir", ptr, src, [0], B, 0x5A4, beta=kappa, alpha=mu,
                                  gamma=nu, max_steps=-1)
    want = kappa + kappa * (mu * nu + (1 - kappa - mu) * kappa)
    assert abs(X.zscore((st[1] == 3).mean(), want, B)) < ZMAX


def test_swir_refuses_kappa_plus_mu_above_one():
    gr = W.from_edges(2, [(0, 1)])
    ptr, src = gr.numpy()
    with pytest.raises(ValueError):
        oracle.simulate("swir", ptr, src, [0], 4, 1, beta=0.7, alpha=0.4, gamma=0.1, max_steps=3)


# -------------------------------------------------------------- LT pins --

@pytest.mark.parametrize("case", [0, 1, 2])
def test_lt_live_edge_equivalence(case):
    """LT with weights 1/indeg and uniform thresholds has the final-set law of
    reachability when every node keeps one uniformly chosen in-arc."""
    rng = np.random.default_rng(70 + case)
    n = 7
    edges = [(int(rng.integers(n)), int(rng.integers(n))) for _ in range(12)]
    gr = W.from_edges(n, edges)
    ptr, src = gr.numpy()
    seeds = [0]
    p = X.lt_exact_marginals(n, ptr, src, seeds)
    B = 40000
    _, cnt, _, absorbed = oracle.simulate("lt", ptr, src, seeds, B, 0x9999 + case)
    assert absorbed == 1
    for v in range(n):
        assert abs(X.zscore(cnt[v] / B, p[v], B)) < ZMAX, (v, cnt[v] / B, p[v])


# ----------------------------------------------------------- invariants --

@pytest.mark.parametrize("model", ["ic", "sir", "sis", "si", "lt"])
def test_invariants(model):
    """Counts are the per-node number of counted replicates; the result of a
    batch does not depend on how it is split over replicate_offset; a run of
    K1 steps is the prefix of a run of K2 > K1 steps (monotone R / active set,
    shrinking S); nothing outside the forward reach of the seeds changes."""
    gr = W.chung_lu(300, 5.0, 2.5, 21)
    ptr, src = gr.numpy()
    seeds = W.uniform_seeds(gr.n, 4, 22)
    kw = dict(p=0.2, beta=0.15, gamma=0.2)
    K1, K2 = 3, 9
    B = 48
    key = 0xC0FFEE
    full = oracle.simulate(model, ptr, src, seeds, B, key, max_steps=K2, **kw)
    st = full[0]
    counted = (st == 1) if model == "sis" else (st != 0)
    assert (counted.sum(axis=1) == full[1]).all()
    a = oracle.simulate(model, ptr, src, seeds, 20, key, max_steps=K2, **kw)
    b = oracle.simulate(model, ptr, src, seeds, B - 20, key, max_steps=K2, replicate_offset=20, **kw)
    assert (np.concatenate([a[0], b[0]], axis=1) == st).all()
    early = oracle.simulate(model, ptr, src, seeds, B, key, max_steps=K1, **kw)[0]
    if model in ("sir", "si", "ic"):
        assert ((early == 0) | (st != 0)).all()       # ever-active only grows
        assert ((early != 2) | (st == 2)).all()       # removed stays removed
    if model == "lt":
        assert ((early == 0) | (st == 1)).all()
    # forward reach of the seeds over all arcs
    reach = X.reach_levels(gr.n, [(u, v) for u, v, _ in X.arcs_of(ptr, src)], list(seeds))
    unreachable = np.array([d < 0 for d in reach])
    assert (st[unreachable] == 0).all()
    if model != "sis":
        assert (st[seeds] != 0).all()
