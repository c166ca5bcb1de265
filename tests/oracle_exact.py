"""Exact reference distributions for tiny graphs, used to pin the oracle.

Each function computes a probability the propagation model fixes in closed
form or by exhaustive enumeration -- never by running the oracle -- so that a
dropped term, a wrong index or a transposed operand in the oracle shows up as
a statistically impossible Monte Carlo frequency.
"""
from __future__ import annotations

import itertools

import numpy as np


def arcs_of(ptr, src):
    """(u, v, edge_id) triples of a pull CSR."""
    out = []
    for v in range(len(ptr) - 1):
        for e in range(ptr[v], ptr[v + 1]):
            out.append((int(src[e]), v, e))
    return out


def reach_levels(n, live_arcs, seeds):
    """Hop distance from the seed set over the given arcs (-1 unreachable)."""
    dist = [-1] * n
    frontier = []
    for s in seeds:
        if dist[s] < 0:
            dist[s] = 0
            frontier.append(s)
    out = {}
    for u, v in live_arcs:
        out.setdefault(u, []).append(v)
    d = 0
    while frontier:
        nxt = []
        for u in frontier:
            for v in out.get(u, []):
                if dist[v] < 0:
                    dist[v] = d + 1
                    nxt.append(v)
        frontier = nxt
        d += 1
    return dist


def ic_exact_marginals(n, ptr, src, seeds, edge_prob):
    """Independent cascade: enumerate all 2^|E| live-edge worlds.  Returns
    P[v ever active] and P[activation step of v == d] as arrays [n] and
    [n, n+1].  ``edge_prob`` gives the probability of each edge id."""
    arcs = arcs_of(ptr, src)
    m = len(arcs)
    assert m <= 20
    p_act = np.zeros(n)
    p_dist = np.zeros((n, n + 1))
    for mask in range(1 << m):
        w = 1.0
        live = []
        for i, (u, v, e) in enumerate(arcs):
            if mask >> i & 1:
                w *= edge_prob[e]
                live.append((u, v))
            else:
                w *= 1.0 - edge_prob[e]
        if w == 0.0:
            continue
        dist = reach_levels(n, live, seeds)
        for v in range(n):
            if dist[v] >= 0:
                p_act[v] += w
                p_dist[v, dist[v]] += w
    return p_act, p_dist


def lt_exact_marginals(n, ptr, src, seeds):
    """Linear threshold with weights 1/indeg and uniform thresholds, through
    its live-edge equivalent (Kempe, Kleinberg, Tardos 2003): every node with
    in-arcs keeps exactly one of them, uniformly.  Returns P[v active at the
    end], enumerating prod(indeg) worlds."""
    choices = []
    for v in range(n):
        row = [(int(src[e]), v) for e in range(ptr[v], ptr[v + 1])]
        choices.append(row if row else [None])
    p = np.zeros(n)
    total = 0.0
    for pick in itertools.product(*choices):
        w = 1.0
        for v in range(n):
            d = ptr[v + 1] - ptr[v]
            if d:
                w /= d
        live = [a for a in pick if a is not None]
        dist = reach_levels(n, live, seeds)
        for v in range(n):
            if dist[v] >= 0:
                p[v] += w
        total += w
    assert abs(total - 1.0) < 1e-9
    return p


def epidemic_exact_marginals(n, ptr, src, seeds, beta, gamma, steps, sis=False):
    """Exact synchronous SIR / SIS Markov chain on all 3^n (2^n) joint states.

    Given the previous joint state every node moves independently:
    S -> I with probability 1 - (1-beta)^k, k = number of infected in-arcs
    (Appendix A.1); I -> R (SIS: I -> S) with probability gamma; R stays.
    Returns P[x_v = s] after ``steps`` steps as an array [n, 3]."""
    nstate = 2 if sis else 3
    indeg_rows = [[int(src[e]) for e in range(ptr[v], ptr[v + 1])] for v in range(n)]
    x0 = [0] * n
    for s in seeds:
        x0[s] = 1
    dist = {tuple(x0): 1.0}
    for _ in range(steps):
        nxt = {}
        for x, mass in dist.items():
            per_node = []
            for v in range(n):
                if x[v] == 0:
                    k = sum(1 for u in indeg_rows[v] if x[u] == 1)
                    pinf = 1.0 - (1.0 - beta) ** k
                    per_node.append([(0, 1.0 - pinf), (1, pinf)])
                elif x[v] == 1:
                    per_node.append([(0 if sis else 2, gamma), (1, 1.0 - gamma)])
                else:
                    per_node.append([(2, 1.0)])
            for combo in itertools.product(*per_node):
                w = mass
                for _, q in combo:
                    w *= q
                if w == 0.0:
                    continue
                y = tuple(s for s, _ in combo)
                nxt[y] = nxt.get(y, 0.0) + w
        dist = nxt
    marg = np.zeros((n, 3))
    for x, mass in dist.items():
        for v in range(n):
            marg[v, x[v]] += mass
    assert nstate in (2, 3)
    return marg


def latent_exact_marginals(n, ptr, src, seeds, beta, alpha, gamma, steps, seis=False):
    """Exact synchronous SEIR / SEIS Markov chain on all 4^n joint states
    (states 0 S, 1 E, 2 I, 3 R; seeds start in I).

    Given the previous joint state every node moves independently:
    S -> E with probability 1 - (1-beta)^k, k = number of in-arcs from
    nodes in I; E -> I with probability alpha; I -> R (SEIS: I -> S) with
    probability gamma; R stays.  Returns P[x_v = s] after ``steps`` steps as
    an array [n, 4]."""
    rows = [[int(src[e]) for e in range(ptr[v], ptr[v + 1])] for v in range(n)]
    x0 = [0] * n
    for s in seeds:
        x0[s] = 2
    dist = {tuple(x0): 1.0}
    for _ in range(steps):
        nxt = {}
        for x, mass in dist.items():
            per_node = []
            for v in range(n):
                if x[v] == 0:
                    k = sum(1 for u in rows[v] if x[u] == 2)
                    q = 1.0 - (1.0 - beta) ** k
                    per_node.append([(0, 1.0 - q), (1, q)])
                elif x[v] == 1:
                    per_node.append([(1, 1.0 - alpha), (2, alpha)])
                elif x[v] == 2:
                    per_node.append([(2, 1.0 - gamma), (0 if seis else 3, gamma)])
                else:
                    per_node.append([(3, 1.0)])
            for combo in itertools.product(*per_node):
                w = mass
                for _, q in combo:
                    w *= q
                if w == 0.0:
                    continue
                y = tuple(s for s, _ in combo)
                nxt[y] = nxt.get(y, 0.0) + w
        dist = nxt
    marg = np.zeros((n, 4))
    for x, mass in dist.items():
        for v in range(n):
            marg[v, x[v]] += mass
    return marg


def zscore(freq, p, B):
    """Binomial z-score of an observed frequency against an exact probability."""
    var = max(p * (1.0 - p), 1e-12) / B
    return (freq - p) / np.sqrt(var)


def swir_exact_marginals(n, ptr, src, seeds, kappa, mu, nu, steps):
    """Exact synchronous SWIR Markov chain on all 4^n joint states (states
    0 S, 1 W, 2 I, 3 R; seeds start in I).

    Given the previous joint state every node moves independently, with k
    the number of in-arcs from nodes in I: S -> I with probability
    1 - (1-kappa)^k, S -> W with probability (1-kappa)^k - (1-kappa-mu)^k;
    W -> I with probability 1 - (1-nu)^k; I -> R; R stays.  Returns
    P[x_v = s] after ``steps`` steps as an array [n, 4]."""
    rows = [[int(src[e]) for e in range(ptr[v], ptr[v + 1])] for v in range(n)]
    x0 = [0] * n
    for s in seeds:
        x0[s] = 2
    dist = {tuple(x0): 1.0}
    for _ in range(steps):
        nxt = {}
        for x, mass in dist.items():
            per_node = []
            for v in range(n):
                k = sum(1 for u in rows[v] if x[u] == 2)
                if x[v] == 0:
                    pi = 1.0 - (1.0 - kappa) ** k
                    pw = (1.0 - kappa) ** k - (1.0 - kappa - mu) ** k
                    per_node.append([(0, 1.0 - pi - pw), (1, pw), (2, pi)])
                elif x[v] == 1:
                    q = 1.0 - (1.0 - nu) ** k
                    per_node.append([(1, 1.0 - q), (2, q)])
                else:
                    per_node.append([(3, 1.0)])
            for combo in itertools.product(*per_node):
                w = mass
                for _, q in combo:
                    w *= q
                if w == 0.0:
                    continue
                y = tuple(s for s, _ in combo)
                nxt[y] = nxt.get(y, 0.0) + w
        dist = nxt
    marg = np.zeros((n, 4))
    for x, mass in dist.items():
        for v in range(n):
            marg[v, x[v]] += mass
    return marg
