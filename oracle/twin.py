"""Pure-Python twin of the C oracle, for tiny inputs (test infrastructure only).

Written separately from ``fsg_oracle.c`` so that a slip in one (an index, a
shift, a state code) shows up as a disagreement with the other.  Same contract:

* Philox4x32-10 from Salmon et al., SC'11 (multipliers 0xD2511F53,
  0xCD9E8D57; Weyl key increments 0x9E3779B9, 0xBB67AE85), on Python ints;
* draw(dom, unit, g, step) uses counter (lo32 unit, g >> 2, step,
  dom << 24 | hi32 unit) and keeps output word g & 3;
* Bernoulli(p) fires iff t == 2^32 - 1 or draw < t, with t = thr(p);
* synchronous update of every node from the previous-round states of its
  in-neighbours (Eq. nodestate; Algorithm 1), SIR as Appendix A.1.
"""
from __future__ import annotations

import math

M32 = 0xFFFFFFFF
ALWAYS = 0xFFFFFFFF
IC, SI, SIS, SIR, LT = 0, 1, 2, 3, 4


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = (int(x) & M32 for x in ctr)
    k0, k1 = (int(x) & M32 for x in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + 0x9E3779B9) & M32
            k1 = (k1 + 0xBB67AE85) & M32
        p0 = 0xD2511F53 * c0
        p1 = 0xCD9E8D57 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0, p1 & M32, (p0 >> 32) ^ c3 ^ k1, p0 & M32)
    return [c0, c1, c2, c3]


def draw(rng_key, dom, unit, g, step):
    ctr = (unit & M32, (g >> 2) & M32, step & M32, ((dom << 24) | (unit >> 32)) & M32)
    key = (rng_key & M32, (rng_key >> 32) & M32)
    return philox4x32_10(ctr, key)[g & 3]


def thr(p):
    if not p > 0.0:
        return 0
    if p >= 1.0:
        return ALWAYS
    return min(int(math.floor(p * 4294967296.0)), 0xFFFFFFFE)


def fires(u, t):
    return t == ALWAYS or u < t


def sir_table(beta, length):
    out, q = [], 1.0
    for k in range(length):
        if k:
            q = q * (1.0 - beta)
        out.append(thr(1.0 - q))
    return out


def simulate(model, ptr, src, seeds, B, rng_key, *, p=0.0, ic_prob=0, edge_p=None, beta=0.0,
             gamma=0.0, max_steps=-1, replicate_offset=0):
    """Returns (states as list of per-node lists [n][B], counts, steps_run, absorbed)."""
    ptr = [int(x) for x in ptr]
    src = [int(x) for x in src]
    n = len(ptr) - 1
    indeg = [ptr[v + 1] - ptr[v] for v in range(n)]
    table = sir_table(beta, max(indeg, default=0) + 1)
    trec = thr(0.0 if model == SI else gamma)

    def t_edge(v, e):
        if ic_prob == 0:
            return thr(p)
        if ic_prob == 2:
            return thr(edge_p[e])
        return thr(1.0 / indeg[v])

    states = [[0] * B for _ in range(n)]
    counts = [0] * n
    steps_run, any_one = 0, False
    for r in range(B):
        g = replicate_offset + r
        x = [0] * n
        for s in seeds:
            x[int(s)] = 1
        t = 0
        while (max_steps < 0 or t < max_steps) and 1 in x:
            t += 1
            y = list(x)
            for v in range(n):
                edges = range(ptr[v], ptr[v + 1])
                if model == IC:
                    if x[v] == 1:
                        y[v] = 2
                    elif x[v] == 0:
                        for e in edges:
                            if x[src[e]] == 1 and fires(draw(rng_key, 1, e, g, 0), t_edge(v, e)):
                                y[v] = 1
                                break
                elif model == LT:
                    if x[v] != 0:
                        y[v] = 2
                    else:
                        c = sum(1 for e in edges if x[src[e]] != 0)
                        u = draw(rng_key, 3, v, g, 0)
                        if c >= 1 and c * 2**32 >= u * indeg[v]:
                            y[v] = 1
                else:
                    u = draw(rng_key, 2, v, g, t)
                    if x[v] == 0:
                        k = sum(1 for e in edges if x[src[e]] == 1)
                        if k > 0 and fires(u, table[k]):
                            y[v] = 1
                    elif x[v] == 1 and fires(u, trec):
                        y[v] = 0 if model == SIS else 2
            x = y
        steps_run = max(steps_run, t)
        any_one = any_one or (1 in x)
        for v in range(n):
            out = int(x[v] != 0) if model == LT else x[v]
            states[v][r] = out
            counts[v] += int(x[v] == 1) if model == SIS else int(x[v] != 0)
    return states, counts, steps_run, int(not any_one)


def hk(ptr, src, h0, eps, max_steps):
    """Hegselmann-Krause (Appendix A.2) on IEEE single scalars: h0 is a list
    of B-long lists of floats (node-major); returns (h, steps_run,
    converged) like the C oracle."""
    import numpy as np
    f32 = np.float32
    e = f32(eps)
    n = len(ptr) - 1
    x = [[f32(v) for v in row] for row in h0]
    B = len(x[0]) if n else 0
    t, changed = 0, True
    while t < max_steps and changed:
        t += 1
        changed = False
        y = []
        for v in range(n):
            row = []
            for r in range(B):
                hv = x[v][r]
                num, cnt = f32(0.0), 0
                for k in range(ptr[v], ptr[v + 1]):
                    hj = x[src[k]][r]
                    if abs(f32(hv - hj)) < e:
                        num = f32(num + hj)
                        cnt += 1
                new = f32(num / f32(cnt)) if cnt else hv
                changed |= bool(new != hv)
                row.append(new)
            y.append(row)
        x = y
    return x, t, int(not changed)
