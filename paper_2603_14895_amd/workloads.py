"""Seeded synthetic inputs: graphs, seed sets and RNG keys.

This module holds none of the propagation arithmetic.  It only builds inputs
-- directed Erdos-Renyi graphs, Chung-Lu power-law graphs, R-MAT graphs, pull
(in-edge) CSR arrays, seed sets and 64-bit keys -- and serves the HIP path and
the CPU oracle alike.  Every generator takes an explicit integer seed; torch
generators are used so the same code runs on the host and, for the large
graphs, on the GPU (where a graph is produced on the GPU, callers copy the
resulting arrays to the host for the oracle rather than regenerating them).

The paper's datasets (Cora, PubMed, Flickr, Yelp, Pokec, Webbase;
Table tab:dataset) are not available, so these generators stand in for them at
similar sizes and degree distributions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import torch

BASE_SEED = 20261203


@dataclasses.dataclass
class Graph:
    """Pull CSR: row v lists the sources u of the arcs u -> v.

    ptr: int64 [n+1]; src: int32 [nnz].  The edge id of an arc is its position
    in ``src``.  Arrays are torch tensors on ``device``.
    """
    n: int
    ptr: torch.Tensor
    src: torch.Tensor
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.src.numel())

    def indeg(self) -> torch.Tensor:
        return self.ptr[1:] - self.ptr[:-1]

    def to(self, device) -> "Graph":
        return Graph(self.n, self.ptr.to(device), self.src.to(device), self.name)

    def numpy(self):
        return self.ptr.cpu().numpy(), self.src.cpu().numpy()


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    return g


def pull_csr(n: int, src: torch.Tensor, dst: torch.Tensor, name: str = "") -> Graph:
    """Arcs (src -> dst) to pull CSR; rows by dst, entries of a row by src."""
    src = src.to(torch.int64)
    dst = dst.to(torch.int64)
    key = dst * n + src
    key, _ = torch.sort(key)
    dst_sorted = torch.div(key, n, rounding_mode="floor")
    src_sorted = (key - dst_sorted * n).to(torch.int32)
    counts = torch.bincount(dst_sorted, minlength=n)
    ptr = torch.zeros(n + 1, dtype=torch.int64, device=src.device)
    ptr[1:] = torch.cumsum(counts, 0)
    return Graph(n, ptr, src_sorted.contiguous(), name)


def reverse_graph(graph: Graph) -> Graph:
    """The same arcs reversed, as a pull CSR: row u lists the targets v of
    the arcs u -> v of ``graph`` (its out-adjacency)."""
    n = graph.n
    dst = torch.repeat_interleave(torch.arange(n, device=graph.ptr.device),
                                  graph.ptr[1:] - graph.ptr[:-1])
    return pull_csr(n, dst, graph.src.to(torch.int64), graph.name + "_rev")


def from_edges(n: int, edges, name: str = "") -> Graph:
    """Small hand-written graphs: ``edges`` is a list of (u, v) arcs."""
    if len(edges) == 0:
        e = torch.zeros((0, 2), dtype=torch.int64)
    else:
        e = torch.tensor(edges, dtype=torch.int64)
    return pull_csr(n, e[:, 0], e[:, 1], name)


def erdos_renyi_directed(n: int, mean_out_degree: float, seed: int, device="cpu") -> Graph:
    """Directed G(n, p), p = mean_out_degree / (n-1): each ordered pair i != j
    independently.  Built row block by row block so memory stays O(n * block)."""
    p = mean_out_degree / (n - 1)
    g = _gen(seed, device)
    srcs, dsts = [], []
    block = max(1, min(n, (1 << 24) // max(n, 1)))
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        m = torch.rand((i1 - i0, n), generator=g, device=device) < p
        rows = torch.arange(i0, i1, device=device)
        m[rows - i0, rows] = False
        s, d = torch.nonzero(m, as_tuple=True)
        srcs.append(s + i0)
        dsts.append(d)
    return pull_csr(n, torch.cat(srcs), torch.cat(dsts), f"er_n{n}_d{mean_out_degree}")


def chung_lu(n: int, mean_degree: float, exponent: float, seed: int, device="cpu",
             chunk: int = 1 << 25) -> Graph:
    """Undirected Chung-Lu graph stored as symmetric arcs.

    Expected weights w_i proportional to (n / (i+1))^(1/(exponent-1)),
    scaled so the mean weight is ``mean_degree``.  n * mean_degree / 2 pairs
    are drawn with both endpoints proportional to w; self-loops and repeated
    pairs are dropped (a simple graph), so the realised mean degree is a little
    below ``mean_degree``.
    """
    g = _gen(seed, device)
    idx = torch.arange(n, dtype=torch.float64, device=device)
    w = (n / (idx + 1.0)) ** (1.0 / (exponent - 1.0))
    w = w * (mean_degree / w.mean())
    cw = torch.cumsum(w, 0)
    total = float(cw[-1])
    m = int(round(n * mean_degree / 2))
    keys = []
    for c0 in range(0, m, chunk):
        c = min(chunk, m - c0)
        a = torch.searchsorted(cw, torch.rand(c, generator=g, device=device, dtype=torch.float64) * total)
        b = torch.searchsorted(cw, torch.rand(c, generator=g, device=device, dtype=torch.float64) * total)
        a = a.clamp_(max=n - 1)
        b = b.clamp_(max=n - 1)
        keep = a != b
        a, b = a[keep], b[keep]
        lo = torch.minimum(a, b)
        hi = torch.maximum(a, b)
        keys.append(lo * n + hi)
    key = torch.unique(torch.cat(keys))
    lo = torch.div(key, n, rounding_mode="floor")
    hi = key - lo * n
    del key
    src = torch.cat([lo, hi])
    dst = torch.cat([hi, lo])
    return pull_csr(n, src, dst, f"chung_lu_n{n}_d{mean_degree}_x{exponent}")


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int, device="cpu",
         chunk: int = 1 << 26, permute: bool = False) -> Graph:
    """R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each of edge_factor * 2^scale
    arcs picks one of four quadrants per level with probabilities (a, b, c, d);
    no noise; duplicates and self-loops are kept, so nnz is exact.  The row bit
    is the source bit and the column bit the destination bit."""
    n = 1 << scale
    m = edge_factor * n
    g = _gen(seed, device)
    ab, abc = a + b, a + b + c
    keys = []
    for c0 in range(0, m, chunk):
        cnt = min(chunk, m - c0)
        s = torch.zeros(cnt, dtype=torch.int64, device=device)
        d = torch.zeros(cnt, dtype=torch.int64, device=device)
        for _ in range(scale):
            u = torch.rand(cnt, generator=g, device=device)
            sbit = (u >= ab).to(torch.int64)
            dbit = ((u >= a) & (u < ab) | (u >= abc)).to(torch.int64)
            s = s * 2 + sbit
            d = d * 2 + dbit
        keys.append(d * n + s)
    key = torch.sort(torch.cat(keys))[0] if len(keys) > 1 else torch.sort(keys[0])[0]
    keys = None
    dst = torch.div(key, n, rounding_mode="floor")
    src = (key - dst * n)
    del key
    if permute:
        perm = torch.randperm(n, generator=g, device=device)
        src, dst = perm[src], perm[dst]
        return pull_csr(n, src, dst, f"rmat_s{scale}_ef{edge_factor}_perm")
    counts = torch.bincount(dst, minlength=n)
    ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    ptr[1:] = torch.cumsum(counts, 0)
    return Graph(n, ptr, src.to(torch.int32).contiguous(), f"rmat_s{scale}_ef{edge_factor}")


def uniform_seeds(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct nodes, uniform without replacement (host int32)."""
    g = _gen(seed, "cpu")
    k = min(k, n)
    return torch.randperm(n, generator=g)[:k].to(torch.int32).numpy()


def uniform_opinions(n: int, B: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Initial opinions of the Hegselmann-Krause model: float32 [n, B], each
    independent and uniform on [lo, hi) (the opinion interval is [-1, 1])."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, B)).astype(np.float32)


def top_indegree_seeds(graph: Graph, k: int) -> np.ndarray:
    """Degree-centrality seeds as in the paper's usage example (Listing 1):
    the k nodes of largest in-degree; ties broken by node id."""
    indeg = graph.indeg().cpu().numpy()
    order = np.lexsort((np.arange(graph.n), -indeg))
    return order[:k].astype(np.int32)


def rng_key(seed: int) -> int:
    g = _gen(seed, "cpu")
    hi = int(torch.randint(0, 2**31, (1,), generator=g)) << 33
    lo = int(torch.randint(0, 2**32, (1,), generator=g))
    mid = int(torch.randint(0, 2, (1,), generator=g)) << 32
    return (hi | mid | lo) & (2**64 - 1)


def loguniform_int(rng: np.random.Generator, lo: float, hi: float) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


# ----------------------------------------------------------------- configs --

def config_c1(device="cpu"):
    """IC on directed G(n=1000, mean out-degree 10), p = 0.1, 10 uniform seeds,
    B = 100, to absorption."""
    s = BASE_SEED + 1
    gr = erdos_renyi_directed(1000, 10.0, s, device)
    return dict(name="c1_ic_er1000", graph=gr, model="ic", p=0.1, ic_prob="uniform",
                seeds=uniform_seeds(gr.n, 10, s + 1), B=100, rng_key=rng_key(s + 2), max_steps=-1)


def config_c2(device="cpu", n: int = 1_000_000, B: int = 1024, steps: int = 200):
    """SIR on a Chung-Lu graph (exponent 2.5, mean degree 20, undirected),
    beta = 0.02, gamma = 0.1, 1% uniform initial infected, 200 steps."""
    s = BASE_SEED + 2
    gr = chung_lu(n, 20.0, 2.5, s, device)
    return dict(name=f"c2_sir_chunglu{n}", graph=gr, model="sir", beta=0.02, gamma=0.1,
                seeds=uniform_seeds(n, max(1, n // 100), s + 1), B=B, rng_key=rng_key(s + 2),
                max_steps=steps)


def config_hk(device="cpu", n: int = 1_000_000, B: int = 256, steps: int = 20):
    """Hegselmann-Krause on the same Chung-Lu graph as the SIR workload
    (exponent 2.5, mean degree 20), eps = 0.32 (the paper's HK setting),
    B = 256 replicates of uniform [-1, 1] initial opinions, 20 steps."""
    s = BASE_SEED + 2
    gr = chung_lu(n, 20.0, 2.5, s, device)
    return dict(name=f"hk_chunglu{n}_eps0.32", graph=gr, model="hk", eps=0.32, B=B,
                max_steps=steps, opinion_seed=s + 7)


def config_c4(device="cpu", scale: int = 26, B: int = 64, edge_factor: int = 16):
    """Web-scale IC: R-MAT (a, b, c) = (0.57, 0.19, 0.19), weighted cascade
    p = 1/indeg(v), 50 uniform seeds, B = 64, to absorption."""
    s = BASE_SEED + 4
    gr = rmat(scale, edge_factor, 0.57, 0.19, 0.19, s, device)
    return dict(name=f"c4_ic_rmat{scale}", graph=gr, model="ic", ic_prob="weighted_cascade",
                p=0.0, seeds=uniform_seeds(gr.n, 50, s + 1), B=B, rng_key=rng_key(s + 2),
                max_steps=-1)


def config_c3_jobs(n_jobs: int = 64, n_lo: float = 1e4, n_hi: float = 2e6, b_lo: float = 64,
                   b_hi: float = 4096, seed_hi: float = 1000, seed: Optional[int] = None):
    """Job descriptors of the mixed batched workload (graphs are built lazily
    by :func:`build_c3_graph`).  Models cycle IC (p = 0.05), SIR (beta = 0.03,
    gamma = 0.1, 200 steps), LT (1/indeg weights, U(0,1) thresholds)."""
    s = BASE_SEED + 3 if seed is None else seed
    rng = np.random.default_rng(np.random.SeedSequence(s))
    jobs = []
    for j in range(n_jobs):
        n = loguniform_int(rng, n_lo, n_hi)
        deg = float(rng.uniform(5.0, 50.0))
        B = max(1, loguniform_int(rng, b_lo, b_hi))
        k = max(1, loguniform_int(rng, 1.0, seed_hi))
        model = ["ic", "sir", "lt"][j % 3]
        job = dict(index=j, n=n, mean_degree=deg, B=B, n_seeds=min(k, n), model=model,
                   graph_seed=s * 1000 + 17 * j + 1, seed_seed=s * 1000 + 17 * j + 2,
                   key=rng_key(s * 1000 + 17 * j + 3))
        if model == "ic":
            job.update(p=0.05, ic_prob="uniform", max_steps=-1)
        elif model == "sir":
            job.update(beta=0.03, gamma=0.1, max_steps=200)
        else:
            job.update(max_steps=-1)
        jobs.append(job)
    return jobs


def build_c3_graph(job, device="cpu") -> Graph:
    return chung_lu(job["n"], job["mean_degree"], 2.5, job["graph_seed"], device)
