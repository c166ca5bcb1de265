"""Learned surrogate of the Monte Carlo SIR spread: training data from the
simulator itself, ensemble training, uncertainty threshold and evaluation
with Monte Carlo fallback.

Orchestration only: labels come from the batched simulator (fsg_batch_run),
the network's forward, backward and Adam steps are the library's kernels
(fsg_gnn_*), and every fallback is a plain fsg_simulate call.  The surrogate's
error is measured against plain simulator runs.
"""
from __future__ import annotations

import math
import time
from typing import List, Sequence

import numpy as np

from . import fsg


def log(*a):
    import sys
    print(*a, file=sys.stderr, flush=True)


def seed_sets(n: int, count: int, rng: np.random.Generator, max_size: int = 1000):
    """Seed sets of size round(exp U(0, ln max_size)), uniform without replacement."""
    out = []
    for _ in range(count):
        k = max(1, int(round(math.exp(rng.uniform(0.0, math.log(max_size))))))
        out.append(np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int32))
    return out


def masks_of(sets: Sequence[np.ndarray], n: int, device="cuda"):
    import torch
    m = torch.zeros((len(sets), n), dtype=torch.uint8)
    for i, s in enumerate(sets):
        m[i, torch.as_tensor(s, dtype=torch.int64)] = 1
    return m.to(device)


def mc_frequencies(graph: fsg.DeviceGraph, sets, betas, gamma: float, max_steps: int, B: int,
                   key_base: int, jobs_per_batch: int = 128):
    """Per-node infection frequencies (ever infected / B) of every seed set,
    from batched runs of the simulator.  Returns (float32 cuda tensor
    [len(sets), n], spreads as numpy [len(sets)], device ms)."""
    import torch
    n = graph.n
    out = torch.empty((len(sets), n), dtype=torch.float32, device=graph.device)
    total_ms = 0.0
    for b0 in range(0, len(sets), jobs_per_batch):
        idx = range(b0, min(len(sets), b0 + jobs_per_batch))
        jobs = [dict(graph=graph, model="sir", B=B, seeds=sets[i], rng_key=key_base + i,
                     beta=float(betas[i]), gamma=gamma, max_steps=max_steps) for i in idx]
        batch = fsg.Batch(jobs, want_states=False)
        _, ms = batch.run()
        total_ms += ms
        for k, i in enumerate(idx):
            out[i] = batch.counts[k].to(torch.float32) / B
        batch.close()
    return out, out.sum(dim=1).cpu().numpy().astype(np.float64), total_ms


class Ensemble:
    """M independently initialised members trained on the same data in
    different orders."""

    def __init__(self, members: int = 4, seed: int = 1, device="cuda"):
        self.members = [fsg.GNN(seed * 1000 + i, device) for i in range(members)]

    def train(self, data, epochs: int, sets_per_step: int, lr: float, seed: int = 0,
              progress_every: int = 1, final_lr_fraction: float = 0.1):
        """data: list of (graph, reverse, masks, betas, targets) per training
        graph.  The learning rate decays geometrically from lr to
        lr * final_lr_fraction over the epochs.  Returns the mean loss of each
        epoch per member."""
        hist = []
        for mi, net in enumerate(self.members):
            rng = np.random.default_rng(seed * 7919 + mi)
            losses = []
            for ep in range(epochs):
                lr_ep = lr * final_lr_fraction ** (ep / max(1, epochs - 1))
                batches = []
                for gi, (_, _, masks, _, _) in enumerate(data):
                    order = rng.permutation(masks.shape[0])
                    for s0 in range(0, len(order), sets_per_step):
                        batches.append((gi, order[s0:s0 + sets_per_step]))
                rng.shuffle(batches)
                tot = 0.0
                for gi, sel in batches:
                    g, rev, masks, betas, targets = data[gi]
                    import torch
                    si = torch.as_tensor(sel, device=masks.device)
                    tot += net.train_step(g, rev, masks[si].contiguous(), [betas[j] for j in sel],
                                          targets[si].contiguous(), lr_ep)
                losses.append(tot / len(batches))
                if progress_every and (ep + 1) % progress_every == 0:
                    log(f"[surrogate] member {mi} epoch {ep + 1}/{epochs}: loss {losses[-1]:.5f}")
            hist.append(losses)
        return hist

    def predict_spreads(self, graph: fsg.DeviceGraph, masks, betas, sets_per_call: int = 8):
        """Predicted spread (sum of p_v) of every member for every seed set:
        numpy [M, n_sets]."""
        out = np.zeros((len(self.members), masks.shape[0]))
        for mi, net in enumerate(self.members):
            for s0 in range(0, masks.shape[0], sets_per_call):
                sl = slice(s0, min(masks.shape[0], s0 + sets_per_call))
                p = net.forward(graph, masks[sl].contiguous(), list(betas[sl]))
                out[mi, sl] = p.sum(dim=1).double().cpu().numpy()
        return out


def uncertainty(pred: np.ndarray):
    """Mean spread and relative sample std across members, per query."""
    mean = pred.mean(axis=0)
    std = pred.std(axis=0, ddof=1) if pred.shape[0] > 1 else np.zeros_like(mean)
    return mean, std / np.maximum(mean, 1e-12)


def calib_features(beta, k):
    """Terms of the spread calibration, per query: [1, x, x^2, x^3, 1/k, x/k,
    1/k^2, ln k, x ln k] with x = 20 beta and k the number of distinct seeds
    (the same terms fsg_estimate_spread evaluates)."""
    x = 20.0 * np.asarray(beta, dtype=np.float64)
    k = np.maximum(np.asarray(k, dtype=np.float64), 1.0)
    lk = np.log(k)
    return np.stack([np.ones_like(x), x, x * x, x ** 3, 1.0 / k, x / k, 1.0 / (k * k), lk, x * lk],
                    axis=-1)


def fit_calibration(pred_mean, label, beta, k, min_seeds: int = 5):
    """Least-squares fit of ln(label / prediction) on the calibration terms,
    over training queries with at least min_seeds seeds; returns the
    coefficient vector (the calibrated spread is prediction * exp(f . c))."""
    pred_mean, label = np.asarray(pred_mean, np.float64), np.asarray(label, np.float64)
    k = np.asarray(k)
    sel = (k >= min_seeds) & (pred_mean > 0) & (label > 0)
    A = calib_features(np.asarray(beta)[sel], k[sel])
    coef, *_ = np.linalg.lstsq(A, np.log(label[sel] / pred_mean[sel]), rcond=None)
    return coef


def apply_calibration(pred_mean, beta, k, coef):
    return np.asarray(pred_mean, np.float64) * np.exp(calib_features(beta, k) @ np.asarray(coef))


def calibrate_gate(spread, unc, ref, k, max_rel_err: float, min_seeds_floor: int = 5,
                   quantile: float = 0.9, quantile_frac: float = 0.25, tau_slack: float = 1.0,
                   min_queries: int = 10, safety: float = 2.0):
    """Acceptance gate from held-out calibration queries (calibrated spread,
    member uncertainty, Monte Carlo reference, seed count).

    A query is accepted iff its seed count is at least min_seeds and its
    member uncertainty at most tau.  Over the pairs (k0 >= min_seeds_floor,
    t) drawn from the calibration queries' own values, the gate takes the one
    that accepts the most calibration queries (at least min_queries) while
    their `quantile` error stays below quantile_frac * max_rel_err and their
    largest error below max_rel_err / safety (a few dozen calibration queries
    understate the largest error of the queries to come); then min_seeds and
    tau / tau_slack are the smallest seed count and the largest uncertainty
    among the queries it accepts.  Near the epidemic threshold the spread is
    sensitive to beta and the members disagree, which the uncertainty bound
    catches at any seed count.  No such pair: everything falls back.
    Returns dict(tau, min_seeds)."""
    spread, unc, ref, k = (np.asarray(a, np.float64) for a in (spread, unc, ref, k))
    err = np.abs(spread - ref) / np.maximum(ref, 1e-12)
    best = None
    for k0 in sorted(set(int(x) for x in k if x >= min_seeds_floor)):
        for t in sorted(set(float(x) for x in unc)):
            sel = (k >= k0) & (unc <= t)
            cnt = int(sel.sum())
            if cnt < min_queries or (best is not None and cnt <= best[0]):
                continue
            if np.quantile(err[sel], quantile) <= quantile_frac * max_rel_err and \
                    err[sel].max() <= max_rel_err / safety:
                best = (cnt, sel)
    if best is None:
        return dict(tau=-1.0, min_seeds=int(k.max()) + 1)
    sel = best[1]
    return dict(tau=float(tau_slack * unc[sel].max()), min_seeds=int(k[sel].min()))


def calibrate_tau(mean, unc, ref, max_rel_err: float):
    """Largest threshold tau such that every calibration query with
    uncertainty <= tau has relative error <= max_rel_err."""
    err = np.abs(mean - ref) / np.maximum(ref, 1e-12)
    order = np.argsort(unc)
    tau = -1.0
    for i in order:
        if err[i] > max_rel_err:
            break
        tau = unc[i]
    return float(tau)
