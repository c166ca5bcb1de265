"""Pins of the surrogate's FP64 oracle: its hand-written backward pass equals
central finite differences of its forward pass (float64, no rounding), the
mean aggregation is the identity on constant inputs and 0 on empty
neighbourhoods, and its transpose satisfies <A x, y> = <x, A^T y>."""
import numpy as np

from oracle import gnn as G
from paper_2603_14895_amd import workloads as W


def _graph():
    return W.from_edges(7, [(0, 1), (1, 2), (2, 0), (3, 1), (4, 4), (0, 5), (5, 0), (2, 5), (6, 3)]).numpy()


def test_param_count():
    assert G.N_PARAMS == 18689


def test_backward_matches_finite_differences():
    ptr, src = _graph()
    n = len(ptr) - 1
    rng = np.random.default_rng(3)
    params = G.glorot(5)
    masks = [(rng.random(n) < 0.4).astype(float) for _ in range(2)]
    betas = [0.02, 0.045]
    ys = [rng.random(n) for _ in range(2)]
    loss, grad = G.loss_and_grad(params, ptr, src, masks, betas, ys)
    idx = list(range(0, G.N_PARAMS, 97)) + list(range(G.N_PARAMS - 70, G.N_PARAMS))
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fp, _ = G.loss_and_grad(pp, ptr, src, masks, betas, ys)
        fm, _ = G.loss_and_grad(pm, ptr, src, masks, betas, ys)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, grad[i])


def test_mean_aggregation_special_cases():
    ptr, src = _graph()
    n = len(ptr) - 1
    X = np.full((n, 3), 2.5)
    M = G.mean_agg(X, ptr, src)
    indeg = np.diff(ptr)
    assert np.allclose(M[indeg > 0], 2.5) and np.allclose(M[indeg == 0], 0.0)
    rng = np.random.default_rng(1)
    x, y = rng.normal(size=(n, 4)), rng.normal(size=(n, 4))
    assert np.isclose(np.sum(G.mean_agg(x, ptr, src) * y), np.sum(x * G.mean_agg_T(y, ptr, src)))


def test_bf16_rounding():
    assert G.bf16(1.0) == 1.0
    assert G.bf16(1.0 + 2 ** -9) == 1.0            # tie to even
    assert G.bf16(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7
    assert G.bf16(-0.1) == -0.10009765625
