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


# ---- Adam (Kingma and Ba, ICLR 2015, Algorithm 1): pins of the oracle's
# single-precision step against the algorithm's closed forms in float64


def _adam_f64(theta, grads, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Float64 reference by the closed forms: m_t = (1 - b1) sum_i b1^(t-i) g_i,
    v_t = (1 - b2) sum_i b2^(t-i) g_i^2, and the parameter after each step.
    The constants are the single-precision values the optimiser stores (0.999
    in single precision is 1.3e-5 away from 0.999 relative to 1 - 0.999)."""
    b1, b2, eps, lr = (float(np.float32(x)) for x in (b1, b2, eps, lr))
    theta = np.array(theta, dtype=np.float64)
    out = []
    for t in range(1, len(grads) + 1):
        m = (1 - b1) * sum(b1 ** (t - i) * np.asarray(grads[i - 1], np.float64) for i in range(1, t + 1))
        v = (1 - b2) * sum(b2 ** (t - i) * np.asarray(grads[i - 1], np.float64) ** 2 for i in range(1, t + 1))
        mh, vh = m / (1 - b1 ** t), v / (1 - b2 ** t)
        theta = theta - lr * mh / (np.sqrt(vh) + eps)
        out.append((theta.copy(), m, v))
    return out


def test_adam_constant_gradient_moments():
    g = np.array([0.5, -2.0, 1e-3, -7e-6, 3.25], dtype=np.float32)
    p = np.zeros_like(g)
    m = np.zeros_like(g)
    v = np.zeros_like(g)
    for t in range(1, 13):
        p, m, v = G.adam_step(p, m, v, g, t, 1e-3)
        g64 = g.astype(np.float64)
        assert np.allclose(m, (1 - 0.9 ** t) * g64, rtol=2e-6, atol=0)
        assert np.allclose(v, (1 - 0.999 ** t) * g64 ** 2, rtol=2e-5, atol=0)
        # with a constant gradient m_hat = g and v_hat = g^2: every step moves
        # each parameter by -lr g / (|g| + eps)
        step = -1e-3 * g64 / (np.abs(g64) + 1e-8)
        assert np.allclose(p, t * step, rtol=2e-5, atol=1e-12)


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.25, 1e-8, -1e-8, 4e-9, 0.0, 123.0], dtype=np.float32)
    p0 = np.linspace(-1, 1, g.size).astype(np.float32)
    p, m, v = G.adam_step(p0, np.zeros_like(g), np.zeros_like(g), g, 1, 2e-3)
    g64 = g.astype(np.float64)
    expect = p0.astype(np.float64) - 2e-3 * g64 / (np.abs(g64) + 1e-8)
    assert np.allclose(p, expect, rtol=0, atol=2e-7)
    assert p[5] == p0[5] and m[5] == 0 and v[5] == 0      # zero gradient: no move
    assert p[0] < p0[0] and p[1] > p0[1]                   # against the gradient's sign
    assert abs((p0[2] - p[2]) - 1e-3) < 1e-6               # |g| = eps: half a step


def test_adam_matches_closed_form_sequence():
    rng = np.random.default_rng(31)
    theta = rng.normal(size=200).astype(np.float32)
    grads = [(rng.normal(size=200) * 10.0 ** rng.uniform(-6, 1, size=200)).astype(np.float32)
             for _ in range(6)]
    ref = _adam_f64(theta, grads, 1e-3)
    p, m, v = theta, np.zeros_like(theta), np.zeros_like(theta)
    for t, gt in enumerate(grads, start=1):
        p, m, v = G.adam_step(p, m, v, gt, t, 1e-3)
        rp, rm, rv = ref[t - 1]
        assert np.allclose(m, rm, rtol=1e-5, atol=1e-30)
        assert np.allclose(v, rv, rtol=1e-5, atol=1e-30)
        assert np.allclose(p, rp, rtol=0, atol=1e-6)


def test_adam_bias_correction_values():
    assert G.adam_bias_correction(0.9, 1) == np.float32(1.0) - np.float32(0.9)
    assert abs(float(G.adam_bias_correction(0.999, 1)) - 0.001) < 1e-7
    assert abs(float(G.adam_bias_correction(0.9, 50)) - (1 - 0.9 ** 50)) < 1e-7


def test_weight_copies_layout():
    params = G.glorot(2)
    wb = G.weight_copies(params)
    assert wb.dtype == np.uint16 and wb.size == 32 * 64 + 128 * 64 + 128 * 64
    P = G.unflatten(params)
    # first entry of W2 in the copies is W2[0][0] rounded to BF16
    w = np.float32(P["W2"][0, 0])
    assert wb[32 * 64] == (G.bf16(w).astype(np.float32).view(np.uint32) >> 16)
