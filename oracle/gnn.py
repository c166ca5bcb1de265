"""FP64 oracle of the learned surrogate (test infrastructure only).

The network is the mean-aggregation message-passing model of the library's
surrogate (message = neighbour state, aggregation = mean over in-neighbours,
update = ReLU of a linear map of [own state | aggregate]; the structure of the
paper's Eq. ms / Eq. agg / Eq. updata with learned functions):

    x_v  = [seed_v, 20 beta, log1p(indeg_v) / 8, 1, 20 beta log1p(indeg_v) / 8,
            log1p(k) / 8, log1p(D) / 16, 0 x 9]
           (k = number of seeds, D = sum of the seeds' in-degrees)
    h1_v = ReLU(W1^T [x_v  | mean_{u in N-(v)} x_u ] + b1)
    h2_v = ReLU(W2^T [h1_v | mean h1_u] + b2)
    h3_v = ReLU(W3^T [h2_v | mean h2_u] + b3)
    p_v  = sigmoid(wo . h3_v + bo)
    loss = mean_v BCE(p_v, y_v)

Written in float64 with plain numpy.  With ``bf16=True`` the values are
rounded to bfloat16 (round to nearest even) at the points where the GPU
stores them in bfloat16: inputs, aggregates, post-ReLU activations, weights
used by the products, and the pre-activation gradient fed to the products.

The optimiser is Adam (Kingma and Ba, ICLR 2015) on single-precision master
weights: ``adam_step``, every operation in single precision.
"""
from __future__ import annotations

import numpy as np

F0, HID = 16, 64
K1, K2 = 2 * F0, 2 * HID
SHAPES = [("W1", (K1, HID)), ("b1", (HID,)), ("W2", (K2, HID)), ("b2", (HID,)),
          ("W3", (K2, HID)), ("b3", (HID,)), ("wo", (HID,)), ("bo", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(flat):
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to bfloat16 (nearest even) through float32, returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def _ident(x):
    return np.asarray(x, dtype=np.float64)


def mean_agg(X, ptr, src):
    """mean_{u in N-(v)} X[u] for every row v (0 for an empty neighbourhood)."""
    n = len(ptr) - 1
    out = np.zeros((n,) + X.shape[1:])
    for v in range(n):
        e0, e1 = ptr[v], ptr[v + 1]
        if e1 > e0:
            out[v] = X[src[e0:e1]].mean(axis=0)
    return out


def mean_agg_T(G, ptr, src):
    """Transpose of mean_agg: out[u] = sum_{v : u in N-(v)} G[v] / indeg(v)."""
    n = len(ptr) - 1
    out = np.zeros_like(G)
    for v in range(n):
        e0, e1 = ptr[v], ptr[v + 1]
        for e in range(e0, e1):
            out[src[e]] += G[v] / (e1 - e0)
    return out


def features(mask, beta, ptr):
    n = len(ptr) - 1
    indeg = np.diff(np.asarray(ptr)).astype(np.float64)
    seed = np.asarray(mask) != 0
    k = float(np.count_nonzero(seed))
    D = float(indeg[seed].sum())
    xb = 20.0 * float(np.float32(beta))
    xd = np.log1p(indeg) * 0.125
    X = np.zeros((n, F0))
    X[:, 0] = seed
    X[:, 1] = xb
    X[:, 2] = xd
    X[:, 3] = 1.0
    X[:, 4] = xb * xd
    X[:, 5] = np.log1p(k) * 0.125
    X[:, 6] = np.log1p(D) * 0.0625
    return X


def forward(params, ptr, src, mask, beta, bf=False):
    """One seed set.  Returns (p, cache)."""
    r = bf16 if bf else _ident
    P = unflatten(params)
    W = {k: r(P[k]) for k in ("W1", "W2", "W3")}
    x = r(features(mask, beta, ptr))
    X1 = np.concatenate([x, r(mean_agg(x, ptr, src))], axis=1)
    Z1 = X1 @ W["W1"] + P["b1"]
    h1 = r(np.maximum(Z1, 0))
    X2 = np.concatenate([h1, r(mean_agg(h1, ptr, src))], axis=1)
    Z2 = X2 @ W["W2"] + P["b2"]
    h2 = r(np.maximum(Z2, 0))
    X3 = np.concatenate([h2, r(mean_agg(h2, ptr, src))], axis=1)
    Z3 = X3 @ W["W3"] + P["b3"]
    h3 = r(np.maximum(Z3, 0))
    z = h3 @ P["wo"] + P["bo"][0]
    p = 1.0 / (1.0 + np.exp(-z))
    return p, dict(P=P, W=W, X=[X1, X2, X3], H=[h1, h2, h3], z=z)


def loss_and_grad(params, ptr, src, masks, betas, targets, bf=False):
    """Mean BCE over all rows of all seed sets and its gradient (flat)."""
    r = bf16 if bf else _ident
    n = len(ptr) - 1
    R = n * len(masks)
    G = {name: np.zeros(shape) for name, shape in SHAPES}
    total = 0.0
    for mask, beta, y in zip(masks, betas, targets):
        p, c = forward(params, ptr, src, mask, beta, bf)
        z = c["z"]
        y = np.asarray(y, dtype=np.float64)
        total += np.sum(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z))))
        dz = (p - y) / R
        P, W, X, H = c["P"], c["W"], c["X"], c["H"]
        G["wo"] += H[2].T @ dz
        G["bo"] += dz.sum()
        dH = np.outer(dz, P["wo"])
        for layer in (2, 1, 0):
            dZ = r(dH * (H[layer] > 0))
            wn = ("W1", "W2", "W3")[layer]
            G[("b1", "b2", "b3")[layer]] += dZ.sum(axis=0)
            G[wn] += X[layer].T @ dZ
            if layer > 0:
                dX = dZ @ W[wn].T
                dH = dX[:, :HID] + mean_agg_T(dX[:, HID:], ptr, src)
    return total / R, flatten(G)


def glorot(seed):
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            a = np.sqrt(6.0 / (shape[0] + shape[1]))
            d[name] = rng.uniform(-a, a, size=shape)
        elif name == "wo":
            d[name] = rng.uniform(-0.3, 0.3, size=shape)
        else:
            d[name] = rng.uniform(-0.1, 0.1, size=shape)
    return flatten(d)


# ------------------------------------------------------------------ Adam --
ADAM_BETA1, ADAM_BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_bias_correction(beta, t):
    """1 - beta^t in single precision: beta^t of the single-precision beta,
    rounded once to single precision, subtracted from 1 in single precision."""
    b = np.float32(beta)
    return np.float32(np.float32(1.0) - np.float32(np.float64(b) ** int(t)))


def adam_step(params, m, v, grad, t, lr, beta1=ADAM_BETA1, beta2=ADAM_BETA2, eps=ADAM_EPS):
    """Step t >= 1 of Adam (Kingma and Ba, ICLR 2015, Algorithm 1) on
    single-precision master weights, every operation rounded to single
    precision:

        m = beta1 m + (1 - beta1) g
        v = beta2 v + (1 - beta2) g^2
        m_hat = m / (1 - beta1^t),  v_hat = v / (1 - beta2^t)
        theta = theta - lr * (m_hat / (sqrt(v_hat) + eps))

    Returns new (params, m, v) as float32 arrays; the inputs are not changed."""
    f = np.float32
    p = np.asarray(params, dtype=np.float32)
    m = np.asarray(m, dtype=np.float32)
    v = np.asarray(v, dtype=np.float32)
    g = np.asarray(grad, dtype=np.float32)
    b1, b2, e, a = f(beta1), f(beta2), f(eps), f(lr)
    one = f(1.0)
    m_new = (b1 * m + (one - b1) * g).astype(np.float32)
    v_new = (b2 * v + (one - b2) * (g * g)).astype(np.float32)
    c1 = adam_bias_correction(beta1, t)
    c2 = adam_bias_correction(beta2, t)
    m_hat = (m_new / c1).astype(np.float32)
    v_hat = (v_new / c2).astype(np.float32)
    upd = (m_hat / (np.sqrt(v_hat) + e)).astype(np.float32)
    p_new = (p - a * upd).astype(np.float32)
    return p_new, m_new, v_new


def bf16_bits(x):
    """bfloat16 bit patterns (uint16) of x rounded to nearest even through
    float32 -- the BF16 weight copies the products use."""
    return (bf16(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def weight_copies(params):
    """BF16 bit patterns of W1, W2, W3 (row-major, in that order) of a flat
    parameter vector."""
    P = unflatten(params)
    return np.concatenate([bf16_bits(P[k].astype(np.float32)).ravel() for k in ("W1", "W2", "W3")])
