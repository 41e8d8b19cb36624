"""FP64 reference of the surrogate network (oracle, test infrastructure only).

The paper has no learned component; this is the reference for the surrogate
that maps a parameter to reduced space-time coefficients.  Architecture:
x (d_in) -> [Linear, GELU] x n_hidden -> Linear -> y (d_out), GELU in its erf
form gelu(z) = z/2 (1 + erf(z / sqrt 2)).  Samples are rows: Z = X W^T + b with
W stored out x in.  Loss: mean squared error over all outputs of the batch.
Optimizer: Adam (Kingma and Ba) with bias correction.
"""
import math

import numpy as np
from scipy.special import erf

INV_SQRT2 = 1.0 / math.sqrt(2.0)
INV_SQRT2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z * INV_SQRT2))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z) (standard normal cdf and pdf)."""
    return 0.5 * (1.0 + erf(z * INV_SQRT2)) + z * INV_SQRT2PI * np.exp(-0.5 * z * z)


def forward(params, X):
    """params: list of (W, b).  Returns (Y, cache) with cache = (inputs, pre-activations)."""
    h = np.asarray(X, dtype=np.float64)
    hs, zs = [h], []
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        zs.append(z)
        h = gelu(z) if li < len(params) - 1 else z
        hs.append(h)
    return h, (hs, zs)


def mse(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(params, cache, Y, T):
    """Hand-derived gradients of mse(Y, T) w.r.t. every (W, b)."""
    hs, zs = cache
    d = 2.0 * (Y - T) / Y.size
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        if li < len(params) - 1:
            d = d * gelu_grad(zs[li])
        grads[li] = (d.T @ hs[li], d.sum(axis=0))
        d = d @ W
    return grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place.  state: dict with 't' and per-parameter m, v."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    if "m" not in state:
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    for li in range(len(params)):
        newp = []
        for pi in range(2):
            p = params[li][pi]
            g = grads[li][pi]
            m = state["m"][li][pi]
            v = state["v"][li][pi]
            m[...] = beta1 * m + (1.0 - beta1) * g
            v[...] = beta2 * v + (1.0 - beta2) * g * g
            p[...] = p - lr * (m / c1) / (np.sqrt(v / c2) + eps)
            newp.append(p)
    return params


def init_params(sizes, rng):
    """He-style init: W ~ N(0, 2/fan_in), b = 0."""
    out = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append((rng.standard_normal((b, a)) * math.sqrt(2.0 / a), np.zeros(b)))
    return out
