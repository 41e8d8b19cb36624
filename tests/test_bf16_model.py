"""CPU checks of the BF16 error model used by the device network tests.

1. A CPU emulation of the device arithmetic (BF16-rounded operands, FP32
   accumulation) stays inside the bounds.
2. Plausible mistakes planted in the oracle network (a dropped bias, a
   transposed or swapped weight, a missing GELU derivative, a wrong factor in
   the loss gradient, the pre-activation used in place of the activation)
   move some output or gradient well outside the bounds, so a device result
   carrying such a mistake cannot pass.
"""
import numpy as np
import pytest

from oracle import mlp as omlp

from . import _bf16_model as M


def _params(sizes, seed):
    rng = np.random.default_rng(seed)
    p = omlp.init_params(sizes, rng)
    return [(M.bf16_round(W), (0.1 * rng.standard_normal(b.shape)).astype(np.float32).astype(np.float64))
            for W, b in p]


def _data(sizes, batch, seed):
    rng = np.random.default_rng(seed)
    X = M.bf16_round(rng.uniform(-1, 1, (batch, sizes[0])))
    T = rng.standard_normal((batch, sizes[-1])).astype(np.float32).astype(np.float64)
    return X, T


CASES = [([3, 64, 64, 40], 100, 1), ([5, 33, 17], 70, 2), ([3, 96, 96, 96, 50], 64, 3)]


@pytest.mark.parametrize("sizes,batch,seed", CASES)
def test_emulated_device_arithmetic_within_bounds(sizes, batch, seed):
    params = _params(sizes, seed)
    X, T = _data(sizes, batch, seed)
    em = M.error_model(params, X, T)
    Ye, ge = M.emulate(params, X, T)
    r = np.abs(Ye - em["Y"]) / em["Y_bound"]
    assert r.max() <= 1.0, r.max()
    for l in range(len(params)):
        for k in range(2):
            r = np.abs(ge[l][k] - em["grads"][l][k]) / em["grad_bounds"][l][k]
            assert r.max() <= 1.0, (l, k, r.max())


def _backward_variant(params, cache, Y, T, variant):
    """The oracle's backward pass with one planted mistake."""
    hs, zs = cache
    scale = 1.0 if variant == "no_factor_two" else 2.0
    d = scale * (Y - T) / Y.size
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        if li < len(params) - 1 and variant != "no_gelu_grad":
            d = d * omlp.gelu_grad(zs[li])
        h_in = hs[li]
        if variant == "preact" and li > 0:
            h_in = zs[li - 1]
        gW = d.T @ h_in
        gb = d.mean(axis=0) if variant == "bias_mean" else d.sum(axis=0)
        grads[li] = (gW, gb)
        d = d @ W
    return grads


def _outside(a, ref, bound):
    return bool(np.any(np.abs(a - ref) > 2.0 * bound))


@pytest.mark.parametrize("sizes,batch,seed", CASES[:2])
def test_planted_mistakes_leave_the_bounds(sizes, batch, seed):
    params = _params(sizes, seed)
    X, T = _data(sizes, batch, seed)
    em = M.error_model(params, X, T)
    Y, cache = omlp.forward(params, X)
    # forward mistakes
    nob = [(W, b if l == len(params) - 1 else 0 * b) for l, (W, b) in enumerate(params)]
    assert _outside(omlp.forward(nob, X)[0], Y, em["Y_bound"])
    if sizes[1] == sizes[2]:
        tr = [(W.T.copy() if l == 1 else W, b) for l, (W, b) in enumerate(params)]
        assert _outside(omlp.forward(tr, X)[0], Y, em["Y_bound"])
    # backward mistakes
    for variant in ("no_gelu_grad", "no_factor_two", "bias_mean", "preact"):
        g = _backward_variant(params, cache, Y, T, variant)
        hit = any(_outside(g[l][k], em["grads"][l][k], em["grad_bounds"][l][k])
                  for l in range(len(params)) for k in range(2))
        assert hit, variant
    if sizes[1] == sizes[2]:
        g = em["grads"]
        assert _outside(g[1][0].T, g[1][0], em["grad_bounds"][1][0])


def test_bf16_rounding_ties_to_even():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to even (1.0)
    assert M.bf16_round(np.float32(1 + 2 ** -8)) == 1.0
    assert M.bf16_round(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6
    assert M.bf16_round(np.float32(1 + 2 ** -8 + 2 ** -20)) == 1 + 2 ** -7
    assert M.is_bf16(np.array([0.5, -3.0, 2 ** -100]))
