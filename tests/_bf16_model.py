"""First-order probabilistic rounding-error bounds for the BF16 surrogate network.

The device network rounds every FP32 operand of a matrix product to BF16
(round to nearest even, unit roundoff u = 2^-8), multiplies exactly and
accumulates in FP32.  With the inputs X and the weights W already
representable in BF16, the error sites of one sample are

  * each product output Z_l (FP32 accumulation of K terms plus the bias:
    at most (K + 1) 2^-24 (|H||W|^T + |b|)),
  * each hidden activation H_l (GELU evaluated in FP32, then rounded to BF16
    where it enters the next product and the dW product: u |H| + 4 2^-24 |H|),
  * each back-propagated dZ_l (FP32 loss gradient or GELU-derivative product,
    then rounded to BF16 for the dW and dH products),
  * each dH_l = dZ_l W_l (FP32 accumulation),

each carrying its own error e_s with |e_s| <= a_s, the same wherever the
value is used.  To first order every output q is the exact value plus
sum_s c_s(q) e_s / a_s with sensitivities c_s obtained by propagation through
the network.  Treating the e_s as independent, mean-zero and bounded (the
probabilistic model of Higham and Mary, SIAM J. Sci. Comput. 41 (2019)),
Hoeffding's inequality gives

  |q_dev - q| <= lam * sqrt(sum_s c_s(q)^2)

except with probability 2 exp(-lam^2 / 2) per output (lam = 8: 2.5e-14).
Samples have disjoint sites, so gradient sums over the batch add the
per-sample sums of squares; the dW and db sums themselves add a local
worst-case FP32 accumulation term.  A factor 1.1 covers second-order terms.

Reference values are the FP64 oracle network's.
"""
import numpy as np

from oracle import mlp as omlp

U_BF16 = 2.0 ** -8
U_F32 = 2.0 ** -24


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def is_bf16(a):
    return np.array_equal(bf16_round(a), np.asarray(a, dtype=np.float64))


def gelu_curv(z):
    """Second derivative of the erf GELU: phi(z) (2 - z^2)."""
    return np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi) * (2.0 - z * z)


def _site_sizes(params, X):
    """Per-layer error magnitudes of the forward sites (a_Z, a_H)."""
    Y, (hs, zs) = omlp.forward(params, X)
    aZ, aH = [], [None]
    for l, (Wm, b) in enumerate(params):
        aZ.append((Wm.shape[1] + 1) * U_F32 * (np.abs(hs[l]) @ np.abs(Wm).T + np.abs(b)))
        if l < len(params) - 1:
            aH.append((U_BF16 + 4 * U_F32) * np.abs(hs[l + 1]))
    return Y, hs, zs, aZ, aH


def forward_bound(params, X, lam=8.0):
    """Oracle output Y and the elementwise bound of the device forward pass
    (reverse-mode sensitivities, one Jacobian per sample)."""
    assert is_bf16(X) and all(is_bf16(Wm) for Wm, _ in params)
    Y, hs, zs, aZ, aH = _site_sizes(params, X)
    L = len(params)
    B, d_out = Y.shape
    J = np.broadcast_to(np.eye(d_out), (B, d_out, d_out))   # dY / dZ_{L-1}
    var = np.zeros((B, d_out))
    for l in range(L - 1, -1, -1):
        var += np.sum((J * aZ[l][:, None, :]) ** 2, axis=2)
        if l == 0:
            break
        JH = np.matmul(J, params[l][0])                       # dY / dH_l
        var += np.sum((JH * aH[l][:, None, :]) ** 2, axis=2)
        J = JH * omlp.gelu_grad(zs[l - 1])[:, None, :]
    return Y, 1.1 * lam * np.sqrt(var)


def error_model(params, X, T=None, lam=8.0):
    """Oracle outputs and elementwise bounds of the device forward pass and,
    with targets T, of the loss and its gradients (forward-mode sensitivities
    over all sites of a sample)."""
    Y, Yb = forward_bound(params, X, lam)
    out = {"Y": Y, "Y_bound": Yb}
    if T is None:
        return out
    _, hs, zs, aZ, aH = _site_sizes(params, X)
    L = len(params)
    B = X.shape[0]
    widths = [Wm.shape[0] for Wm, _ in params]
    offs, o = {}, 0
    for l in range(L):
        offs["Z", l] = o
        o += widths[l]
        offs["D", l] = o
        o += widths[l]
        if l >= 1:
            offs["H", l] = o
            o += widths[l - 1]
            offs["dH", l] = o
            o += widths[l - 1]
    ns = o

    def site(key, mag):
        S = np.zeros((B, mag.shape[1], ns))
        idx = np.arange(mag.shape[1])
        S[:, idx, offs[key] + idx] = mag
        return S

    # forward sensitivities (Z_l, and the rounded input H_l of layer l)
    SH = [np.zeros((B, X.shape[1], ns))]
    SZ = []
    for l, (Wm, b) in enumerate(params):
        SZ.append(np.matmul(Wm, SH[l]) + site(("Z", l), aZ[l]))
        if l < L - 1:
            SH.append(omlp.gelu_grad(zs[l])[:, :, None] * SZ[l] + site(("H", l + 1), aH[l + 1]))
    n = Y.size
    out["loss"] = omlp.mse(Y, T)
    grads = omlp.backward(params, (hs, zs), Y, T)
    out["grads"] = grads
    d = 2.0 * (Y - T) / n
    Sd = (2.0 / n) * SZ[-1]
    gb = [None] * L
    for l in range(L - 1, -1, -1):
        Wm, _ = params[l]
        # FP32 value of dZ_l (own rounding of the loss gradient or of dH * gelu'), then BF16 for the products
        Sdr = Sd + site(("D", l), (U_BF16 + 4 * U_F32) * np.abs(d))
        H = hs[l]
        SHl = SH[l]
        NH = np.sum(SHl ** 2, axis=2)
        ND = np.sum(Sdr ** 2, axis=2)
        C = np.matmul(Sdr, SHl.transpose(0, 2, 1))
        var_w = (d ** 2).T @ NH + ND.T @ (H ** 2) + 2.0 * np.sum(d[:, :, None] * H[:, None, :] * C, axis=0)
        var_w = np.maximum(var_w, 0.0)
        eW = 1.1 * lam * np.sqrt(var_w) + (B + 1) * U_F32 * (np.abs(d).T @ np.abs(H))
        SdF = Sd + site(("D", l), 4 * U_F32 * np.abs(d))   # colsum reads the FP32 dZ
        var_b = np.sum(np.sum(SdF ** 2, axis=2), axis=0)
        eb = 1.1 * lam * np.sqrt(var_b) + (B + 1) * U_F32 * np.abs(d).sum(axis=0)
        gb[l] = (eW, eb)
        if l > 0:
            dh = d @ Wm
            Sdh = np.matmul(Wm.T, Sdr) + site(("dH", l), (Wm.shape[0] + 1) * U_F32 * (np.abs(d) @ np.abs(Wm)))
            gp = omlp.gelu_grad(zs[l - 1])
            Sd = gp[:, :, None] * Sdh + (dh * gelu_curv(zs[l - 1]))[:, :, None] * SZ[l - 1]
            d = dh * gp
    out["grad_bounds"] = gb
    return out


def emulate(params, X, T=None):
    """CPU emulation of the device arithmetic model (BF16-rounded operands,
    FP32 products and accumulation, FP32 epilogues): used only to check the
    bounds above on the CPU."""
    f32 = np.float32

    def gemm(A, Bm):
        return (bf16_round(A).astype(f32) @ bf16_round(Bm).astype(f32)).astype(f32)

    from scipy.special import erf
    h = np.asarray(X, f32)
    hs, zs = [h], []
    for l, (Wm, b) in enumerate(params):
        z = (gemm(h, np.asarray(Wm, f32).T) + np.asarray(b, f32)).astype(f32)
        zs.append(z)
        if l < len(params) - 1:
            h = (f32(0.5) * z * (f32(1) + erf(z.astype(np.float64) / np.sqrt(2)).astype(f32))).astype(f32)
        else:
            h = z
        hs.append(h)
    Y = h
    if T is None:
        return Y
    n = Y.size
    d = (f32(2) * (Y - np.asarray(T, f32)) * f32(1.0 / n)).astype(f32)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        Wm, _ = params[l]
        grads[l] = (gemm(d.T, hs[l]), d.sum(axis=0, dtype=f32))
        if l > 0:
            z = zs[l - 1].astype(np.float64)
            gp = (0.5 * (1 + erf(z / np.sqrt(2))) + z * np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi)).astype(f32)
            d = (gemm(d, np.asarray(Wm, f32)) * gp).astype(f32)
    return Y, grads
