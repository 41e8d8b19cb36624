"""Learned surrogate of the reduced space-time solve, with a certified check.

Not part of the paper's method.  A multilayer perceptron maps the (scaled)
parameter mu to the reduced space-time coefficients c of Eq. (st-galerkin).
Every prediction is certified by the FP64 residual of the reduced system:
with sym(A) <= 0 the symmetric part of Ahat_st is bounded below by
gamma = 1 - cos(pi / (N_t + 1)) (the backward-Euler space-time matrix of
Sec. 2 dominates a tridiagonal Toeplitz matrix, and the orthonormal Galerkin
projection of Sec. 3.2 keeps the bound), so

    ||c - c*|| / ||c*|| <= e / (1 - e),   e = ||b - Ahat_st c|| / (gamma ||c||).

Queries whose certificate exceeds the tolerance fall back to the batched
reduced solve (st_solve with those queries not skipped).

Training, inference, the certificate and the fallback all run in the
library's kernels; this module only holds parameters, moves data and loops.
"""
import ctypes
import math
from typing import Optional

import numpy as np
import torch

from . import strom


def coercivity_floor(N_t: int) -> float:
    """Smallest eigenvalue of tridiag(-1/2, 1, -1/2) of order N_t: a lower bound
    of lambda_min(sym Ahat_st) when sym(A) <= 0 (st_coercivity_floor)."""
    return strom.st_coercivity_floor(N_t)


def scaled_inputs(box_lo, box_hi, mus) -> np.ndarray:
    """Parameters mapped affinely from their box to [-1, 1]^d (FP32 network input)."""
    lo = np.asarray(box_lo, dtype=np.float64)
    hi = np.asarray(box_hi, dtype=np.float64)
    return np.ascontiguousarray((2.0 * (np.atleast_2d(mus) - lo) / (hi - lo) - 1.0).astype(np.float32))


class Surrogate:
    """MLP d_in -> [width, GELU] x n_hidden -> d_out on the device.

    FP32 master parameters (one flat array in the library's order: W_1, b_1,
    W_2, ...), Adam moments, and the output standardisation (mean, scale) that
    maps network outputs to coefficients."""

    def __init__(self, d_in: int, d_out: int, width: int = 512, n_hidden: int = 4, seed: int = 191001263,
                 device="cuda"):
        self.shape = strom.mlp_shape(d_in, width, n_hidden, d_out)
        self.device = device
        self.n_params = strom.st_mlp_param_count(self.shape)
        rng = np.random.default_rng(seed)
        sizes = [d_in] + [width] * n_hidden + [d_out]
        flat = []
        for a, b in zip(sizes[:-1], sizes[1:]):
            flat.append((rng.standard_normal((b, a)) * math.sqrt(2.0 / a)).astype(np.float32).ravel())
            flat.append(np.zeros(b, dtype=np.float32))
        flat = np.concatenate(flat)
        assert flat.size == self.n_params
        self.params = torch.tensor(flat, device=device)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.step = 0
        self.mean: Optional[torch.Tensor] = None
        self.scale: Optional[torch.Tensor] = None
        self._ws = {}

    # -- workspace --------------------------------------------------------------
    def workspace(self, batch: int):
        if batch not in self._ws:
            nb = strom.lib().st_mlp_workspace(ctypes.byref(self.shape), int(batch))
            self._ws[batch] = (torch.empty(max(nb, 1), dtype=torch.uint8, device=self.device), nb)
        return self._ws[batch]

    # -- standardisation ----------------------------------------------------------
    def set_standardization(self, C):
        """Per-coefficient mean and standard deviation of the training targets
        (n x d FP64, host or device; st_mlp_colstats)."""
        C = torch.as_tensor(C, dtype=torch.float64, device=self.device)
        self.mean, self.scale = strom.st_mlp_colstats(C)

    def standardize(self, C) -> torch.Tensor:
        """FP32 training targets (C - mean) / scale on the device (st_mlp_standardize)."""
        C = torch.as_tensor(C, dtype=torch.float64, device=self.device)
        return strom.st_mlp_standardize(C, self.mean, self.scale)

    # -- training ------------------------------------------------------------------
    def train_step(self, X: torch.Tensor, T: torch.Tensor, lr: float):
        """One Adam step on the mean squared error of network(X) against T."""
        ws = self.workspace(int(X.shape[0]))
        strom.st_mlp_grad(self.shape, self.params, X, T, self.grads, self.loss, ws)
        self.step += 1
        strom.st_mlp_adam(self.params, self.grads, self.m, self.v, self.step, lr)

    def fit(self, X: np.ndarray, C: np.ndarray, steps: int, batch: int = 1024, lr: float = 1e-3,
            lr_final: float = 1e-5, val_frac: float = 0.1, seed: int = 191001264, log=None):
        """Train on (X, C) (host arrays, C in coefficients): standardise C, hold out
        val_frac for validation, and run `steps` Adam steps on shuffled minibatches
        with a cosine learning-rate decay from lr to lr_final.  Returns the
        history of (step, train loss, validation loss)."""
        n = X.shape[0]
        rng = np.random.default_rng(seed)
        perm = rng.permutation(n)
        n_val = max(1, int(round(val_frac * n)))
        val, tr = perm[:n_val], perm[n_val:]
        self.set_standardization(C[tr])
        T_all = self.standardize(C)
        Xv = torch.tensor(X[val], device=self.device)
        Tv = T_all[torch.as_tensor(val, device=self.device)].contiguous()
        batch = min(batch, len(tr))
        n_b = len(tr) // batch
        # one epoch of minibatches lives on the device; reshuffled on the host per epoch
        Xe = torch.empty((n_b * batch, X.shape[1]), dtype=torch.float32, device=self.device)
        Te = torch.empty((n_b * batch, C.shape[1]), dtype=torch.float32, device=self.device)
        history = []
        step = 0
        while step < steps:
            order = tr[rng.permutation(len(tr))[:n_b * batch]]
            Xe.copy_(torch.from_numpy(np.ascontiguousarray(X[order])))
            Te.copy_(T_all[torch.as_tensor(order, device=self.device)])
            for b in range(n_b):
                if step >= steps:
                    break
                frac = step / max(1, steps - 1)
                lr_t = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * frac))
                self.train_step(Xe[b * batch:(b + 1) * batch], Te[b * batch:(b + 1) * batch], lr_t)
                step += 1
                if step % max(1, steps // 20) == 0 or step == steps:
                    tl = float(self.loss.item())
                    vl = self.validation_loss(Xv, Tv)
                    history.append((step, tl, vl))
                    if log:
                        log(f"step {step}: train {tl:.3e} val {vl:.3e}")
        return history

    def validation_loss(self, Xv: torch.Tensor, Tv: torch.Tensor) -> float:
        """Mean squared error on held-out samples (the grad call's loss; the
        gradient it also writes goes to a scratch buffer)."""
        scratch = torch.empty_like(self.grads)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        strom.st_mlp_grad(self.shape, self.params, Xv, Tv, scratch, loss, self.workspace(int(Xv.shape[0])))
        return float(loss.item())

    # -- inference + certificate + fallback -------------------------------------------------
    def predict(self, X: torch.Tensor) -> torch.Tensor:
        return strom.st_mlp_forward(self.shape, self.params, X, self.workspace(int(X.shape[0])))

    def check(self, desc, rom, theta_A, theta_f, theta_0, Y, gamma: float, tol: float, coeff: torch.Tensor):
        """Write the de-standardised coefficients of Y into coeff (full-width
        packing) and return (cert, accept)."""
        n_q = int(theta_A.shape[0])
        cert = torch.empty(max(n_q, 1), dtype=torch.float64, device=self.device)
        accept = torch.empty(max(n_q, 1), dtype=torch.int32, device=self.device)
        strom.st_surrogate_check(desc, rom, theta_A, theta_f, theta_0, Y, self.mean, self.scale, gamma, tol, coeff,
                                 cert, accept)
        return cert, accept

    def solve(self, desc, rom, theta_A, theta_f, theta_0, X: torch.Tensor, gamma: float, tol: float,
              bufs: strom.SolveBuffers, lu_prec: int = strom.ST_F64, ir_tol: float = 0.0, ir_max: int = 0):
        """Surrogate + certificate; the rejected queries are solved by st_solve
        into the same coefficient buffer.  info[q] = -2 marks accepted
        predictions.  Returns (bufs, cert, accept)."""
        Y = self.predict(X)
        cert, accept = self.check(desc, rom, theta_A, theta_f, theta_0, Y, gamma, tol, bufs.coeff)
        strom.st_solve(desc, rom, theta_A, theta_f, theta_0, None, lu_prec, ir_tol, ir_max, bufs=bufs, skip=accept)
        return bufs, cert, accept

