"""Shared seeded test cases: problems, snapshots, oracle bases, oracle systems.

Both sides receive the same arrays; expected values come from the oracle only.
"""
import functools

import numpy as np

from oracle import pod, rom
from paper_1910_01260_amd import workloads as W


@functools.lru_cache(maxsize=None)
def problem(name):
    if name == "c1":
        return W.advdiff1d()
    if name == "cb":
        return W.advdiff1d(n_train=32)
    if name == "c2":
        return W.transport2d()
    if name == "c2_small":
        return W.transport2d(nx=32, N_t=100)
    if name == "cs":
        return W.transport2d_absorber()
    if name == "cs_small":
        return W.transport2d_absorber(nx=16, N_t=60)
    if name == "c_long":
        # 40 modes x 320 steps: the residual's n_s x N_t arrays exceed LDS (gather path)
        return W.advdiff1d(N=128, N_t=320, n_train=4)
    raise KeyError(name)


BASIS_SIZES = {"c1": (8, 8), "cb": (40, 32), "c2": (40, 20), "c2_small": (20, 12), "cs": (40, 30),
               "cs_small": (12, 10), "c_long": (40, 4)}


@functools.lru_cache(maxsize=None)
def snapshots(name):
    return W.snapshots(problem(name))


@functools.lru_cache(maxsize=None)
def oracle_bases(name, tau_t=1e-7):
    """Oracle POD (thin SVD) and temporal bases with completion."""
    prob = problem(name)
    n_s, n_t = BASIS_SIZES[name]
    U = snapshots(name)
    Phi_s, sigma, V = pod.pod(U, n_s)
    Phi_t, ranks = pod.temporal_bases(V, prob.N_t, len(prob.train_mu), np.full(n_s, n_t), tau_t)
    return Phi_s, sigma, V, Phi_t, ranks


@functools.lru_cache(maxsize=None)
def oracle_spatial(name):
    prob = problem(name)
    Phi_s = oracle_bases(name)[0]
    Ahat = [rom.spatial_operator(Phi_s, A) for A in prob.terms]
    bhat = rom.reduced_vector(Phi_s, prob.Bf) if prob.Qf else np.zeros((Phi_s.shape[1], 0))
    u0hat = rom.reduced_vector(Phi_s, prob.u0) if prob.Q0 else np.zeros((Phi_s.shape[1], 0))
    return Ahat, bhat, u0hat


def oracle_system(name, theta_A, theta_f, theta_0, nt=None):
    """Oracle reduced system of one query (nt: per-mode prefix sizes or None)."""
    prob = problem(name)
    Phi_t = oracle_bases(name)[3]
    if nt is not None:
        Phi_t = [Phi_t[i][:, :int(nt[i])] for i in range(len(Phi_t))]
    Ahat, bhat, u0hat = oracle_spatial(name)
    return rom.reduced_system(Ahat, theta_A, bhat, theta_f, prob.g, u0hat, theta_0, Phi_t, prob.dt)
