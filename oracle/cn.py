"""Crank-Nicolson variant of the space-time ROM (oracle, test infrastructure only).

The paper treats backward Euler and notes that other time integrators give
space-time systems of other block structure (Sec. 2).  With the trapezoidal
rule the full-order step is
    (I - dt_k/2 A) u^(k) = (I + dt_k/2 A) u^(k-1) + dt_k B f^(k),
where f^(k) is the input of step k (the trapezoidal average of the input at
the step's two ends when the input varies in time).  The space-time matrix is
lower block-bidiagonal with diagonal blocks I - dt_k/2 A and sub-diagonal
blocks -(I + dt_k/2 A) (the sub-diagonal of row k carries that row's step),
f_st stacks dt_k B f^(k), and u0_st = [(I + dt_1/2 A) u^(0); 0; ...].

Its Galerkin projection with the Kronecker space-time basis keeps the block
structure of Sec. 4.3 with one more temporal contraction: for spatial modes
(i', i) and temporal vectors (j', j),
    delta_i'i [sum_k phi_i'j'(k) phi_ij(k) - sum_{k>1} phi_i'j'(k) phi_ij(k-1)]
  - Ahat[i', i] [ (1/2) sum_k dt_k phi_i'j'(k) phi_ij(k)
                  + (1/2) sum_{k>1} dt_k phi_i'j'(k) phi_ij(k-1) ],
the input vector is that of backward Euler, and the initial vector has the
entries phi_ij(1) (Phi_s^T (I + dt_1/2 A) u^(0))_i.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def crank_nicolson(A, F, u0, dt):
    """Full-order trapezoidal march; F: N x N_t step inputs B f^(k).
    Returns [u^(1) ... u^(N_t)] (N x N_t)."""
    A = sp.csc_matrix(A)
    N = A.shape[0]
    I = sp.identity(N, format="csc")
    u = np.array(u0, dtype=np.float64)
    out = np.zeros((N, len(dt)))
    for k in range(len(dt)):
        h = float(dt[k])
        u = spla.spsolve(sp.csc_matrix(I - 0.5 * h * A), (I + 0.5 * h * A) @ u + h * F[:, k])
        out[:, k] = u
    return out


def space_time_system(A, F, u0, dt):
    """Explicit Crank-Nicolson space-time system (time-major stacking, small sizes)."""
    A = sp.csr_matrix(A)
    N = A.shape[0]
    Nt = len(dt)
    I = sp.identity(N, format="csr")
    blocks = [[None] * Nt for _ in range(Nt)]
    for k in range(Nt):
        blocks[k][k] = I - 0.5 * dt[k] * A
        if k > 0:
            blocks[k][k - 1] = -(I + 0.5 * dt[k] * A)
    A_st = sp.bmat(blocks, format="csr")
    f_st = np.concatenate([dt[k] * F[:, k] for k in range(Nt)])
    u0_st = np.zeros(N * Nt)
    u0_st[:N] = (I + 0.5 * dt[0] * A) @ u0
    return A_st, f_st, u0_st


def _offsets(Phi_t):
    return np.concatenate([[0], np.cumsum([P.shape[1] for P in Phi_t])]).astype(np.int64)


def block_operator(Ahat, Phi_t, dt):
    """Reduced Crank-Nicolson space-time operator, mode-major (module header)."""
    off = _offsets(Phi_t)
    n = int(off[-1])
    n_s = len(Phi_t)
    M = np.zeros((n, n))
    for ip in range(n_s):
        for i in range(n_s):
            Pp, P = Phi_t[ip], Phi_t[i]
            tw = 0.5 * (Pp.T @ (dt[:, None] * P) + Pp[1:].T @ (dt[1:, None] * P[:-1]))
            blk = -Ahat[ip, i] * tw
            if ip == i:
                blk = blk + Pp.T @ P - Pp[1:].T @ P[:-1]
            M[off[ip]:off[ip + 1], off[i]:off[i + 1]] = blk
    return M


def initial_vector(u0hat, Au0hat, Phi_t, dt):
    """Entries phi_ij(1) (u0hat + dt_1/2 Au0hat)_i with u0hat = Phi_s^T u^(0) and
    Au0hat = Phi_s^T A u^(0)."""
    v = u0hat + 0.5 * dt[0] * Au0hat
    return np.concatenate([P[0] * v[i] for i, P in enumerate(Phi_t)])


def input_vector(BF_hat, Phi_t, dt):
    """Entries sum_k dt_k phi_ij(k) (Bhat f^(k))_i (as backward Euler)."""
    return np.concatenate([P.T @ (dt * BF_hat[i]) for i, P in enumerate(Phi_t)])


def reduced_system(Ahat_terms, theta_A, bhat_terms, theta_f, g, u0hat_terms, Au0hat_terms, theta_0, Phi_t, dt):
    """Reduced Crank-Nicolson system for affine data (as rom.reduced_system), with
    Au0hat_terms[q] = Phi_s^T A_q u0_q0 (n_s x Q0 per affine term q)."""
    n_s = len(Phi_t)
    Ahat = sum(theta_A[q] * Ahat_terms[q] for q in range(len(Ahat_terms)))
    BF = np.zeros((n_s, len(dt)))
    for q in range(len(theta_f)):
        BF += theta_f[q] * np.outer(bhat_terms[:, q], g[:, q])
    u0hat = np.zeros(n_s)
    Au0 = np.zeros(n_s)
    for q0 in range(len(theta_0)):
        u0hat += theta_0[q0] * u0hat_terms[:, q0]
        for q in range(len(Ahat_terms)):
            Au0 += theta_A[q] * theta_0[q0] * Au0hat_terms[q][:, q0]
    return (block_operator(Ahat, Phi_t, dt),
            input_vector(BF, Phi_t, dt) + initial_vector(u0hat, Au0, Phi_t, dt))
