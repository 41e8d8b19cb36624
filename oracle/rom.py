"""Spatial and space-time reduced operators (oracle, test infrastructure only).

Sec. 3 (Galerkin ROMs) and Sec. 4.3 (block structure of the space-time
basis).  Two index orders appear:

* paper order: column i + n_s (j - 1) of Phi_st is phi^t_ij (x) phi^s_i
  (Eq. (spacetimebasis), (spacetimebasisvec)); needs one n_t for all modes;
* mode-major order: mode i's n_t,i columns are contiguous, which also
  covers a different n_t,i per mode (the Kronecker definition of each column
  is unchanged; the reduced system is the same up to a symmetric permutation).

Reading of Eq. (first-block-initial-vector): the printed formula puts
(sum_k D_k^1) u0hat in the first block and zeros elsewhere.  Projecting
u0_st = [u0; 0; ...; 0] onto the Kronecker columns gives phi^t_ij(1) (phi^s_i . u0)
for every (i, j) instead, i.e. block j equals D_1^j u0hat.  The brute-force
projection decides: ``initial_vector_printed`` keeps the printed form for the
test that shows the mismatch, ``initial_vector`` is the projection.
The reference state is zero for the space-time ROM (Eq. (ststateapproximation)
has none), so u0hat = Phi_s^T u0.
"""
import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# spatial Galerkin ROM, Sec. 3.1
# ----------------------------------------------------------------------------

def spatial_operator(Phi_s, A):
    """Eq. (galerkin): Ahat = Phi_s^T A Phi_s."""
    return Phi_s.T @ (A @ Phi_s)


def reduced_vector(Phi_s, b):
    """Eq. (galerkin): Bhat = Phi_s^T B (and u0hat = Phi_s^T u0 with u_ref = 0)."""
    return Phi_s.T @ b


def spatial_rom_march(Ahat, BF_hat, u0hat, dt):
    """Eq. (space_reduced_discretized_ODE) with u_ref = 0:
    (I - dt_k Ahat) uhat^(k) = uhat^(k-1) + dt_k Bhat f^(k).
    BF_hat is n_s x N_t (column k = Bhat f^(k)).  Returns n_s x N_t."""
    n = Ahat.shape[0]
    u = np.array(u0hat, dtype=np.float64)
    out = np.zeros((n, len(dt)))
    for k in range(len(dt)):
        u = np.linalg.solve(np.eye(n) - dt[k] * Ahat, u + dt[k] * BF_hat[:, k])
        out[:, k] = u
    return out


def spatial_rom_output(Chat, U_hat):
    """Eq. (outputFromReducedsol) with u_ref = 0: y^(k) = Chat^T uhat^(k),
    Chat = Phi_s^T C (N_s x n_out output matrix C).  U_hat is n_s x N_t;
    returns n_out x N_t."""
    return np.asarray(Chat).T @ np.asarray(U_hat)


# ----------------------------------------------------------------------------
# explicit space-time basis (small sizes), Sec. 3.2 / 4.1
# ----------------------------------------------------------------------------

def spacetime_basis(Phi_s, Phi_t, order="mode"):
    """Eq. (spacetimebasisvec): phi^st_(i,j) = phi^t_ij (x) phi^s_i, formed
    explicitly (N_s N_t rows: small sizes only).

    Phi_t is a list of per-mode temporal bases (N_t x n_t,i).  order="paper"
    (uniform n_t) returns columns i + n_s j; order="mode" mode-major."""
    n_s = Phi_s.shape[1]
    cols = []
    if order == "paper":
        n_t = Phi_t[0].shape[1]
        assert all(P.shape[1] == n_t for P in Phi_t)
        for j in range(n_t):
            for i in range(n_s):
                cols.append(np.kron(Phi_t[i][:, j], Phi_s[:, i]))
    else:
        for i in range(n_s):
            for j in range(Phi_t[i].shape[1]):
                cols.append(np.kron(Phi_t[i][:, j], Phi_s[:, i]))
    return np.stack(cols, axis=1)


def project_space_time(Phi_st, A_st, f_st, u0_st):
    """Eq. (st-galerkin): Ahat_st = Phi_st^T A_st Phi_st, fhat_st = Phi_st^T f_st,
    u0hat_st = Phi_st^T u0_st (brute force)."""
    A_st = sp.csr_matrix(A_st)
    return Phi_st.T @ (A_st @ Phi_st), Phi_st.T @ f_st, Phi_st.T @ u0_st


# ----------------------------------------------------------------------------
# block formulas, Sec. 4.3, paper order (uniform n_t)
# ----------------------------------------------------------------------------

def D(Phi_t, k, j):
    """Eq. (temporaldiagonal): D_k^j = diag(phi^t_1j(k), ..., phi^t_nsj(k))."""
    return np.diag([P[k, j] for P in Phi_t])


def block_operator_paper(Ahat, Phi_t, dt):
    """Eq. (block-reduced-state-mat), (ij-block-matrix), paper order:
    block (j', j) = sum_k (D_k^j' D_k^j - dt_k D_k^j' Ahat D_k^j)
                    - sum_{k < N_t} D_{k+1}^j' D_k^j."""
    n_s = Ahat.shape[0]
    n_t = Phi_t[0].shape[1]
    N_t = Phi_t[0].shape[0]
    M = np.zeros((n_s * n_t, n_s * n_t))
    for jp in range(n_t):
        for j in range(n_t):
            blk = np.zeros((n_s, n_s))
            for k in range(N_t):
                blk += D(Phi_t, k, jp) @ D(Phi_t, k, j) - dt[k] * D(Phi_t, k, jp) @ Ahat @ D(Phi_t, k, j)
            for k in range(N_t - 1):
                blk -= D(Phi_t, k + 1, jp) @ D(Phi_t, k, j)
            M[jp * n_s:(jp + 1) * n_s, j * n_s:(j + 1) * n_s] = blk
    return M


def input_vector_paper(BF_hat, Phi_t, dt):
    """Eq. (block-reduced-input-vec), (j-block-vector), paper order:
    block j = sum_k dt_k D_k^j Bhat f^(k).  BF_hat: n_s x N_t."""
    n_t = Phi_t[0].shape[1]
    N_t = Phi_t[0].shape[0]
    out = []
    for j in range(n_t):
        b = np.zeros(BF_hat.shape[0])
        for k in range(N_t):
            b += dt[k] * (D(Phi_t, k, j) @ BF_hat[:, k])
        out.append(b)
    return np.concatenate(out)


def input_vector_constant_paper(Bf_hat, Phi_t, dt):
    """Eq. (j-block-vector-constant-input): block j = (sum_k dt_k D_k^j) Bhat f."""
    n_t = Phi_t[0].shape[1]
    N_t = Phi_t[0].shape[0]
    return np.concatenate([sum(dt[k] * D(Phi_t, k, j) for k in range(N_t)) @ Bf_hat for j in range(n_t)])


def initial_vector_printed(u0hat, Phi_t):
    """Eq. (block-reduced-initial-vec), (first-block-initial-vector) as printed:
    block 1 = (sum_k D_k^1) u0hat, other blocks zero (does not equal the
    projection; see the module header)."""
    n_s = u0hat.shape[0]
    n_t = Phi_t[0].shape[1]
    N_t = Phi_t[0].shape[0]
    out = np.zeros(n_s * n_t)
    out[:n_s] = sum(D(Phi_t, k, 0) for k in range(N_t)) @ u0hat
    return out


def initial_vector_paper(u0hat, Phi_t):
    """Projection of u0_st (paper order): block j = D_1^j u0hat."""
    n_t = Phi_t[0].shape[1]
    return np.concatenate([D(Phi_t, 0, j) @ u0hat for j in range(n_t)])


# ----------------------------------------------------------------------------
# block formulas in mode-major order (per-mode n_t,i)
# ----------------------------------------------------------------------------

def mode_offsets(Phi_t):
    return np.concatenate([[0], np.cumsum([P.shape[1] for P in Phi_t])]).astype(np.int64)


def block_operator(Ahat, Phi_t, dt):
    """Eq. (ij-block-matrix) written per spatial-mode pair (i', i), mode-major:
    the (j', j) entry of block (i', i) is
        delta_i'i sum_k phi^t_i'j'(k) phi^t_ij(k)
      - Ahat[i', i] sum_k dt_k phi^t_i'j'(k) phi^t_ij(k)
      - delta_i'i sum_{k < N_t} phi^t_i'j'(k+1) phi^t_ij(k),
    i.e. the (i', i) entry of each diagonal-matrix product in Eq.
    (ij-block-matrix)."""
    off = mode_offsets(Phi_t)
    n = int(off[-1])
    n_s = len(Phi_t)
    M = np.zeros((n, n))
    for ip in range(n_s):
        for i in range(n_s):
            Pp, P = Phi_t[ip], Phi_t[i]
            blk = -Ahat[ip, i] * (Pp.T @ (dt[:, None] * P))
            if ip == i:
                blk = blk + Pp.T @ P - Pp[1:].T @ P[:-1]
            M[off[ip]:off[ip + 1], off[i]:off[i + 1]] = blk
    return M


def input_vector(BF_hat, Phi_t, dt):
    """Eq. (j-block-vector), mode-major: entry (i, j) = sum_k dt_k phi^t_ij(k)
    (Bhat f^(k))_i.  BF_hat: n_s x N_t."""
    return np.concatenate([P.T @ (dt * BF_hat[i]) for i, P in enumerate(Phi_t)])


def initial_vector(u0hat, Phi_t):
    """Projection of u0_st, mode-major: entry (i, j) = phi^t_ij(1) u0hat_i."""
    return np.concatenate([P[0] * u0hat[i] for i, P in enumerate(Phi_t)])


def solve(Ast, rhs):
    """Eq. (st-galerkin): Ahat_st c = fhat_st + u0hat_st, LAPACK gesv
    (LU with partial pivoting)."""
    return np.linalg.solve(Ast, rhs)


def reconstruct(Phi_s, Phi_t, c):
    """Eq. (ststateapproximation): u^(k) ~ sum_i phi^s_i sum_j phi^t_ij(k) c_ij
    (mode-major c).  Returns N_s x N_t."""
    off = mode_offsets(Phi_t)
    Z = np.stack([Phi_t[i] @ c[off[i]:off[i + 1]] for i in range(len(Phi_t))], axis=0)  # n_s x N_t
    return Phi_s @ Z


# ----------------------------------------------------------------------------
# whole reduced system for a parameter (mode-major), from spatial pieces
# ----------------------------------------------------------------------------

def reduced_system(Ahat_terms, theta_A, bhat_terms, theta_f, g, u0hat_terms, theta_0, Phi_t, dt):
    """Assemble Ahat_st(mu), fhat_st(mu) + u0hat_st(mu) for affine data:
    Ahat(mu) = sum_q theta_A[q] Ahat_q, Bhat f^(k) = sum_q theta_f[q] g[k, q] bhat_q,
    u0hat = sum_q theta_0[q] u0hat_q.  Returns (Ahat_st, rhs)."""
    n_s = len(Phi_t)
    Ahat = sum(theta_A[q] * Ahat_terms[q] for q in range(len(Ahat_terms)))
    BF = np.zeros((n_s, len(dt)))
    for q in range(len(theta_f)):
        BF += theta_f[q] * np.outer(bhat_terms[:, q], g[:, q])
    u0hat = np.zeros(n_s)
    for q in range(len(theta_0)):
        u0hat += theta_0[q] * u0hat_terms[:, q]
    return block_operator(Ahat, Phi_t, dt), input_vector(BF, Phi_t, dt) + initial_vector(u0hat, Phi_t)
