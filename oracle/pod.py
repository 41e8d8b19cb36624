"""Proper orthogonal decomposition (oracle, test infrastructure only).

Sec. 4.1: snapshot matrix, thin SVD, spatial basis, temporal snapshot
matrices and temporal bases.

Readings where the paper is silent (stated once here, mirrored by the HIP
path in code of its own):

* Signs.  Singular vectors are defined up to sign; the paper fixes none.  A
  vector is made to have a positive entry at the first index whose magnitude
  is at least one quarter of the vector's largest magnitude.  For spatial
  modes the pair (w_i, v_i) is flipped together, so U = W S V^T still holds.
* Temporal bases wider than the data.  The temporal snapshot matrix of mode
  i has only n_mu columns, so its SVD yields at most rank(Y_i) <= n_mu
  meaningful left vectors, while a basis of n_t > n_mu vectors is asked for.
  We read "the first n_t left singular vectors" as: keep the left singular
  vectors whose singular value exceeds tau_t times the largest (at most
  n_t of them), then complete with DCT-II vectors c_m(k) = cos(pi m (k+1/2)/N_t),
  m = 0, 1, 2, ..., each orthogonalised twice (classical Gram-Schmidt) against
  the vectors kept so far and accepted when at least 1e-2 of its norm
  survives.  Any orthonormal completion gives a valid Galerkin basis; this one
  is deterministic, so both implementations agree.
"""
import numpy as np

SIGN_FRACTION = 0.25
COMPLETION_KEEP = 1e-2


def sign_fix(v):
    """Sign convention: positive at the first entry with |v_k| >= max|v| / 4.
    Returns (sign, signed vector)."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    m = a.max() if a.size else 0.0
    if m == 0.0:
        return 1.0, v.copy()
    k = int(np.argmax(a >= SIGN_FRACTION * m))
    s = 1.0 if v[k] >= 0 else -1.0
    return s, s * v


def snapshot_matrix(trajectories):
    """Sec. 4.1, Eq. (snapshotmat): U = [U_1 ... U_nmu], U_p = [u^(1) ... u^(N_t)]
    at parameter mu_p (the initial state is not a column)."""
    return np.concatenate([np.asarray(t, dtype=np.float64) for t in trajectories], axis=1)


def pod(U, n_s):
    """Sec. 4.1, Eq. (POD)/(SVD): thin SVD U = W S V^T (LAPACK gesdd); the
    spatial basis is the first n_s left singular vectors.

    Returns (Phi_s N_s x n_s, sigma (all singular values), V n_mu N_t x n_s),
    each pair (w_i, v_i) sign-fixed on w_i.
    """
    W, s, Vt = np.linalg.svd(np.asarray(U, dtype=np.float64), full_matrices=False)
    W = W[:, :n_s].copy()
    V = Vt[:n_s].T.copy()
    for i in range(n_s):
        sg, W[:, i] = sign_fix(W[:, i])
        V[:, i] *= sg
    return W, s, V


def temporal_snapshot(V, i, N_t, n_mu):
    """Sec. 4.1: Y_i = [v_i^1 ... v_i^nmu], v_i^p = V((p-1)N_t+1 : p N_t, i)
    (one column per training parameter, N_t x n_mu)."""
    return np.stack([V[p * N_t:(p + 1) * N_t, i] for p in range(n_mu)], axis=1)


def dct2_vector(m, N_t):
    """DCT-II vector c_m(k) = cos(pi m (k + 1/2) / N_t), k = 0..N_t-1."""
    k = np.arange(N_t, dtype=np.float64)
    return np.cos(np.pi * m * (k + 0.5) / N_t)


def temporal_basis(Y, n_t, tau_t=1e-7):
    """Sec. 4.1, Eq. (temporalSVD): Y_i = Lam S Psi^T; Phi_t^i = Lam(:, 1:n_t),
    with the numerical-rank cut and the completion rule in the module header.

    Returns (Phi_t^i N_t x n_t, r_i = numerical rank of Y_i, number of data
    vectors kept = min(r_i, n_t)).
    """
    Y = np.asarray(Y, dtype=np.float64)
    N_t = Y.shape[0]
    if n_t > N_t:
        raise ValueError("n_t exceeds N_t")
    Lam, s, _ = np.linalg.svd(Y, full_matrices=False)
    r = int(np.sum(s > tau_t * s[0])) if s.size and s[0] > 0 else 0
    keep = min(r, n_t)
    cols = [sign_fix(Lam[:, j])[1] for j in range(keep)]
    m = 0
    while len(cols) < n_t:
        if m >= N_t:
            raise RuntimeError("temporal completion ran out of DCT vectors")
        c = dct2_vector(m, N_t)
        v = c.copy()
        if cols:
            B = np.stack(cols, axis=1)
            v = v - B @ (B.T @ v)
            v = v - B @ (B.T @ v)
        nv = np.linalg.norm(v)
        if nv >= COMPLETION_KEEP * np.linalg.norm(c):
            cols.append(sign_fix(v / nv)[1])
        m += 1
    return np.stack(cols, axis=1), r, keep


def temporal_bases(V, N_t, n_mu, n_t, tau_t=1e-7):
    """Temporal bases of every spatial mode (list of N_t x n_t,i arrays)."""
    out, ranks = [], []
    for i in range(V.shape[1]):
        B, r, _ = temporal_basis(temporal_snapshot(V, i, N_t, n_mu), int(n_t[i]), tau_t)
        out.append(B)
        ranks.append(r)
    return out, np.array(ranks)
