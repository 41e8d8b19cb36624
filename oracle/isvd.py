"""Incremental SVD of a snapshot stream (oracle, test infrastructure only).

Sec. 4.2, Alg. 1 (initialisation) and Alg. 2 (rank-one update, after Brand).
The thin SVD  U_k = W_k diag(s_k) V_k^T  of the first k snapshots is updated
for a new snapshot u through the factorisation Eq. (factorization2) with the
middle matrix Eq. (middleMat)
    Q = [[diag(s), l], [0, p]],   l = W^T u,   p = ||u - W l||,
whose SVD Q = Uq Sq Vq^T (Eq. (svdMiddleMat)) gives, by Eq. (rankOneUpdateSVD2),
    W <- [W, j] Uq,   s <- diag(Sq),   V <- [[V, 0], [0, 1]] Vq,
with j = (u - W l) / p.  A snapshot with p < eps_svd is numerically dependent
on W: p is set to 0 and only the leading r components are kept.  A trailing
singular value below eps_sv is dropped.  The spatial basis is the first n_s
columns of W after all snapshots (Eq. (spatialincrementalbasis)); the temporal
snapshot matrices are cut from the columns of V as in the batch POD
(Eq. (incrementaltemporalsnapshotmat), (temporalincrementalbasis)).

Readings of the printed algorithm (the device code follows the same ones):
  * p is the norm of the residual u - W l rather than sqrt(u^T u - l^T l),
    which cancels and can go negative; j is formed only when p >= eps_svd.
    The residual is orthogonalised twice against W (classical Gram-Schmidt
    with one re-orthogonalisation); l collects both passes.
  * The update uses the previous factors W_{k-1}, s_{k-1}, V_{k-1}.
  * V keeps one row per snapshot: a snapshot skipped by the initialisation
    (norm <= eps_svd while the basis is empty) leaves a zero row, so V always
    has k rows and U is reproduced column by column.
  * When the rank would exceed r_max, the update is made and the trailing
    triplet dropped (rather than restarting, which would discard the basis).
  * The orthogonality test compares |W(:,1)^T W(:,end)| with
    min(eps_svd, eps N_s), eps the machine epsilon.  When it fails, W is
    replaced by the Q factor of its QR factorisation, taken with a positive
    diagonal of R so that Q stays next to W; R is dropped, as the algorithm
    does (W is orthonormal up to that test's tolerance, so R = I to it).
"""
import numpy as np

from .pod import sign_fix, temporal_bases


def initialize(u, eps_svd):
    """Alg. 1: the first snapshot, if its norm exceeds eps_svd.  Returns
    (W N x r, s (r,), V 1 x r) with r = 1 or 0."""
    nu = float(np.linalg.norm(u))
    if nu > eps_svd:
        return (u / nu)[:, None], np.array([nu]), np.ones((1, 1))
    return np.zeros((len(u), 0)), np.zeros(0), np.zeros((1, 0))


def orthonormal_q(W):
    """Q factor of W = QR with diag(R) > 0."""
    Qw, Rw = np.linalg.qr(W)
    sg = np.where(np.diag(Rw) < 0, -1.0, 1.0)
    return Qw * sg


def update(W, s, V, u, eps_svd, eps_sv, r_max):
    """Alg. 2 for one snapshot u given the factors of the previous ones (V has
    one row per previous snapshot).  Returns the updated (W, s, V, event) with
    event one of 'init', 'skip', 'dependent', 'update', the last two with
    '+qr' appended when the orthogonality test re-orthonormalised W."""
    r = W.shape[1]
    k = V.shape[0]
    if r == 0:
        W1, s1, V1 = initialize(u, eps_svd)
        # the earlier snapshots were all skipped: zero rows for them
        return W1, s1, np.vstack([np.zeros((k, V1.shape[1])), V1]), ("init" if len(s1) else "skip")
    l = W.T @ u
    res = u - W @ l
    l2 = W.T @ res
    res = res - W @ l2
    l = l + l2
    p = float(np.linalg.norm(res))
    dependent = p < eps_svd
    Q = np.zeros((r + 1, r + 1))
    Q[:r, :r] = np.diag(s)
    Q[:r, r] = l
    Q[r, r] = 0.0 if dependent else p
    Vext = np.zeros((k + 1, r + 1))
    Vext[:k, :r] = V
    Vext[k, r] = 1.0
    if dependent:
        # Q has a zero last row: its left singular vectors of nonzero singular
        # value lie in the first r coordinates, so the leading r components are
        # the SVD of the r x (r+1) block (taken directly, which keeps the r x r
        # factor orthogonal when some singular values are tiny)
        Uq, sq, Vqt = np.linalg.svd(Q[:r, :], full_matrices=False)
        W = W @ Uq
        s = sq
        V = Vext @ Vqt.T
    else:
        Uq, sq, Vqt = np.linalg.svd(Q)
        W = np.concatenate([W, (res / p)[:, None]], axis=1) @ Uq
        s = sq
        V = Vext @ Vqt.T
    if len(s) > 0 and s[-1] < eps_sv:
        W, s, V = W[:, :-1], s[:-1], V[:, :-1]
    if len(s) > r_max:
        W, s, V = W[:, :r_max], s[:r_max], V[:, :r_max]
    ev = "dependent" if dependent else "update"
    if W.shape[1] > 1 and abs(float(W[:, 0] @ W[:, -1])) > min(eps_svd, np.finfo(float).eps * W.shape[0]):
        W = orthonormal_q(W)
        ev += "+qr"
    return W, s, V, ev


def incremental_svd(U, eps_svd=1e-12, eps_sv=1e-12, r_max=None, events=None):
    """Streams the columns of U (N_s x m) through Alg. 1-2 (the first column
    through Alg. 1).  Returns (W, s, V) with V of m rows; appends each
    column's event to `events` when a list is given."""
    N, m = U.shape
    r_max = m if r_max is None else r_max
    W, s, V = np.zeros((N, 0)), np.zeros(0), np.zeros((0, 0))
    for c in range(m):
        W, s, V, ev = update(W, s, V, U[:, c], eps_svd, eps_sv, r_max)
        if events is not None:
            events.append(ev)
    return W, s, V


def bases(W, s, V, N_t, n_mu, n_s, n_t, tau_t=1e-7):
    """Eq. (spatialincrementalbasis), (incrementaltemporalsnapshotmat),
    (temporalincrementalbasis): Phi_s = W(:, 1:n_s) and the temporal bases of
    the columns of V, with the batch POD's sign and completion rules.  Columns
    beyond the rank are zero.  Returns (Phi_s, sigma (n_s,), Phi_t list, ranks)."""
    r = W.shape[1]
    Phi = np.zeros((W.shape[0], n_s))
    Vs = np.zeros((V.shape[0], n_s))
    sig = np.zeros(n_s)
    for i in range(min(r, n_s)):
        sg, Phi[:, i] = sign_fix(W[:, i])
        Vs[:, i] = sg * V[:, i]
        sig[i] = s[i]
    Pt, ranks = temporal_bases(Vs, N_t, n_mu, n_t, tau_t)
    return Phi, sig, Pt, ranks
