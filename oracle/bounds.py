"""A-posteriori error bounds of Sec. 5 (oracle, test infrastructure only)."""
import numpy as np


def residual_fom(A, Bf_k, u_k, u_km1, dt_k):
    """Sec. 5.1, Eq. (residual): r^(k) = u^(k) - u^(k-1) - dt_k A u^(k) - dt_k B f^(k)."""
    return u_k - u_km1 - dt_k * (A @ u_k) - dt_k * Bf_k


def theorem1_bound(A, F, U_approx, u0, dt):
    """Theorem 1 (res-basedErrorBoundforSpace): for each k,
    ||u^(k) - u~^(k)|| <= sum_{i<=k} (prod_{j=i..k} ||(I - dt_j A)^{-1}||_2) ||r^(i)||.
    A dense; F: N x N_t inputs; U_approx: N x N_t; requires u~^(0) = u^(0)."""
    A = np.asarray(A)
    N = A.shape[0]
    Nt = len(dt)
    tau = np.array([1.0 / np.linalg.svd(np.eye(N) - dt[k] * A, compute_uv=False)[-1] for k in range(Nt)])
    res = []
    prev = u0
    for k in range(Nt):
        res.append(np.linalg.norm(residual_fom(A, F[:, k], U_approx[:, k], prev, dt[k])))
        prev = U_approx[:, k]
    res = np.array(res)
    out = np.zeros(Nt)
    for k in range(Nt):
        out[k] = sum(np.prod(tau[i:k + 1]) * res[i] for i in range(k + 1))
    return out


def theorem2_bound(A, F, U_approx, dt):
    """Theorem 2 (specificErrorBoundforSpace): with beta_k = 1/(1 - dt_k ||A||_2),
    ||u^(k) - u~^(k)|| <= sum_{i<=k} (prod_{j=i..k} beta_j) ||dt_i (A u~^(i) + B f^(i))||.
    Valid for u~ from the spatial Galerkin ROM with u~^(0) = u^(0), dt_k ||A|| < 1."""
    A = np.asarray(A)
    nA = np.linalg.norm(A, 2)
    Nt = len(dt)
    beta = 1.0 / (1.0 - dt * nA)
    q = np.array([np.linalg.norm(dt[i] * (A @ U_approx[:, i] + F[:, i])) for i in range(Nt)])
    return np.array([sum(np.prod(beta[i:k + 1]) * q[i] for i in range(k + 1)) for k in range(Nt)])


def st_inf_norm(x, N):
    """Eq. (spacetimeinfnorm): max_k ||u^(k)||_2 over time-major blocks of size N."""
    return float(np.max(np.linalg.norm(np.asarray(x).reshape(-1, N), axis=1)))


def theorem3_bound(A_st, f_st, u0_st, u_st_approx, N):
    """Theorem 3 (res-basedErrorBoundforSpaceTime):
    ||du_st||_inf <= sqrt(N_t) ||A_st^{-1}||_2 ||A_st u~ - f_st - u0_st||_inf."""
    A_st = np.asarray(A_st.todense()) if hasattr(A_st, "todense") else np.asarray(A_st)
    Nt = A_st.shape[0] // N
    inv_norm = 1.0 / np.linalg.svd(A_st, compute_uv=False)[-1]
    r = A_st @ u_st_approx - f_st - u0_st
    return np.sqrt(Nt) * inv_norm * st_inf_norm(r, N)


def coercivity_floor(N_t):
    """Lower bound of lambda_min(sym Ahat_st) when sym(A) <= 0.

    The backward-Euler space-time matrix of Sec. 2 has blocks I - dt_k A on
    the diagonal and -I below it.  With sym(A) <= 0 its symmetric part
    dominates the tridiagonal Toeplitz matrix (1 on the diagonal, -1/2 beside
    it) Kronecker I, whose smallest eigenvalue is 1 - cos(pi / (N_t + 1)); the
    Galerkin projection with orthonormal Phi_st (Sec. 3.2) keeps the bound."""
    return 1.0 - np.cos(np.pi / (N_t + 1))


def certificate(M, rhs, c, gamma):
    """Relative error certificate of an approximate reduced solution c.

    Coercivity gives ||c - c*|| <= ||rhs - M c|| / gamma =: delta, and so
    ||c - c*|| / ||c*|| <= e / (1 - e) with e = delta / ||c|| (infinite when
    e >= 1 or c = 0).  The residual is that of the reduced system Eq. (st-galerkin)."""
    r = rhs - M @ c
    cn = np.linalg.norm(c)
    if cn == 0.0:
        return np.inf
    e = np.linalg.norm(r) / (gamma * cn)
    return e / (1.0 - e) if e < 1.0 else np.inf
