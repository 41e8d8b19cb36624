"""Full-order model (oracle, test infrastructure only).

Sec. 2: du/dt = A u + B f, backward Euler, and its space-time form.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def backward_euler(A, F, u0, dt):
    """Sec. 2, Eq. (fom): (I - dt_k A) u^(k) = u^(k-1) + dt_k B f^(k).

    A   : N x N (sparse or dense) state matrix A(mu)
    F   : N x N_t, column k holds B f^(k)
    u0  : N initial state u^(0)
    dt  : N_t step sizes
    Returns the trajectory [u^(1) ... u^(N_t)] as an N x N_t array (u^(0) is
    not included).  Direct sparse LU per step size (SuperLU).
    """
    A = sp.csc_matrix(A)
    N = A.shape[0]
    dt = np.asarray(dt, dtype=np.float64)
    I = sp.identity(N, format="csc")
    facs = {}
    u = np.array(u0, dtype=np.float64)
    out = np.zeros((N, dt.size))
    for k in range(dt.size):
        h = float(dt[k])
        if h not in facs:
            facs[h] = spla.splu(sp.csc_matrix(I - h * A))
        u = facs[h].solve(u + h * F[:, k])
        out[:, k] = u
    return out


def space_time_system(A, F, u0, dt):
    """Sec. 2, Eq. (stsystemmat) and (ststate): the explicit space-time system.

    A_st is lower block-bidiagonal with diagonal blocks (I - dt_k A) and
    sub-diagonal blocks -I; f_st stacks dt_k B f^(k); u0_st = [u0; 0; ...; 0].
    Time-major stacking: entry (k, s) sits at row k*N + s.  Only for small
    sizes (the matrix has N N_t rows).
    """
    A = sp.csr_matrix(A)
    N = A.shape[0]
    Nt = len(dt)
    I = sp.identity(N, format="csr")
    blocks = [[None] * Nt for _ in range(Nt)]
    for k in range(Nt):
        blocks[k][k] = I - dt[k] * A
        if k > 0:
            blocks[k][k - 1] = -I
    A_st = sp.bmat(blocks, format="csr")
    f_st = np.concatenate([dt[k] * F[:, k] for k in range(Nt)])
    u0_st = np.zeros(N * Nt)
    u0_st[:N] = u0
    return A_st, f_st, u0_st
