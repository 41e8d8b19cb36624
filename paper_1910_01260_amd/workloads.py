"""Seeded synthetic workloads for the space-time ROM hot path.

This module only generates inputs.  It builds the sparse model operators as
affine terms A(mu) = sum_q theta_q(mu) A_q, the input vectors B f_q with their
time profiles, the initial states u0_q, the parameter samples, and the
per-query temporal-basis truncation profiles.  It also provides the
full-order backward-Euler march (the paper's full-order model, Sec. 2,
Eq. (fom)) that produces the snapshot matrix.  That march is the user's
simulator: it runs upstream of the reduced-order method, and in the paper it
was an external transport code.  No step of the reduced-order method (POD,
projection, space-time assembly, reduced solve) lives here, and both the HIP
path and the CPU oracle receive these arrays as plain inputs.

Model problems (all synthetic, seeded, shaped like the paper's workloads):

* ``advdiff1d``   1-D periodic advection-diffusion (N_s = 256, N_t = 128).
* ``transport2d`` 2-D discrete-ordinates transport, upwind streaming,
  isotropic scattering, direction-major unknown ordering (N_s = 64*64*12).
  It stands in for the paper's 3-D multigroup Boltzmann problems (Sec. 6-7),
  whose code and data are not public.
* ``transport2d_absorber`` the same with a third parameter: extra
  absorption in a central box.
* ``advdiff3d``   3-D periodic advection-diffusion on a 7-point stencil; its
  snapshots at 128^3 come from ``periodic_snapshots_device`` (the same
  backward-Euler march, solved exactly in Fourier space on the GPU).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

TEST_SEED = 191001260
SURROGATE_SEED = 191001261
PROFILE_SEED = 191001262


@dataclasses.dataclass
class Problem:
    """A parametric linear system du/dt = A(mu) u + B f(t; mu), u(0) = u0(mu).

    A(mu) = sum_q theta_A(mu)[q] * terms[q]
    B f(t_k; mu) = sum_q theta_f(mu)[q] * g[k, q] * Bf[:, q]
    u0(mu) = sum_q theta_0(mu)[q] * u0[:, q]
    """

    name: str
    terms: List[sp.csr_matrix]
    theta_A: Callable[[np.ndarray], np.ndarray]
    Bf: np.ndarray                 # N_s x Qf
    theta_f: Callable[[np.ndarray], np.ndarray]
    g: np.ndarray                  # N_t x Qf time profiles of the inputs
    u0: np.ndarray                 # N_s x Q0
    theta_0: Callable[[np.ndarray], np.ndarray]
    dt: np.ndarray                 # N_t step sizes
    box_lo: np.ndarray             # parameter box
    box_hi: np.ndarray
    train_mu: np.ndarray           # n_mu x d training parameters
    lagged_term: Optional[int] = None  # term iterated explicitly in march()
    sweep_order: Optional[np.ndarray] = None  # unknown order making the rest triangular
    lagged_apply: Optional[Callable[[np.ndarray], np.ndarray]] = None  # x -> terms[lagged_term] @ x

    @property
    def N_s(self) -> int:
        return self.terms[0].shape[0]

    @property
    def N_t(self) -> int:
        return int(self.dt.shape[0])

    @property
    def Q(self) -> int:
        return len(self.terms)

    @property
    def Qf(self) -> int:
        return int(self.Bf.shape[1])

    @property
    def Q0(self) -> int:
        return int(self.u0.shape[1])

    def thetas(self, mus: np.ndarray):
        """Affine coefficients for a batch of parameters (n_q x d)."""
        mus = np.atleast_2d(np.asarray(mus, dtype=np.float64))
        tA = np.array([self.theta_A(m) for m in mus], dtype=np.float64).reshape(len(mus), self.Q)
        tf = np.array([self.theta_f(m) for m in mus], dtype=np.float64).reshape(len(mus), self.Qf)
        t0 = np.array([self.theta_0(m) for m in mus], dtype=np.float64).reshape(len(mus), self.Q0)
        return tA, tf, t0

    def operator(self, mu) -> sp.csr_matrix:
        th = self.theta_A(np.asarray(mu, dtype=np.float64))
        A = th[0] * self.terms[0]
        for q in range(1, self.Q):
            A = A + th[q] * self.terms[q]
        return A.tocsr()

    def forcing(self, mu) -> np.ndarray:
        """N_s x N_t matrix whose column k is B f^(k)(mu) (zero if Qf = 0)."""
        F = np.zeros((self.N_s, self.N_t))
        if self.Qf:
            th = self.theta_f(np.asarray(mu, dtype=np.float64))
            F += (self.Bf * th[None, :]) @ self.g.T
        return F

    def initial(self, mu) -> np.ndarray:
        x = np.zeros(self.N_s)
        if self.Q0:
            x += self.u0 @ self.theta_0(np.asarray(mu, dtype=np.float64))
        return x


def csr_arrays(A: sp.csr_matrix):
    """(row_ptr int32, col_idx int32, val float64) of a square CSR matrix."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    return (np.ascontiguousarray(A.indptr, dtype=np.int32),
            np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


# ----------------------------------------------------------------------------
# 1-D periodic advection-diffusion
# ----------------------------------------------------------------------------

def advdiff1d(N: int = 256, N_t: int = 128, n_train: int = 4, c: float = 1.0,
              mu_lo: float = 0.005, mu_hi: float = 0.02,
              center: float = 0.3, width: float = 0.05) -> Problem:
    """u_t = -c u_x + mu u_xx on [0,1) periodic, first-order upwind advection.

    theta_A(mu) = (1, mu), A_1 = -c D_up, A_2 = L (periodic 3-point Laplacian).
    u0 = exp(-((x - center)/width)^2), no input (Qf = 0), dt = 1/N_t.
    Training parameters are an even grid of n_train values in [mu_lo, mu_hi].
    """
    h = 1.0 / N
    i = np.arange(N)
    im = (i - 1) % N
    ip = (i + 1) % N
    Dup = sp.csr_matrix((np.r_[np.full(N, 1.0 / h), np.full(N, -1.0 / h)],
                         (np.r_[i, i], np.r_[i, im])), shape=(N, N))
    L = sp.csr_matrix((np.r_[np.full(N, -2.0 / h ** 2), np.full(N, 1.0 / h ** 2), np.full(N, 1.0 / h ** 2)],
                       (np.r_[i, i, i], np.r_[i, im, ip])), shape=(N, N))
    x = i * h
    u0 = np.exp(-((x - center) / width) ** 2)[:, None]
    return Problem(
        name="advdiff1d",
        terms=[(-c * Dup).tocsr(), L.tocsr()],
        theta_A=lambda m: np.array([1.0, float(np.ravel(m)[0])]),
        Bf=np.zeros((N, 0)),
        theta_f=lambda m: np.zeros(0),
        g=np.zeros((N_t, 0)),
        u0=u0,
        theta_0=lambda m: np.array([1.0]),
        dt=np.full(N_t, 1.0 / N_t),
        box_lo=np.array([mu_lo]), box_hi=np.array([mu_hi]),
        train_mu=np.linspace(mu_lo, mu_hi, n_train)[:, None],
    )


# ----------------------------------------------------------------------------
# 2-D discrete-ordinates transport (one group, isotropic scattering)
# ----------------------------------------------------------------------------

def _transport_parts(nx: int, ndir: int):
    h = 1.0 / nx
    ncell = nx * nx
    ang = (np.arange(ndir) + 0.5) * (2.0 * np.pi / ndir)
    ox, oy = np.cos(ang), np.sin(ang)
    w = np.full(ndir, 1.0 / ndir)
    ix, iy = np.meshgrid(np.arange(nx), np.arange(nx), indexing="xy")
    ix = ix.ravel()
    iy = iy.ravel()
    cell = ix + nx * iy                      # x fastest
    rows, cols, vals = [], [], []
    for l in range(ndir):
        base = l * ncell
        ax, ay = abs(ox[l]) / h, abs(oy[l]) / h
        rows.append(base + cell); cols.append(base + cell); vals.append(np.full(ncell, ax + ay))
        sx = 1 if ox[l] > 0 else -1            # upwind neighbour is ix - sx
        ux = ix - sx
        ok = (ux >= 0) & (ux < nx)             # vacuum inflow outside the box
        rows.append(base + cell[ok]); cols.append(base + ux[ok] + nx * iy[ok]); vals.append(np.full(ok.sum(), -ax))
        sy = 1 if oy[l] > 0 else -1
        uy = iy - sy
        ok = (uy >= 0) & (uy < nx)
        rows.append(base + cell[ok]); cols.append(base + ix[ok] + nx * uy[ok]); vals.append(np.full(ok.sum(), -ay))
    N = ncell * ndir
    C = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    # isotropic scattering: (P psi)_l = sum_l' w_l' psi_l'  (same cell)
    r, c_, v = [], [], []
    for l in range(ndir):
        for lp in range(ndir):
            r.append(l * ncell + np.arange(ncell)); c_.append(lp * ncell + np.arange(ncell))
            v.append(np.full(ncell, w[lp]))
    P = sp.csr_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c_))), shape=(N, N))
    xc = (ix + 0.5) * h
    yc = (iy + 0.5) * h
    # sweep order: per direction, cells from the inflow corner downstream, so
    # the streaming operator is lower triangular in this order
    order = []
    for l in range(ndir):
        xs = np.arange(nx) if ox[l] > 0 else np.arange(nx)[::-1]
        ys = np.arange(nx) if oy[l] > 0 else np.arange(nx)[::-1]
        gx, gy = np.meshgrid(xs, ys, indexing="xy")
        order.append(l * ncell + (gx + nx * gy).ravel())
    return N, ncell, C, P, xc, yc, np.concatenate(order)


def transport2d(nx: int = 64, ndir: int = 12, N_t: int = 200, T: float = 1.0) -> Problem:
    """psi_t = -Omega.grad psi - sigma_t psi + sigma_t c sum_l w_l psi_l + q.

    mu = (sigma_t in [1,5], c in [0.5,0.95]); theta_A = (1, -sigma_t, sigma_t c)
    with A_1 = -C (upwind streaming, vacuum inflow), A_2 = I, A_3 = P_iso.
    Isotropic unit source on the central box [0.375, 0.625]^2, constant in
    time; zero initial state (Q0 = 0).  Training: sigma_t on a 4-point grid
    times c in {0.5, 0.95}.
    """
    N, ncell, C, P, xc, yc, order = _transport_parts(nx, ndir)
    src = ((xc > 0.375) & (xc < 0.625) & (yc > 0.375) & (yc < 0.625)).astype(np.float64)
    Bf = np.tile(src, ndir)[:, None]
    st = np.linspace(1.0, 5.0, 4)
    cc = np.array([0.5, 0.95])
    train = np.array([[a, b] for a in st for b in cc])
    return Problem(
        name="transport2d",
        terms=[(-C).tocsr(), sp.identity(N, format="csr"), P.tocsr()],
        theta_A=lambda m: np.array([1.0, -m[0], m[0] * m[1]]),
        Bf=Bf,
        theta_f=lambda m: np.array([1.0]),
        g=np.ones((N_t, 1)),
        u0=np.zeros((N, 0)),
        theta_0=lambda m: np.zeros(0),
        dt=np.full(N_t, T / N_t),
        box_lo=np.array([1.0, 0.5]), box_hi=np.array([5.0, 0.95]),
        train_mu=train,
        lagged_term=2,
        sweep_order=order,
        lagged_apply=lambda x: np.tile((x.reshape(ndir, -1) * (1.0 / ndir)).sum(axis=0), ndir),
    )


def transport2d_absorber(nx: int = 64, ndir: int = 12, N_t: int = 200, T: float = 1.0) -> Problem:
    """transport2d with a third parameter sigma_abs in [1, 10]: extra absorption
    on the central box [0.4, 0.6]^2 (theta_4 = sigma_abs, A_4 = -chi_box).
    Training: 3 x 2 x 2 grid over (sigma_t, c, sigma_abs)."""
    base = transport2d(nx, ndir, N_t, T)
    N, ncell, C, P, xc, yc, _ = _transport_parts(nx, ndir)
    box = ((xc > 0.4) & (xc < 0.6) & (yc > 0.4) & (yc < 0.6)).astype(np.float64)
    A4 = sp.diags(-np.tile(box, ndir), format="csr")
    train = np.array([[a, b, s] for a in (1.0, 3.0, 5.0) for b in (0.5, 0.95) for s in (1.0, 10.0)])
    base.name = "transport2d_absorber"
    base.terms = base.terms + [A4]
    base.theta_A = lambda m: np.array([1.0, -m[0], m[0] * m[1], m[2]])
    base.box_lo = np.array([1.0, 0.5, 1.0])
    base.box_hi = np.array([5.0, 0.95, 10.0])
    base.train_mu = train
    return base


# ----------------------------------------------------------------------------
# 3-D periodic advection-diffusion (7-point stencil)
# ----------------------------------------------------------------------------

def advdiff3d(n: int = 128, N_t: int = 500, n_train: int = 16,
              mu_lo: float = 0.005, mu_hi: float = 0.02, width: float = 0.05) -> Problem:
    """u_t = -c.grad u + mu Lap u on [0,1)^3 periodic, c = (1,1,1)/sqrt(3),
    first-order upwind advection, 7-point Laplacian; theta_A = (1, mu)."""
    h = 1.0 / n
    N = n ** 3
    idx = np.arange(N)
    x = idx % n
    y = (idx // n) % n
    z = idx // (n * n)

    def nb(dx, dy, dz):
        return ((x + dx) % n) + n * (((y + dy) % n) + n * ((z + dz) % n))

    cv = 1.0 / np.sqrt(3.0)
    rows = np.concatenate([idx] * 4)
    cols = np.concatenate([idx, nb(-1, 0, 0), nb(0, -1, 0), nb(0, 0, -1)])
    vals = np.concatenate([np.full(N, -3 * cv / h)] + [np.full(N, cv / h)] * 3)
    Adv = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    rows = np.concatenate([idx] * 7)
    cols = np.concatenate([idx, nb(-1, 0, 0), nb(1, 0, 0), nb(0, -1, 0), nb(0, 1, 0), nb(0, 0, -1), nb(0, 0, 1)])
    vals = np.concatenate([np.full(N, -6.0 / h ** 2)] + [np.full(N, 1.0 / h ** 2)] * 6)
    Lap = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    xc, yc, zc = x * h, y * h, z * h
    u0 = np.exp(-(((xc - 0.3) ** 2 + (yc - 0.3) ** 2 + (zc - 0.3) ** 2) / width ** 2))[:, None]
    return Problem(
        name="advdiff3d",
        terms=[Adv.tocsr(), Lap.tocsr()],
        theta_A=lambda m: np.array([1.0, float(np.ravel(m)[0])]),
        Bf=np.zeros((N, 0)),
        theta_f=lambda m: np.zeros(0),
        g=np.zeros((N_t, 0)),
        u0=u0,
        theta_0=lambda m: np.array([1.0]),
        dt=np.full(N_t, 1.0 / N_t),
        box_lo=np.array([mu_lo]), box_hi=np.array([mu_hi]),
        train_mu=np.linspace(mu_lo, mu_hi, n_train)[:, None],
    )


def periodic_snapshots_device(prob: Problem, n: int, mus: Optional[Sequence] = None, dtype=None,
                              device: str = "cuda"):
    """Snapshot matrix of a periodic, constant-coefficient stencil problem on an
    n^3 grid (``advdiff3d``), computed on the GPU: N_s x (n_mu N_t), column-major
    (a transposed contiguous tensor), parameter-major, time inside, u^(0) excluded.

    Each backward-Euler step (I - dt_k A(mu)) u^(k) = u^(k-1) is solved exactly
    in Fourier space: a translation-invariant operator is diagonal in the
    discrete Fourier basis, with symbol lambda(k) = sum_j A[0, j]
    exp(2 pi i k . x_j / n) read off the first CSR row of each affine term, so
    u^(k) = IFFT(FFT(u^(k-1)) / (1 - dt_k lambda_mu)).  The march runs in FP64
    (torch.fft) and the snapshots are stored in ``dtype`` (float32 by default).
    This is the user's full-order simulator, as ``march`` is; it needs the
    operators to be periodic stencils (it is checked against ``march``)."""
    import torch

    dtype = torch.float32 if dtype is None else dtype
    mus = prob.train_mu if mus is None else np.atleast_2d(mus)
    N = n ** 3
    assert prob.N_s == N and prob.Qf == 0
    kk = torch.arange(n, device=device, dtype=torch.float64)
    kz, ky, kx = torch.meshgrid(kk, kk, kk, indexing="ij")
    symbols = []
    for A in prob.terms:
        A = sp.csr_matrix(A)
        lam = torch.zeros((n, n, n), dtype=torch.complex128, device=device)
        for j, a in zip(A.indices[A.indptr[0]:A.indptr[1]], A.data[A.indptr[0]:A.indptr[1]]):
            dx, dy, dz = j % n, (j // n) % n, j // (n * n)
            lam += float(a) * torch.exp(1j * (2.0 * np.pi / n) * (kx * dx + ky * dy + kz * dz))
        symbols.append(lam)
    U = torch.empty((len(mus) * prob.N_t, N), dtype=dtype, device=device)
    for p, mu in enumerate(mus):
        th = prob.theta_A(np.asarray(mu, dtype=np.float64))
        lam = sum(float(th[q]) * symbols[q] for q in range(prob.Q))
        u_hat = torch.fft.fftn(torch.tensor(prob.initial(mu).reshape(n, n, n), device=device))
        for k in range(prob.N_t):
            u_hat = u_hat / (1.0 - float(prob.dt[k]) * lam)
            U[p * prob.N_t + k] = torch.fft.ifftn(u_hat).real.reshape(N).to(dtype)
    return U.T


# ----------------------------------------------------------------------------
# parameters, profiles, snapshots
# ----------------------------------------------------------------------------

def sample_params(prob: Problem, n: int, seed: int = TEST_SEED) -> np.ndarray:
    """n parameters drawn uniformly (seeded) in the problem's box."""
    rng = np.random.default_rng(seed)
    return rng.uniform(prob.box_lo, prob.box_hi, size=(n, prob.box_lo.shape[0]))


def ragged_profiles(n_q: int, n_s: int, seed: int = PROFILE_SEED,
                    lo: int = 10, hi: int = 30, nt_min: int = 8, nt_max: int = 32) -> np.ndarray:
    """Per-query, per-mode temporal basis counts (n_q x n_s int32).

    Query q draws a level L_q uniformly in {lo..hi}; mode i keeps
    clamp(L_q + delta_i, nt_min, nt_max) temporal vectors with delta_i = +2
    for the first quarter of the modes, 0 for the middle half and -2 for the
    last quarter.  With n_s = 40 the widths sum_i n_t,i span 400..1200.
    """
    rng = np.random.default_rng(seed)
    L = rng.integers(lo, hi + 1, size=n_q)
    delta = np.zeros(n_s, dtype=np.int64)
    delta[: n_s // 4] = 2
    delta[n_s - n_s // 4:] = -2
    nt = np.clip(L[:, None] + delta[None, :], nt_min, nt_max)
    return np.ascontiguousarray(nt, dtype=np.int32)


def march(prob: Problem, mu, tol: float = 1e-14, max_iter: int = 200) -> np.ndarray:
    """Full-order backward-Euler trajectory [u^(1) ... u^(N_t)] (N_s x N_t).

    (I - dt_k A(mu)) u^(k) = u^(k-1) + dt_k B f^(k), u^(0) = u0(mu).  Each step
    is a sparse LU solve (one factorisation per distinct step size).  When the
    problem names a lagged term (the isotropic scattering of the transport
    problems) the step is solved by source iteration instead: the remaining
    operator is block-diagonal over directions and cheap to factor, and the
    iteration contracts by dt*sigma_s/(1 + dt*sigma_t) per sweep; it runs to a
    relative change of ``tol``.
    """
    mu = np.asarray(mu, dtype=np.float64)
    th = prob.theta_A(mu)
    F = prob.forcing(mu)
    u = prob.initial(mu)
    I = sp.identity(prob.N_s, format="csc")
    s = prob.lagged_term
    A_impl = None
    for q in range(prob.Q):
        if q == s:
            continue
        A_impl = th[q] * prob.terms[q] if A_impl is None else A_impl + th[q] * prob.terms[q]
    A_impl = A_impl.tocsc()
    A_lag = None
    if s is not None:
        if prob.lagged_apply is not None:
            A_lag = lambda x, c=th[s], f=prob.lagged_apply: c * f(x)
        else:
            A_lag = lambda x, M=(th[s] * prob.terms[s]).tocsr(): M @ x
    perm = prob.sweep_order if s is not None else None
    lus = {}
    out = np.empty((prob.N_s, prob.N_t))
    for k in range(prob.N_t):
        d = float(prob.dt[k])
        if d not in lus:
            M = (I - d * A_impl).tocsr()
            if perm is None:
                lus[d] = spla.splu(M.tocsc(), permc_spec="MMD_AT_PLUS_A").solve
            else:
                Mp = M[perm][:, perm].tocsc()
                lu = spla.splu(Mp, permc_spec="NATURAL", diag_pivot_thresh=0.0)

                def solve(b, lu=lu):
                    x = np.empty_like(b)
                    x[perm] = lu.solve(b[perm])
                    return x
                lus[d] = solve
        rhs = u + d * F[:, k]
        if A_lag is None:
            u = lus[d](rhs)
        else:
            x = lus[d](rhs + d * A_lag(u))
            for _ in range(max_iter):
                x_new = lus[d](rhs + d * A_lag(x))
                delta = np.linalg.norm(x_new - x)
                x = x_new
                if delta <= tol * np.linalg.norm(x):
                    break
            else:
                raise RuntimeError("source iteration did not converge")
            u = x
        out[:, k] = u
    return out


def snapshots(prob: Problem, mus: Optional[Sequence] = None, threads: int = 8) -> np.ndarray:
    """Snapshot matrix [U_1 ... U_nmu] (N_s x n_mu N_t), parameter-major,
    time inside, u^(0) excluded; Fortran order (column-major).  Trajectories
    run on a thread pool (the sparse solves release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    mus = prob.train_mu if mus is None else np.atleast_2d(mus)
    U = np.empty((prob.N_s, len(mus) * prob.N_t), order="F")

    def run(p):
        U[:, p * prob.N_t:(p + 1) * prob.N_t] = march(prob, mus[p])

    if threads <= 1 or len(mus) == 1:
        for p in range(len(mus)):
            run(p)
    else:
        with ThreadPoolExecutor(max_workers=min(threads, len(mus))) as ex:
            list(ex.map(run, range(len(mus))))
    return U
