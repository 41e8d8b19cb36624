"""Precision at scale: the 3-D periodic advection-diffusion problem on 128^3
cells (N_s = 2,097,152), 16 training parameters x 500 backward-Euler steps,
i.e. 8000 snapshots kept on the device in FP32 (67 GB), a snapshot Gram of
8000 x 8000, n_s = 100 spatial modes with 30 temporal vectors each (reduced
width n = 3000).

What is checked, at that size (the oracle cannot run it whole):
  * the GPU snapshot generator against the oracle's full-order march on 32^3;
  * sampled Gram entries in each arithmetic (FP64, FP32, split-BF16) against
    the exactly rounded sum of the FP32 products (math.fsum), within each
    arithmetic's worst-case rounding bound;
  * the POD in each arithmetic: FP64 singular values against the eigenvalues
    of the FP64 Gram (LAPACK on the host), and the reduced-precision Grams,
    whose eigenvectors only seed the FP64 refinement through U, giving the same
    singular values and modes as the FP64 Gram;
  * the 3000-wide reduced systems of a few queries, assembled and solved on
    the device (FP64 LU, and FP32 LU with FP64 refinement), against the
    oracle's block formulas and LAPACK on the host, with the spatial operators
    projected on the host from the device's basis.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import torch

from oracle import fom, rom as orom
from paper_1910_01260_amd import strom
from paper_1910_01260_amd import workloads as W
from tests._gpu import colmajor

pytestmark = pytest.mark.gpu

N3, NT, NMU, NS, NTM = 128, 500, 16, 100, 30
EPS32 = 2.0 ** -24


@pytest.fixture(scope="module")
def c4():
    prob = W.advdiff3d(n=N3, N_t=NT, n_train=NMU)
    U = W.periodic_snapshots_device(prob, N3)  # FP32, column-major, on the device
    torch.cuda.synchronize()
    data = {"prob": prob, "U": U}
    yield data
    data.clear()
    del U
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_generator_matches_oracle_fom():
    prob = W.advdiff3d(n=32, N_t=12, n_train=2)
    U = W.periodic_snapshots_device(prob, 32, dtype=torch.float64).cpu().numpy()
    ref = np.concatenate([fom.backward_euler(prob.operator(m), np.zeros((prob.N_s, prob.N_t)), prob.initial(m),
                                             prob.dt) for m in prob.train_mu], axis=1)
    assert np.abs(U - ref).max() <= 1e-12 * np.abs(ref).max()


def test_gram_sampled_entries_all_precisions(c4):
    U = c4["U"]
    K, m = U.shape
    assert (K, m) == (N3 ** 3, NT * NMU)
    rng = np.random.default_rng(11)
    pairs = [(i, i) for i in rng.choice(m, 12, replace=False)]
    pairs += [(i, i + 1) for i in rng.choice(m - 1, 12, replace=False)]
    pairs += [tuple(rng.choice(m, 2, replace=False)) for _ in range(16)]
    cols = sorted({c for p in pairs for c in p})
    host = {c: U[:, c].cpu().numpy().astype(np.float64) for c in cols}
    exact = {(i, j): math.fsum(host[i] * host[j]) for i, j in pairs}  # FP32 x FP32 products are exact in FP64
    absum = {(i, j): float(np.sum(np.abs(host[i] * host[j]))) for i, j in pairs}
    # worst-case rounding bounds relative to sum |u_i u_j| (K terms in FP64; FP32 over 1024-term
    # stretches; split-BF16 adds the dropped lo*lo term and the second split, 3 * 2^-18)
    bound = {strom.ST_F64: K * 2.0 ** -53 * 1.01, strom.ST_F32: 1026 * EPS32,
             strom.ST_BF16X3: 1026 * EPS32 + 3 * 2.0 ** -18}
    worst = {}
    for prec in (strom.ST_F64, strom.ST_F32, strom.ST_BF16X3):
        G = strom.st_gram(U, prec)
        torch.cuda.synchronize()
        got = {(i, j): float(G[i, j]) for i, j in pairs}
        assert all(float(G[i, j]) == float(G[j, i]) for i, j in pairs)
        r = max(abs(got[p] - exact[p]) / absum[p] for p in pairs)
        worst[prec] = r
        assert r <= bound[prec], (prec, r, bound[prec])
        del G
    print("Gram sampled errors / sum|u_i u_j|:", {k: f"{v:.2e}" for k, v in worst.items()})


def test_pod_precisions_and_gram_eigenvalues(c4):
    U = c4["U"]
    G64 = strom.st_gram(U, strom.ST_F64)
    gmax = float(G64.abs().max())
    delta = {}
    for prec in (strom.ST_F32, strom.ST_BF16X3):
        Gp = strom.st_gram(U, prec)
        delta[prec] = float((Gp - G64).abs().max()) / gmax
        del Gp
    G = G64.cpu().numpy()
    del G64
    m = G.shape[0]
    lam = sla.eigh(G, subset_by_index=[m - NS, m - 1], eigvals_only=True, driver="evr")[::-1]
    del G
    res = {}
    for prec in (strom.ST_F64, strom.ST_F32, strom.ST_BF16X3):
        Phi_s, Phi_t, sig, rank = strom.st_build_bases(U, NT, NMU, NS, [NTM] * NS, gram_prec=prec)
        torch.cuda.synchronize()
        res[prec] = (Phi_s, Phi_t, sig.cpu().numpy())
    Phi64, Phit64, s64 = res[strom.ST_F64]
    s1 = s64[0]
    # FP64 singular values against the square roots of the FP64 Gram's eigenvalues (LAPACK on the
    # host); those carry the Gram's rounding, ~1e-12 ||G|| on this size, i.e. ~1e-12 sigma_1^2/sigma_i
    ref = np.sqrt(np.maximum(lam, 0.0))
    tol = 1e-12 * s1 + 2e-12 * s1 ** 2 / np.maximum(s64, 1e-300)
    assert np.all(np.abs(s64 - ref) <= tol), np.max(np.abs(s64 - ref) / tol)
    assert np.abs((Phi64.T @ Phi64).cpu().numpy() - np.eye(NS)).max() <= 1e-12
    # A reduced-precision Gram only seeds the FP64 refinement through U.  Modes whose eigenvalue
    # the Gram's perturbation moves by at most a tenth (delta sigma_1^2 <= 0.1 sigma_i^2, delta
    # the Gram's largest entry error relative to its largest entry) come out as with the FP64
    # Gram, to rounding; the rest are printed.
    for prec in (strom.ST_F32, strom.ST_BF16X3):
        Phi, _, s = res[prec]
        dsig = np.abs(s - s64) / s1
        cosv = torch.abs(torch.sum(Phi * Phi64, dim=0)).cpu().numpy()
        seeded = delta[prec] * s1 ** 2 <= 0.1 * s64 ** 2
        assert seeded[:10].all(), (prec, delta[prec])
        assert np.all(dsig[seeded] <= 1e-13), (prec, dsig[seeded].max())
        assert np.all(1.0 - cosv[seeded] <= 1e-12), (prec, (1.0 - cosv[seeded]).max())
        print(f"gram_prec {prec}: Gram error {delta[prec]:.1e} of max|G|; {seeded.sum()} modes seeded: "
              f"|dsigma| <= {dsig[seeded].max():.1e} sigma_1, 1-|cos| <= {(1.0 - cosv[seeded]).max():.1e}; "
              f"all {NS}: |dsigma| <= {dsig.max():.1e} sigma_1")
    c4["bases"] = (Phi64, Phit64)


def test_rom_width_3000_matches_oracle(c4):
    prob = c4["prob"]
    U = c4["U"]
    if "bases" in c4:
        Phi_s, Phi_t = c4["bases"]
    else:
        Phi_s, Phi_t, _, _ = strom.st_build_bases(U, NT, NMU, NS, [NTM] * NS)
    desc = strom.RomDesc([NTM] * NS, NT, prob.Q, prob.Qf, prob.Q0)
    csr = [strom.csr_to_device(*W.csr_arrays(A)) for A in prob.terms]
    dt = torch.tensor(prob.dt, device="cuda")
    u0 = colmajor(prob.u0)
    romb = strom.st_assemble(desc, Phi_s, Phi_t, dt, [c[0] for c in csr], None, None, u0)
    mus = W.sample_params(prob, 4)
    tA, tf, t0 = prob.thetas(mus)
    nt = np.full((len(mus), NS), NTM, dtype=np.int32)
    args = (torch.tensor(tA, device="cuda"), None, torch.tensor(t0, device="cuda"), torch.tensor(nt, device="cuda"))
    out64 = strom.st_solve(desc, romb, *args, lu_prec=strom.ST_F64)
    out32 = strom.st_solve(desc, romb, *args, lu_prec=strom.ST_F32, ir_tol=1e-12, ir_max=8)
    torch.cuda.synchronize()
    # the oracle's reduced systems from the device basis
    P = Phi_s.cpu().numpy()
    Pt_all = Phi_t.cpu().numpy()
    Pt = [Pt_all[:, i * NTM:(i + 1) * NTM] for i in range(NS)]
    Ahat = [orom.spatial_operator(P, A) for A in prob.terms]
    u0hat = orom.reduced_vector(P, prob.u0)
    del P
    off = out64.coeff_off.cpu().numpy()
    c64 = out64.coeff.cpu().numpy()
    c32 = out32.coeff.cpu().numpy()
    assert (out64.info.cpu().numpy()[:len(mus)] == 0).all()
    assert np.isin(out32.info.cpu().numpy()[:len(mus)], (0, -6)).all()
    for q in range(len(mus)):
        M, b = orom.reduced_system(Ahat, tA[q], np.zeros((NS, 0)), tf[q], prob.g, u0hat, t0[q], Pt, prob.dt)
        assert M.shape == (NS * NTM, NS * NTM)
        c = np.linalg.solve(M, b)
        e64 = np.linalg.norm(c64[off[q]:off[q + 1]] - c) / np.linalg.norm(c)
        e32 = np.linalg.norm(c32[off[q]:off[q + 1]] - c) / np.linalg.norm(c)
        assert e64 <= 1e-10 and e32 <= 1e-10, (q, e64, e32)
