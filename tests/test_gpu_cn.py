"""Crank-Nicolson space-time ROM on the device (the other block structure the
paper mentions for other time integrators, Sec. 2) against the oracle's
Crank-Nicolson block formulas (oracle/cn.py), through the C ABI: the shifted
temporal contraction, per-query assembly, the batched FP64 and FP32 + FP64
refinement solves (matrix-free and gather residuals) and the certificate."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import cn, rom as orom  # noqa: E402
from paper_1910_01260_amd import strom  # noqa: E402
from paper_1910_01260_amd import workloads as W  # noqa: E402

from . import _cases as C  # noqa: E402
from ._gpu import DeviceRom, thetas_device  # noqa: E402

RTOL = 1e-10


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.fixture(scope="module", params=["cb", "c2_small"])
def cn_rom(request):
    name = request.param
    prob = C.problem(name)
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases(name)
    print(f"[{name}] building Crank-Nicolson device ROM", flush=True)
    dr = DeviceRom(prob, Phi_s, Phi_t, integrator=strom.ST_CRANK_NICOLSON)
    Ahat, bhat, u0hat = C.oracle_spatial(name)
    Au0hat = [Phi_s.T @ (A @ prob.u0) if prob.Q0 else np.zeros((Phi_s.shape[1], 0)) for A in prob.terms]
    return name, dr, (Ahat, bhat, u0hat, Au0hat), Phi_t


def _oracle_cn(prob, pieces, Phi_t, tA, tf, t0, nt):
    Ahat, bhat, u0hat, Au0hat = pieces
    Pt = [Phi_t[i][:, :int(nt[i])] for i in range(len(Phi_t))] if nt is not None else Phi_t
    return cn.reduced_system(Ahat, tA, bhat, tf, prob.g, u0hat, Au0hat, t0, Pt, prob.dt)


def _profiles(name, n_q, seed):
    if name == "cb":
        return W.ragged_profiles(n_q, 40, seed=seed)
    rng = np.random.default_rng(seed)
    return rng.integers(1, 13, size=(n_q, 20)).astype(np.int32)


def test_cn_temporal_contraction(cn_rom):
    name, dr, pieces, Phi_t = cn_rom
    prob = dr.prob
    n = dr.desc.n
    P = np.concatenate(Phi_t, axis=1)
    T = P.T @ (prob.dt[:, None] * P)
    S = P[1:].T @ (prob.dt[1:, None] * P[:-1])
    got = dr.section("Tcn").cpu().numpy()[: n * n].reshape(n, n)        # row-major
    np.testing.assert_allclose(got, 0.5 * (T + S), rtol=0, atol=1e-14)
    t32 = dr.section("T32").cpu().numpy()[: n * n].reshape(n, n)
    np.testing.assert_array_equal(t32, got.astype(np.float32))


@pytest.mark.parametrize("out_prec", [strom.ST_F64, strom.ST_F32])
def test_cn_form_matches_oracle(cn_rom, out_prec):
    name, dr, pieces, Phi_t = cn_rom
    prob = dr.prob
    n_q = 6
    nt = _profiles(name, n_q, 81)
    mus = W.sample_params(prob, n_q, seed=82)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    mats, rhs, coff, moff, info = strom.st_form(dr.desc, dr.rom, dA, df, d0, torch.tensor(nt, device="cuda"), out_prec)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    mats, rhs, coff, moff = mats.cpu().numpy(), rhs.cpu().numpy(), coff.cpu().numpy(), moff.cpu().numpy()
    tol = 1e-12 if out_prec == strom.ST_F64 else 2.0 ** -23
    for q in range(n_q):
        M, b = _oracle_cn(prob, pieces, Phi_t, tA[q], tf[q], t0[q], nt[q])
        w = M.shape[0]
        Mg = mats[moff[q]: moff[q] + w * w].reshape(w, w)
        assert np.abs(Mg - M).max() <= tol * np.abs(M).max(), (q, np.abs(Mg - M).max())
        assert np.abs(rhs[coff[q]: coff[q] + w] - b).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("lu_prec", [strom.ST_F64, strom.ST_F32])
def test_cn_solve_matches_oracle(cn_rom, lu_prec):
    name, dr, pieces, Phi_t = cn_rom
    prob = dr.prob
    n_q = 10
    nt = _profiles(name, n_q, 83)
    mus = W.sample_params(prob, n_q, seed=84)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    ntd = torch.tensor(nt, device="cuda")
    b = strom.st_solve(dr.desc, dr.rom, dA, df, d0, ntd, lu_prec=lu_prec,
                       ir_tol=1e-13 if lu_prec == strom.ST_F32 else 0.0, ir_max=12 if lu_prec == strom.ST_F32 else 0)
    torch.cuda.synchronize()
    info = b.info.cpu().numpy()[:n_q]
    relres = b.relres.cpu().numpy()[:n_q]
    coeff, off = b.coeff.cpu().numpy(), b.coeff_off.cpu().numpy()
    assert (info == 0).all(), info
    assert relres.max() <= 1e-12
    for q in range(n_q):
        M, rhs = _oracle_cn(prob, pieces, Phi_t, tA[q], tf[q], t0[q], nt[q])
        assert _rel(coeff[off[q]:off[q + 1]], orom.solve(M, rhs)) <= RTOL
    # the certificate evaluates the same Crank-Nicolson residual
    rr, cert = strom.st_certify(dr.desc, dr.rom, dA, df, d0, b.coeff, ntd)
    torch.cuda.synchronize()
    assert rr.cpu().numpy().max() <= 1e-12


def test_cn_long_horizon_gather_residual():
    """N_t = 320 with 40 modes: the refinement residual takes the gather kernel over the
    row-major T_cn and K; FP32 + refinement against the oracle."""
    prob = C.problem("c_long")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("c_long")
    dr = DeviceRom(prob, Phi_s, Phi_t, integrator=strom.ST_CRANK_NICOLSON)
    Ahat, bhat, u0hat = C.oracle_spatial("c_long")
    Au0hat = [Phi_s.T @ (A @ prob.u0) for A in prob.terms]
    mus = W.sample_params(prob, 4, seed=85)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    b = strom.st_solve(dr.desc, dr.rom, dA, df, d0, None, lu_prec=strom.ST_F32, ir_tol=1e-13, ir_max=12)
    torch.cuda.synchronize()
    assert (b.info.cpu().numpy()[:4] == 0).all()
    coeff, off = b.coeff.cpu().numpy(), b.coeff_off.cpu().numpy()
    for q in range(4):
        M, rhs = cn.reduced_system(Ahat, tA[q], bhat, tf[q], prob.g, u0hat, Au0hat, t0[q], Phi_t, prob.dt)
        assert _rel(coeff[off[q]:off[q + 1]], orom.solve(M, rhs)) <= RTOL


def test_cn_unsupported_paths_report_it():
    prob = C.problem("c1")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("c1")
    dr = DeviceRom(prob, Phi_s, Phi_t, integrator=strom.ST_CRANK_NICOLSON)
    mus = W.sample_params(prob, 2, seed=86)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    with pytest.raises(strom.StromError) as e:
        strom.st_spatial_march(dr.desc, dr.rom, dA, df, d0)
    assert e.value.code == -5
