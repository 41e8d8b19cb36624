"""GPU parity of the online path against the CPU oracle, through the C ABI.

Identical bases (the oracle's POD) are fed to both sides, so these tests pin
projection, temporal contractions, per-query assembly and the batched solve.
FP64 results must match the oracle to 1e-10 relative; the FP32-LU path with
FP64 refinement must reach its residual tolerance and the same 1e-10 error on
the coefficients once refined to 1e-12.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import rom as orom  # noqa: E402
from paper_1910_01260_amd import strom  # noqa: E402
from paper_1910_01260_amd import workloads as W  # noqa: E402

from . import _cases as C  # noqa: E402
from ._gpu import DeviceRom, thetas_device  # noqa: E402

RTOL = 1e-10


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.fixture(scope="module")
def c1_rom():
    prob = C.problem("c1")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("c1")
    print(f"[c1] building device ROM n_s={Phi_s.shape[1]} n={sum(P.shape[1] for P in Phi_t)}", flush=True)
    return DeviceRom(prob, Phi_s, Phi_t)


@pytest.fixture(scope="module")
def cb_rom():
    prob = C.problem("cb")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("cb")
    print(f"[cb] building device ROM n_s={Phi_s.shape[1]} n={sum(P.shape[1] for P in Phi_t)}", flush=True)
    return DeviceRom(prob, Phi_s, Phi_t)


@pytest.fixture(scope="module")
def c2s_rom():
    prob = C.problem("c2_small")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("c2_small")
    print(f"[c2_small] building device ROM N_s={prob.N_s}", flush=True)
    return DeviceRom(prob, Phi_s, Phi_t)


def test_library_version():
    assert strom.st_version() == 2


@pytest.mark.parametrize("name", ["c1", "cb", "c2s"])
def test_projection_and_temporal_pieces(name, request):
    """Ahat_q = Phi_s^T A_q Phi_s (Eq. (galerkin)), bhat, u0hat, and the temporal
    pieces T, K, Wf, P1 against their definitions."""
    dr = request.getfixturevalue({"c1": "c1_rom", "cb": "cb_rom", "c2s": "c2s_rom"}[name])
    key = {"c1": "c1", "cb": "cb", "c2s": "c2_small"}[name]
    prob = dr.prob
    Ahat, bhat, u0hat = C.oracle_spatial(key)
    n_s = Ahat[0].shape[0]
    got = dr.section("Ahat").cpu().numpy()[: prob.Q * n_s * n_s].reshape(prob.Q, n_s, n_s)
    for q in range(prob.Q):
        np.testing.assert_allclose(got[q].T, Ahat[q], rtol=0, atol=1e-12 * np.abs(Ahat[q]).max())
    if prob.Qf:
        gb = dr.section("bhat").cpu().numpy()[: prob.Qf * n_s].reshape(prob.Qf, n_s).T
        np.testing.assert_allclose(gb, bhat, rtol=0, atol=1e-12 * np.abs(bhat).max())
    if prob.Q0:
        gu = dr.section("u0hat").cpu().numpy()[: prob.Q0 * n_s].reshape(prob.Q0, n_s).T
        np.testing.assert_allclose(gu, u0hat, rtol=0, atol=1e-12 * np.abs(u0hat).max())
    Phi_t = C.oracle_bases(key)[3]
    P = np.concatenate(Phi_t, axis=1)
    n = P.shape[1]
    T = dr.section("T").cpu().numpy()[: n * n].reshape(n, n).T
    np.testing.assert_allclose(T, P.T @ (prob.dt[:, None] * P), rtol=0, atol=1e-14)
    np.testing.assert_allclose(dr.section("P1").cpu().numpy()[:n], P[0], rtol=0, atol=0)
    # the bases and steps copied into the buffer for the residual
    np.testing.assert_array_equal(dr.section("Phit").cpu().numpy()[: prob.N_t * n].reshape(n, prob.N_t).T, P)
    np.testing.assert_array_equal(dr.section("dt").cpu().numpy()[: prob.N_t], prob.dt)
    K = dr.section("K").cpu().numpy()
    off = 0
    for Pi in Phi_t:
        m = Pi.shape[1]
        Ki = K[off: off + m * m].reshape(m, m).T
        np.testing.assert_allclose(Ki, Pi.T @ Pi - Pi[1:].T @ Pi[:-1], rtol=0, atol=1e-14)
        off += m * m


def _form_and_compare(dr, key, mus, nt=None, out_prec=strom.ST_F64, tol=1e-12):
    prob = dr.prob
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    nt_d = torch.tensor(nt, device="cuda") if nt is not None else None
    mats, rhs, coff, moff, info = strom.st_form(dr.desc, dr.rom, dA, df, d0, nt_d, out_prec)
    torch.cuda.synchronize()
    mats = mats.cpu().numpy()
    rhs = rhs.cpu().numpy()
    coff = coff.cpu().numpy()
    moff = moff.cpu().numpy()
    assert (info.cpu().numpy() == 0).all()
    for q in range(len(mus)):
        M, b = C.oracle_system(key, tA[q], tf[q], t0[q], None if nt is None else nt[q])
        w = M.shape[0]
        assert coff[q + 1] - coff[q] == w
        Mg = mats[moff[q]: moff[q] + w * w].reshape(w, w)
        scale = max(np.abs(M).max(), 1e-300)
        assert np.abs(Mg - M).max() <= tol * scale, (q, np.abs(Mg - M).max() / scale)
        assert np.abs(rhs[coff[q]: coff[q] + w] - b).max() <= 1e-12 * max(np.abs(b).max(), 1e-300) + 1e-300


def test_form_c1_full_width(c1_rom):
    prob = C.problem("c1")
    _form_and_compare(c1_rom, "c1", W.sample_params(prob, 6))


def test_form_cb_ragged(cb_rom):
    prob = C.problem("cb")
    nt = W.ragged_profiles(12, 40)
    _form_and_compare(cb_rom, "cb", W.sample_params(prob, 12), nt)


def test_form_c2_small(c2s_rom):
    prob = C.problem("c2_small")
    nt = np.tile(np.array([12, 7, 3, 12, 1, 12, 5, 12, 12, 2, 12, 12, 9, 12, 12, 4, 12, 12, 6, 12], dtype=np.int32),
                 (3, 1))
    _form_and_compare(c2s_rom, "c2_small", W.sample_params(prob, 3), nt)


def test_form_fp32_rounding(cb_rom):
    """FP32 systems: each entry is computed from the FP32 copy of T and rounded to
    FP32, so it carries at most two FP32 roundings (2 * 2^-24 of the scale)."""
    prob = C.problem("cb")
    nt = W.ragged_profiles(4, 40, seed=3)
    _form_and_compare(cb_rom, "cb", W.sample_params(prob, 4, seed=4), nt, out_prec=strom.ST_F32, tol=2.0 ** -23)


def _solve_and_compare(dr, key, mus, nt=None, lu_prec=strom.ST_F64, ir_tol=0.0, ir_max=0, rtol=RTOL):
    prob = dr.prob
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    nt_d = torch.tensor(nt, device="cuda") if nt is not None else None
    print(f"[{key}] st_solve n_q={len(mus)} prec={lu_prec} ir_max={ir_max}", flush=True)
    b = strom.st_solve(dr.desc, dr.rom, dA, df, d0, nt_d, lu_prec=lu_prec, ir_tol=ir_tol, ir_max=ir_max)
    torch.cuda.synchronize()
    coeff = b.coeff.cpu().numpy()
    coff = b.coeff_off.cpu().numpy()
    info = b.info.cpu().numpy()[: len(mus)]
    relres = b.relres.cpu().numpy()[: len(mus)]
    assert (info == 0).all(), info
    errs = []
    for q in range(len(mus)):
        M, rhs = C.oracle_system(key, tA[q], tf[q], t0[q], None if nt is None else nt[q])
        c = orom.solve(M, rhs)
        errs.append(_rel(coeff[coff[q]: coff[q + 1]], c))
    assert max(errs) <= rtol, max(errs)
    return relres, b.iters.cpu().numpy()[: len(mus)], errs


def test_solve_fp64_c1(c1_rom):
    prob = C.problem("c1")
    relres, _, errs = _solve_and_compare(c1_rom, "c1", W.sample_params(prob, 16))
    assert relres.max() < 1e-12


def test_solve_fp64_cb_ragged(cb_rom):
    prob = C.problem("cb")
    nt = W.ragged_profiles(24, 40)
    relres, _, errs = _solve_and_compare(cb_rom, "cb", W.sample_params(prob, 24), nt)
    assert relres.max() < 1e-12


def test_solve_fp32_ir_cb_ragged(cb_rom):
    prob = C.problem("cb")
    nt = W.ragged_profiles(24, 40, seed=7)
    relres, iters, errs = _solve_and_compare(cb_rom, "cb", W.sample_params(prob, 24, seed=8), nt,
                                             lu_prec=strom.ST_F32, ir_tol=1e-13, ir_max=12)
    assert relres.max() <= 1e-13
    assert iters.max() <= 12


def test_solve_c2_small_fp64_and_fp32(c2s_rom):
    prob = C.problem("c2_small")
    mus = W.sample_params(prob, 6)
    _solve_and_compare(c2s_rom, "c2_small", mus)
    _solve_and_compare(c2s_rom, "c2_small", mus, lu_prec=strom.ST_F32, ir_tol=1e-13, ir_max=12)


def test_solve_long_horizon_gather_residual():
    """N_t = 320 with 40 modes: the refinement residual takes the gather kernel over T and
    K (its time-grid arrays do not fit in LDS); FP64 and FP32 + refinement vs the oracle."""
    prob = C.problem("c_long")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("c_long")
    assert 2 * 40 * prob.N_t * 8 > 150 * 1024
    print(f"[c_long] building device ROM n = {sum(P.shape[1] for P in Phi_t)}", flush=True)
    dr = DeviceRom(prob, Phi_s, Phi_t)
    mus = W.sample_params(prob, 6, seed=13)
    _solve_and_compare(dr, "c_long", mus)
    relres, iters, errs = _solve_and_compare(dr, "c_long", mus, lu_prec=strom.ST_F32, ir_tol=1e-13, ir_max=12)
    assert relres.max() <= 1e-13


def test_solve_edge_widths(cb_rom):
    """Zero-width modes, width-1 queries, one full-width query, ragged tails."""
    prob = C.problem("cb")
    nt = np.zeros((5, 40), dtype=np.int32)
    nt[0, 0] = 1                                   # width 1
    nt[1, 5] = 3; nt[1, 39] = 2                    # two modes only
    nt[2] = 32                                     # full width 1280
    nt[3, :] = np.arange(40) % 33                  # ragged, zeros included
    nt[4, ::3] = 17
    _solve_and_compare(cb_rom, "cb", W.sample_params(prob, 5, seed=11), nt)
    _solve_and_compare(cb_rom, "cb", W.sample_params(prob, 5, seed=11), nt, lu_prec=strom.ST_F32, ir_tol=1e-13,
                       ir_max=12)


def test_solve_empty_batch(cb_rom):
    prob = C.problem("cb")
    dA = torch.zeros((0, prob.Q), dtype=torch.float64, device="cuda")
    b = strom.st_solve(cb_rom.desc, cb_rom.rom, dA, None, torch.zeros((0, 1), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert b.n_q == 0


def test_solve_flags_bad_queries(cb_rom):
    """Invalid profile -> -4, non-finite theta -> -5, capacity -> -3; the
    remaining queries are still solved correctly."""
    prob = C.problem("cb")
    mus = W.sample_params(prob, 4, seed=12)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    dA[2, 1] = float("nan")
    nt = np.full((4, 40), 10, dtype=np.int32)
    nt[1, 3] = 33                                   # > 32 available
    nt_d = torch.tensor(nt, device="cuda")
    widths = nt.sum(axis=1)
    b = strom.SolveBuffers(cb_rom.desc, 4, widths, strom.ST_F64)
    b.sum_w = int(widths[0] + widths[3])            # capacity for two queries of width 400
    out = strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, nt_d, bufs=b)
    torch.cuda.synchronize()
    info = out.info.cpu().numpy()[:4]
    assert info[1] == -4 and info[2] == -5
    assert info[0] == 0 and info[3] == 0            # invalid queries take no space
    M, rhs = C.oracle_system("cb", tA[3], tf[3], t0[3], nt[3])
    coff = out.coeff_off.cpu().numpy()
    assert _rel(out.coeff.cpu().numpy()[coff[3]: coff[4]], orom.solve(M, rhs)) <= RTOL
    b2 = strom.SolveBuffers(cb_rom.desc, 4, widths, strom.ST_F64)
    b2.sum_w = 500
    ok = np.full((4, 40), 10, dtype=np.int32)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    out = strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, torch.tensor(ok, device="cuda"), bufs=b2)
    torch.cuda.synchronize()
    info = out.info.cpu().numpy()[:4]
    assert info[0] == 0 and (info[1:] == -3).all()


def test_exactly_singular_query_reports_pivot():
    """A crafted one-unknown ROM with Ahat_st = 1 - theta * 1 * 0.5 = 0 exactly
    (theta = 2): info = 1 and NaN coefficients; theta = 1 solves."""
    import scipy.sparse as sp

    N, Nt = 4, 4
    prob = W.Problem(name="unit", terms=[sp.identity(N, format="csr")], theta_A=lambda m: np.array([m[0]]),
                     Bf=np.zeros((N, 0)), theta_f=lambda m: np.zeros(0), g=np.zeros((Nt, 0)),
                     u0=np.eye(N)[:, :1], theta_0=lambda m: np.array([1.0]), dt=np.full(Nt, 0.5),
                     box_lo=np.array([0.0]), box_hi=np.array([3.0]), train_mu=np.array([[1.0]]))
    dr = DeviceRom(prob, np.eye(N)[:, :1], [np.eye(Nt)[:, :1]])
    mus = np.array([[2.0], [1.0]])
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    out = strom.st_solve(dr.desc, dr.rom, dA, df, d0)
    torch.cuda.synchronize()
    info = out.info.cpu().numpy()[:2]
    coeff = out.coeff.cpu().numpy()
    assert info[0] == 1 and np.isnan(coeff[0])
    assert info[1] == 0 and abs(coeff[1] - 1.0 / (1.0 - 0.5)) < 1e-15


def test_unconverged_refinement_falls_back_to_fp64(cb_rom):
    """FP32 LU with no refinement steps and a tolerance the FP32 solve cannot meet:
    every query ends unconverged and is re-formed and re-solved with the FP64 LU
    (info -6); the results then meet the FP64 parity bar."""
    prob = C.problem("cb")
    nt = W.ragged_profiles(12, 40, seed=41)
    mus = W.sample_params(prob, 12, seed=42)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    print("[cb] st_solve FP32, ir_max=0, ir_tol=1e-14 (forced FP64 re-solve)", flush=True)
    # a workspace sized for FP64 systems holds every re-solve
    bufs = strom.SolveBuffers(cb_rom.desc, 12, nt.sum(axis=1), strom.ST_F64)
    b = strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, torch.tensor(nt, device="cuda"), lu_prec=strom.ST_F32,
                       ir_tol=1e-14, ir_max=0, bufs=bufs)
    torch.cuda.synchronize()
    info = b.info.cpu().numpy()[:12]
    relres = b.relres.cpu().numpy()[:12]
    coeff, off = b.coeff.cpu().numpy(), b.coeff_off.cpu().numpy()
    assert (info == -6).all(), info
    assert relres.max() <= 1e-12, relres
    for q in range(12):
        M, rhs = C.oracle_system("cb", tA[q], tf[q], t0[q], nt[q])
        assert _rel(coeff[off[q]:off[q + 1]], orom.solve(M, rhs)) <= RTOL


def test_fp64_resolve_that_does_not_fit_keeps_minus_one(cb_rom):
    """A workspace sized for the FP32 systems only holds FP64 copies of about half
    of them: the first unconverged queries (in query order) are re-solved in FP64
    (info -6, FP64 accuracy), the rest keep info -1 and the FP32 iterate."""
    prob = C.problem("cb")
    n_q = 6
    nt = np.full((n_q, 40), 32, dtype=np.int32)
    mus = W.sample_params(prob, n_q, seed=44)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    print("[cb] st_solve FP32 with an FP32-sized workspace, forced FP64 re-solve", flush=True)
    b = strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, torch.tensor(nt, device="cuda"), lu_prec=strom.ST_F32,
                       ir_tol=1e-14, ir_max=0)
    torch.cuda.synchronize()
    info = b.info.cpu().numpy()[:n_q]
    relres = b.relres.cpu().numpy()[:n_q]
    coeff, off = b.coeff.cpu().numpy(), b.coeff_off.cpu().numpy()
    k = int(np.sum(info == -6))
    assert 1 <= k < n_q and (info[:k] == -6).all() and (info[k:] == -1).all(), info
    for q in range(n_q):
        M, rhs = C.oracle_system("cb", tA[q], tf[q], t0[q], nt[q])
        err = _rel(coeff[off[q]:off[q + 1]], orom.solve(M, rhs))
        if q < k:
            assert err <= RTOL and relres[q] <= 1e-12
        else:
            assert relres[q] > 1e-14 and err <= 1e-3     # the FP32 solve, unrefined


def test_certify_ragged_matches_oracle_certificate(cb_rom):
    """st_certify on perturbed solutions of ragged queries: relative residual and
    certificate equal the oracle's (bounds.certificate), and the certificate bounds
    the true relative error."""
    from oracle import bounds
    prob = C.problem("cb")
    n_q = 10
    nt = W.ragged_profiles(n_q, 40, seed=45)
    mus = W.sample_params(prob, n_q, seed=46)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    widths = nt.sum(axis=1)
    off = np.concatenate([[0], np.cumsum(widths)])
    rng = np.random.default_rng(47)
    gamma = bounds.coercivity_floor(prob.N_t)
    assert abs(strom.st_coercivity_floor(prob.N_t) - gamma) <= 1e-16
    packed, exact, systems = [], [], []
    for q in range(n_q):
        M, rhs = C.oracle_system("cb", tA[q], tf[q], t0[q], nt[q])
        c = orom.solve(M, rhs)
        pert = 10.0 ** rng.uniform(-10, -4)
        packed.append(c + pert * np.linalg.norm(c) * rng.standard_normal(len(c)) / np.sqrt(len(c)))
        exact.append(c)
        systems.append((M, rhs))
    coeff = torch.tensor(np.concatenate(packed), device="cuda")
    print(f"[cb] st_certify n_q={n_q}", flush=True)
    relres, cert = strom.st_certify(cb_rom.desc, cb_rom.rom, dA, df, d0, coeff, torch.tensor(nt, device="cuda"))
    torch.cuda.synchronize()
    relres, cert = relres.cpu().numpy(), cert.cpu().numpy()
    for q in range(n_q):
        M, rhs = systems[q]
        x = packed[q]
        ref_rel = np.linalg.norm(rhs - M @ x) / np.linalg.norm(rhs)
        ref_cert = bounds.certificate(M, rhs, x, gamma)
        assert abs(relres[q] - ref_rel) <= 1e-8 * ref_rel + 1e-13 * (1 + np.linalg.norm(M) * np.linalg.norm(x)
                                                                     / np.linalg.norm(rhs)), (q, relres[q], ref_rel)
        # the residual of a near-solution is a cancellation: both sides round it to
        # ~eps (||b|| + ||M|| ||x||) absolutely, which the certificate divides by gamma ||x||
        slack = 1e-13 * (np.linalg.norm(rhs) + np.linalg.norm(M) * np.linalg.norm(x)) / (gamma * np.linalg.norm(x))
        if np.isinf(ref_cert):
            assert np.isinf(cert[q]) or cert[q] >= 1.0 / slack, (q, cert[q])
        else:
            assert abs(cert[q] - ref_cert) <= 1e-8 * ref_cert + slack * (1 + ref_cert) ** 2, (q, cert[q], ref_cert)
        assert _rel(x, exact[q]) <= cert[q]
    assert np.isfinite(cert).sum() >= n_q // 2


@pytest.mark.parametrize("prec", [strom.ST_F32, strom.ST_BF16X3])
def test_reduced_precision_projection_reports_error(prec):
    """Projection in reduced precision (FP32 SpMM with FP32 accumulation, then
    Phi_s^T (A_q Phi_s) on the matrix cores in FP32 or split-BF16) on the transport
    problem's three affine terms, against the FP64 oracle (Sec. 3.1, Eq. (galerkin)).

    Elementwise a priori bound (deterministic): the FP32 rounding of the values and
    the basis, the SpMM's FP32 sums of nnz_row terms and the product's sums of N_s
    terms each add at most (k + 2) u relative to |Phi|^T |A_q| |Phi|, with u = 2^-24,
    or u = 2^-16 for the split-BF16 products.  Errors and the resulting ROM solution
    error are printed against FP64."""
    name = "c2_small"
    prob = C.problem(name)
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases(name)
    print(f"[{name}] st_assemble proj_prec={prec}", flush=True)
    dr = DeviceRom(prob, Phi_s, Phi_t, proj_prec=prec)
    n_s = Phi_s.shape[1]
    got = dr.section("Ahat").cpu().numpy()[: prob.Q * n_s * n_s].reshape(prob.Q, n_s, n_s)
    Ahat, bhat, u0hat = C.oracle_spatial(name)
    u_prod = 2.0 ** -16 if prec == strom.ST_BF16X3 else 2.0 ** -24
    worst = 0.0
    for q, Aq in enumerate(prob.terms):
        absA = abs(Aq)
        scale = np.abs(Phi_s).T @ (absA @ np.abs(Phi_s))
        nnz_row = int(np.diff(Aq.indptr).max())
        bound = ((nnz_row + 4) * 2.0 ** -24 + (prob.N_s + 2) * u_prod) * scale
        err = np.abs(got[q].T - Ahat[q])
        assert (err <= bound + 1e-300).all(), (q, float((err / np.maximum(bound, 1e-300)).max()))
        worst = max(worst, float(err.max() / np.abs(Ahat[q]).max()))
    # the ROM solution from the reduced-precision operators, against FP64
    ref = DeviceRom(prob, Phi_s, Phi_t)
    mus = W.sample_params(prob, 4, seed=61)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    b1 = strom.st_solve(dr.desc, dr.rom, dA, df, d0)
    b0 = strom.st_solve(ref.desc, ref.rom, dA, df, d0)
    torch.cuda.synchronize()
    c1, c0 = b1.coeff.cpu().numpy(), b0.coeff.cpu().numpy()
    sol = _rel(c1, c0)
    print(f"[{name}] proj_prec={prec}: max |dAhat|/max|Ahat| {worst:.2e}, ROM solution rel err {sol:.2e}")
    assert sol <= 1e-2
