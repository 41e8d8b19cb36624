"""HIP-graph replay of st_solve and the batched-LU autotuner, on the GPU.

Graph replays must reproduce the eager launch sequence bit for bit (the same
kernels on the same data), including after the inputs behind the recorded
pointers change.  Every LU configuration the autotuner can pick must meet the
same oracle tolerance as the default, in both width classes (total reduced
width up to 1536, and above).
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
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def cb_rom():
    prob = C.problem("cb")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("cb")
    return DeviceRom(prob, Phi_s, Phi_t)


@pytest.fixture(scope="module")
def wide_rom():
    """Transport (32^2, N_t = 100) with n_s = 20 modes of 100 temporal vectors: n = 2000."""
    prob = C.problem("c2_small")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("c2_small")
    from oracle import pod as opod
    Pt, _ = opod.temporal_bases(V, prob.N_t, len(prob.train_mu), np.full(20, 100), 1e-7)
    print(f"[wide] building device ROM n = {sum(P.shape[1] for P in Pt)}", flush=True)
    return DeviceRom(prob, Phi_s, Pt), Phi_s, Pt


def _oracle_coeffs(prob, Phi_s, Phi_t, tA, tf, t0, nt=None, with_cond=False):
    Ahat = [orom.spatial_operator(Phi_s, A) for A in prob.terms]
    bhat = orom.reduced_vector(Phi_s, prob.Bf) if prob.Qf else np.zeros((Phi_s.shape[1], 0))
    u0hat = orom.reduced_vector(Phi_s, prob.u0) if prob.Q0 else np.zeros((Phi_s.shape[1], 0))
    out, cond = [], []
    for q in range(tA.shape[0]):
        Pt = Phi_t if nt is None else [Phi_t[i][:, :int(nt[q][i])] for i in range(len(Phi_t))]
        M, b = orom.reduced_system(Ahat, tA[q], bhat, tf[q], prob.g, u0hat, t0[q], Pt, prob.dt)
        out.append(orom.solve(M, b))
        if with_cond:
            cond.append(float(np.linalg.cond(M)))
    return (out, cond) if with_cond else out


U32 = 2.0 ** -24


def _check_f32_factors(bufs, ref, cond):
    """Plain FP32-LU solve (no refinement): a backward-stable factorization with
    backward error below 20 u_32 gives a forward error below 20 kappa_2 u_32.
    Broken factors (a wrong block of the trailing update, say) miss this by
    orders of magnitude even where refinement would still converge."""
    torch.cuda.synchronize()
    coeff = bufs.coeff.cpu().numpy()
    off = bufs.coeff_off.cpu().numpy()
    errs = [_rel(coeff[off[q]:off[q + 1]], ref[q]) for q in range(len(ref))]
    bounds = [20.0 * k * U32 for k in cond]
    print("  FP32 factors: max err", f"{max(errs):.2e}", "min bound", f"{min(bounds):.2e}", flush=True)
    for q, (e, bd) in enumerate(zip(errs, bounds)):
        assert e <= bd, (q, e, bd)


def _check(bufs, ref):
    torch.cuda.synchronize()
    coeff = bufs.coeff.cpu().numpy()
    off = bufs.coeff_off.cpu().numpy()
    info = bufs.info.cpu().numpy()[: len(ref)]
    assert (info == 0).all(), info
    errs = [_rel(coeff[off[q]:off[q + 1]], ref[q]) for q in range(len(ref))]
    assert max(errs) <= RTOL, max(errs)
    return max(errs)


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_lu_variants_match_oracle_ragged(cb_rom, variant):
    prob = C.problem("cb")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("cb")
    mus = W.sample_params(prob, 12, seed=41)
    nt = W.ragged_profiles(12, 40, seed=42)
    nt[0] = 32   # one full-width query
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    ref, cond = _oracle_coeffs(prob, Phi_s, Phi_t, tA, tf, t0, nt, with_cond=True)
    ntd = torch.tensor(nt, device="cuda")
    n = cb_rom.desc.n
    try:
        for prec in (strom.ST_F64, strom.ST_F32):
            strom.st_autotune_set(prec, n, variant)
            print(f"[variant {variant}] cb prec={prec}", flush=True)
            b = strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, ntd, lu_prec=prec,
                               ir_tol=1e-13 if prec == strom.ST_F32 else 0.0, ir_max=12 if prec == strom.ST_F32 else 0)
            print(f"  max rel err {_check(b, ref):.2e}")
            if prec == strom.ST_F32:
                b = strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, ntd, lu_prec=prec, ir_max=0)
                _check_f32_factors(b, ref, cond)
    finally:
        for prec in (strom.ST_F64, strom.ST_F32):
            strom.st_autotune_set(prec, n, -1)


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_lu_variants_edge_widths(cb_rom, variant):
    """Width 1, two-mode queries, the full width, ragged profiles with zero-width modes and
    widths that are not multiples of any tile, for every LU configuration and precision."""
    prob = C.problem("cb")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("cb")
    nt = np.zeros((7, 40), dtype=np.int32)
    nt[0, 0] = 1                                   # width 1
    nt[1, 5] = 3; nt[1, 39] = 2                    # width 5, two modes
    nt[2] = 32                                     # full width 1280
    nt[3, :] = np.arange(40) % 33                  # ragged, zeros included
    nt[4, ::3] = 17                                # 14 modes of 17: width 238
    nt[5, :4] = [16, 16, 16, 17]                   # width 65: one column past a 64-column block
    nt[6, :5] = [32, 32, 32, 31, 2]                # width 129
    mus = W.sample_params(prob, len(nt), seed=49)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    ref, cond = _oracle_coeffs(prob, Phi_s, Phi_t, tA, tf, t0, nt, with_cond=True)
    ntd = torch.tensor(nt, device="cuda")
    n = cb_rom.desc.n
    try:
        for prec in (strom.ST_F64, strom.ST_F32):
            strom.st_autotune_set(prec, n, variant)
            print(f"[variant {variant}] edge widths prec={prec}", flush=True)
            b = strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, ntd, lu_prec=prec,
                               ir_tol=1e-13 if prec == strom.ST_F32 else 0.0, ir_max=12 if prec == strom.ST_F32 else 0)
            print(f"  max rel err {_check(b, ref):.2e}")
            if prec == strom.ST_F32:
                b = strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, ntd, lu_prec=prec, ir_max=0)
                _check_f32_factors(b, ref, cond)
    finally:
        for prec in (strom.ST_F64, strom.ST_F32):
            strom.st_autotune_set(prec, n, -1)


@pytest.mark.parametrize("variant", [0, 1])
def test_lu_variants_match_oracle_wide(wide_rom, variant):
    dr, Phi_s, Pt = wide_rom
    prob = dr.prob
    mus = W.sample_params(prob, 3, seed=43)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    ref, cond = _oracle_coeffs(prob, Phi_s, Pt, tA, tf, t0, with_cond=True)
    n = dr.desc.n
    assert n > 1536
    try:
        for prec in (strom.ST_F64, strom.ST_F32):
            strom.st_autotune_set(prec, n, variant)
            print(f"[variant {variant}] wide n={n} prec={prec}", flush=True)
            b = strom.st_solve(dr.desc, dr.rom, dA, df, d0, None, lu_prec=prec,
                               ir_tol=1e-13 if prec == strom.ST_F32 else 0.0, ir_max=12 if prec == strom.ST_F32 else 0)
            print(f"  max rel err {_check(b, ref):.2e}")
            if prec == strom.ST_F32:
                b = strom.st_solve(dr.desc, dr.rom, dA, df, d0, None, lu_prec=prec, ir_max=0)
                _check_f32_factors(b, ref, cond)
    finally:
        for prec in (strom.ST_F64, strom.ST_F32):
            strom.st_autotune_set(prec, n, -1)


def test_autotune_records_a_choice(cb_rom):
    prob = C.problem("cb")
    mus = W.sample_params(prob, 64, seed=44)
    nt = W.ragged_profiles(64, 40, seed=45)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    ntd = torch.tensor(nt, device="cuda")
    n = cb_rom.desc.n
    try:
        print("[autotune] cb 64 queries FP32", flush=True)
        choice, ms = strom.st_autotune(cb_rom.desc, cb_rom.rom, dA, df, d0, ntd, strom.ST_F32)
        print(f"  choice {choice}, ms {ms}")
        assert choice in (0, 1, 2) and all(t > 0 for t in ms)
        assert strom.st_autotune_choice(strom.ST_F32, n) == choice
        Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("cb")
        ref = _oracle_coeffs(prob, Phi_s, Phi_t, tA[:8], tf[:8], t0[:8], nt[:8])
        b = strom.st_solve(cb_rom.desc, cb_rom.rom, dA[:8].contiguous(), df[:8].contiguous() if df is not None else None,
                           d0[:8].contiguous() if d0 is not None else None, ntd[:8].contiguous(), lu_prec=strom.ST_F32,
                           ir_tol=1e-13, ir_max=12)
        _check(b, ref)
    finally:
        strom.st_autotune_set(strom.ST_F32, n, -1)


def test_graph_replay_matches_eager(cb_rom):
    prob = C.problem("cb")
    n_q = 16
    mus = W.sample_params(prob, n_q, seed=46)
    nt = W.ragged_profiles(n_q, 40, seed=47)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    ntd = torch.tensor(nt, device="cuda")
    widths = nt.astype(np.int64).sum(axis=1)
    kw = dict(lu_prec=strom.ST_F32, ir_tol=1e-12, ir_max=6)

    def eager(dA_):
        b = strom.st_solve(cb_rom.desc, cb_rom.rom, dA_.clone(), df, d0, ntd, widths=widths, **kw)
        torch.cuda.synchronize()
        return b.coeff.cpu().numpy().copy(), b.relres.cpu().numpy()[:n_q].copy(), b.info.cpu().numpy()[:n_q].copy()

    ce, re, ie = eager(dA)
    strom.st_graph_reset()
    strom.st_graph_enable(True)
    try:
        bufs = strom.SolveBuffers(cb_rom.desc, n_q, widths, strom.ST_F32, "cuda")
        for rep in range(4):
            print(f"[graph] replay {rep}", flush=True)
            strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, ntd, bufs=bufs, **kw)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(bufs.coeff.cpu().numpy(), ce)
            np.testing.assert_array_equal(bufs.relres.cpu().numpy()[:n_q], re)
            np.testing.assert_array_equal(bufs.info.cpu().numpy()[:n_q], ie)
            # unrelated eager work and a clobbered output between replays
            x = torch.randn(1 << 20, device="cuda")
            _ = float((x * x).sum())
            bufs.coeff.fill_(float("nan"))
            torch.cuda.synchronize()
        assert strom.st_graph_count() == 1
        # new parameter values behind the same pointers: the replay must see them
        mus2 = W.sample_params(prob, n_q, seed=48)
        tA2, _, _ = prob.thetas(mus2)
        dA.copy_(torch.tensor(tA2, device="cuda"))
        strom.st_solve(cb_rom.desc, cb_rom.rom, dA, df, d0, ntd, bufs=bufs, **kw)
        torch.cuda.synchronize()
        assert strom.st_graph_count() == 1
        got = bufs.coeff.cpu().numpy().copy()
        strom.st_graph_enable(False)
        ce2, _, _ = eager(dA)
        np.testing.assert_array_equal(got, ce2)
        assert not np.array_equal(ce2, ce)
    finally:
        strom.st_graph_enable(False)
        strom.st_graph_reset()
    assert strom.st_graph_count() == 0
