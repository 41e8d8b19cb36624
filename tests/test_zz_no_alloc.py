"""st_solve_noalloc (static workspace) against st_solve (caller workspace),
through the C ABI: the same kernels on the same inputs give the same results.
Two calls in a row, the second with a smaller ragged batch, so the second
reuses the static array with the first call's contents in it."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import rom as orom  # noqa: E402
from paper_1910_01260_amd import strom  # noqa: E402
from paper_1910_01260_amd import workloads as W  # noqa: E402

from . import _cases as C  # noqa: E402
from ._gpu import DeviceRom, thetas_device  # noqa: E402


def _run_pair(dr, key, n_q, seed, lu_prec, ir_tol, ir_max):
    prob = dr.prob
    mus = W.sample_params(prob, n_q, seed=seed)
    nt = W.ragged_profiles(n_q, dr.desc.n_s, seed=seed + 1)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    nt_d = torch.tensor(nt, device="cuda")
    print(f"[{key}] n_q={n_q} prec={lu_prec}: st_solve then st_solve_noalloc", flush=True)
    ref = strom.st_solve(dr.desc, dr.rom, dA, df, d0, nt_d, lu_prec=lu_prec, ir_tol=ir_tol, ir_max=ir_max)
    got = strom.st_solve_noalloc(dr.desc, dr.rom, dA, df, d0, nt_d, lu_prec=lu_prec, ir_tol=ir_tol, ir_max=ir_max)
    torch.cuda.synchronize()
    for name in ("coeff_off", "info", "iters"):
        np.testing.assert_array_equal(getattr(got, name).cpu().numpy()[: n_q + 1],
                                      getattr(ref, name).cpu().numpy()[: n_q + 1])
    np.testing.assert_array_equal(got.relres.cpu().numpy()[:n_q], ref.relres.cpu().numpy()[:n_q])
    off = ref.coeff_off.cpu().numpy()
    np.testing.assert_array_equal(got.coeff.cpu().numpy()[: off[n_q]], ref.coeff.cpu().numpy()[: off[n_q]])
    assert (got.info.cpu().numpy()[:n_q] == 0).all()
    coeff = got.coeff.cpu().numpy()
    worst = 0.0
    for q in range(n_q):
        M, rhs = C.oracle_system(key, tA[q], tf[q], t0[q], nt[q])
        c = orom.solve(M, rhs)
        worst = max(worst, np.linalg.norm(coeff[off[q]:off[q + 1]] - c) / np.linalg.norm(c))
    assert worst <= 1e-10, worst
    return worst


def test_noalloc_matches_solve_twice():
    prob = C.problem("cb")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("cb")
    dr = DeviceRom(prob, Phi_s, Phi_t)
    n = dr.desc.n
    # the largest batch that fits the static array at full width (FP32 matrices)
    n_big = 8
    assert strom.lib().st_solve_workspace(dr.desc.ref(), n_big, n_big * n, n_big * n * n, strom.ST_F32) \
        <= strom.NOALLOC_SCRATCH_BYTES
    e1 = _run_pair(dr, "cb", n_big, 31, strom.ST_F32, 1e-12, 10)
    e2 = _run_pair(dr, "cb", 3, 33, strom.ST_F32, 1e-12, 10)
    e3 = _run_pair(dr, "cb", 2, 35, strom.ST_F64, 0.0, 0)
    print(f"[cb] st_solve_noalloc vs oracle: {e1:.2e}, {e2:.2e}, {e3:.2e}")


def test_noalloc_rejects_batches_beyond_the_array():
    prob = C.problem("cb")
    Phi_s, sigma, V, Phi_t, ranks = C.oracle_bases("cb")
    dr = DeviceRom(prob, Phi_s, Phi_t)
    n = dr.desc.n
    n_q = 64      # 64 full-width FP64 systems of width 1280 need 840 MB
    mus = W.sample_params(prob, n_q, seed=3)
    (tA, tf, t0), (dA, df, d0) = thetas_device(prob, mus)
    bufs = strom.SolveBuffers(dr.desc, 1, np.array([1]), strom.ST_F64)
    code = strom.lib().st_solve_noalloc(dr.desc.ref(), strom._ptr(dr.rom), n_q, strom._ptr(dA), None,
                                        strom._ptr(d0), None, None, strom.ST_F64, 0.0, 0, strom._ptr(bufs.coeff),
                                        n_q * n, strom._ptr(bufs.coeff_off), strom._ptr(bufs.relres),
                                        strom._ptr(bufs.info), None, None)
    assert code == -3     # ST_EWORKSPACE, before any launch
