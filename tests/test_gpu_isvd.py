"""GPU parity of the incremental SVD (Sec. 4.2, Alg. 1-2) against the oracle.

The device stream (st_isvd_update, called through the C ABI) and the oracle's
stream (oracle.isvd) see the same seeded snapshots and thresholds; they must
take the same decisions (rank, dependent snapshots) and agree on the factors
to rounding: singular values to 1e-12 of sigma_1, singular vectors up to sign
within a bound that scales with 1 / (relative gap), the snapshot
reconstruction and the orthonormality of W.
"""
import numpy as np
import pytest
import torch

from oracle import isvd as oisvd
from oracle import pod
from paper_1910_01260_amd import strom
from tests import _cases as C
from tests._gpu import colmajor

pytestmark = pytest.mark.gpu


def _stream(U, r_max, eps_svd, eps_sv, m_max=None, chunks=1):
    N, m = U.shape
    dev = strom.IncrementalSVD(N, r_max, m if m_max is None else m_max, eps_svd, eps_sv)
    Ud = colmajor(U)
    cuts = np.linspace(0, m, chunks + 1).astype(int)
    for a, b in zip(cuts[:-1], cuts[1:]):
        if b > a:
            dev.update(Ud[:, a:b])
    torch.cuda.synchronize()
    return dev


def _rel_gaps(s):
    s = np.asarray(s)
    g = np.full(len(s), np.inf)
    for i in range(len(s)):
        others = np.delete(s, i)
        if len(others):
            g[i] = np.min(np.abs(others - s[i])) / s[0]
    return g


def _compare(dev, Wo, so, Vo, s_tol=1e-12, vec_tol=1e-12, orth_tol=1e-13):
    W, s, V = dev.factors()
    assert len(s) == len(so), (len(s), len(so))
    s1 = so[0]
    assert np.abs(s - so).max() <= s_tol * s1, np.abs(s - so).max() / s1
    gaps = _rel_gaps(so)
    for i in range(len(so)):
        sg = 1.0 if W[:, i] @ Wo[:, i] >= 0 else -1.0
        bound = vec_tol / max(gaps[i], 1e-300) + 1e-13
        assert np.linalg.norm(sg * W[:, i] - Wo[:, i]) <= bound, (i, np.linalg.norm(sg * W[:, i] - Wo[:, i]), bound)
        assert np.linalg.norm(sg * V[:, i] - Vo[:, i]) <= bound, (i, np.linalg.norm(sg * V[:, i] - Vo[:, i]), bound)
    assert np.abs(W.T @ W - np.eye(len(s))).max() <= orth_tol
    return W, s, V


@pytest.mark.parametrize("r_max", [256, 128])
def test_isvd_advection_diffusion_stream_matches_oracle(r_max):
    # 1-D advection-diffusion, N_s = 256, 4 x 128 snapshots; thresholds in a gap
    # of the spectrum (between sigma_35 and sigma_36), at two rank limits (the
    # factor updates stage (r_max + 1)-column tiles).
    U = C.snapshots("c1")
    sc = np.linalg.norm(U, axis=0).max()
    eps = 2.5e-11 * sc
    ev = []
    Wo, so, Vo = oisvd.incremental_svd(U, eps, eps, r_max=r_max, events=ev)
    dev = _stream(U, r_max, eps, eps)
    cnt = dev.counters()
    assert cnt["snapshots"] == U.shape[1] and cnt["refused"] == 0
    assert cnt["dependent"] == sum(e.startswith("dependent") for e in ev)
    W, s, V = _compare(dev, Wo, so, Vo)
    rec = np.linalg.norm(U - W @ np.diag(s) @ V.T) / np.linalg.norm(U)
    rec_o = np.linalg.norm(U - Wo @ np.diag(so) @ Vo.T) / np.linalg.norm(U)
    assert rec <= 1.5 * rec_o + 1e-13, (rec, rec_o)


@pytest.mark.parametrize("seed,N,m,r", [(0, 300, 200, 40), (1, 77, 130, 77)])
def test_isvd_graded_stream_matches_oracle(seed, N, m, r):
    # graded spectrum 1 .. 1e-6 over r directions; the second case has a full
    # row rank (r = N), so late snapshots are dependent on a complete basis
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((N, r)) @ np.diag(10.0 ** -np.linspace(0, 6, r)) @ rng.standard_normal((r, m))
    ev = []
    Wo, so, Vo = oisvd.incremental_svd(U, 1e-11, 1e-13, r_max=256, events=ev)
    dev = _stream(U, 256, 1e-11, 1e-13)
    assert dev.counters()["dependent"] == sum(e.startswith("dependent") for e in ev)
    _compare(dev, Wo, so, Vo)
    sb = np.linalg.svd(U, compute_uv=False)
    assert np.abs(dev.factors()[1] - sb[:len(so)]).max() <= 1e-13 * sb[0]


def test_isvd_chunked_calls_equal_one_call():
    # the stream is the same whether the snapshots come in one call or several
    U = C.snapshots("c1")[:, :200]
    a = _stream(U, 64, 1e-9, 1e-9, chunks=1)
    b = _stream(U, 64, 1e-9, 1e-9, chunks=7)
    for x, y in zip(a.factors(), b.factors()):
        assert np.array_equal(x, y)
    assert a.counters() == b.counters()


def test_isvd_hand_cases():
    e = np.eye(6)
    # zero first snapshot (skipped, zero row), then u, then 2u (dependent)
    u = np.array([0.0, 3.0, 4.0, 0.0, 0.0, 0.0])
    dev = _stream(np.stack([np.zeros(6), u, 2 * u], axis=1), 4, 1e-10, 1e-12)
    c = dev.counters()
    assert (c["rank"], c["snapshots"], c["skipped"], c["dependent"]) == (1, 3, 1, 1)
    W, s, V = dev.factors()
    assert abs(s[0] - 5.0 * np.sqrt(5.0)) < 1e-13
    assert V[0, 0] == 0.0 and np.allclose(np.abs(V[1:, 0]), np.array([1, 2]) / np.sqrt(5.0), atol=1e-15)
    # u1 = 3 e1, u2 = 4 e2: sigma = (4, 3), W = [e2, e1]
    dev = _stream(np.stack([3 * e[0], 4 * e[1]], axis=1), 4, 1e-12, 1e-12)
    W, s, V = dev.factors()
    assert np.allclose(s, [4, 3], atol=1e-15) and np.allclose(np.abs(W), np.abs(e[:, [1, 0]]), atol=1e-15)
    # rank cap r_max = 1 keeps the larger triplet
    dev = _stream(np.stack([3 * e[0], 4 * e[1]], axis=1), 1, 1e-12, 1e-12)
    W, s, V = dev.factors()
    assert dev.counters()["truncated"] == 1 and np.allclose(s, [4]) and np.allclose(np.abs(V[:, 0]), [0, 1])
    # m_max = 2 refuses the third snapshot
    dev = _stream(np.stack([3 * e[0], 4 * e[1], e[2]], axis=1), 4, 1e-12, 1e-12, m_max=2)
    c = dev.counters()
    assert (c["snapshots"], c["refused"], c["rank"]) == (2, 1, 2)


def test_isvd_rank_cap_at_the_limit():
    # full-rank stream of 300 snapshots into r_max = 256: the last 44 updates each
    # drop their trailing triplet, on both sides
    rng = np.random.default_rng(5)
    U = rng.standard_normal((400, 300)) * (0.98 ** np.arange(300))
    Wo, so, Vo = oisvd.incremental_svd(U, 1e-12, 1e-14, r_max=256)
    dev = _stream(U, 256, 1e-12, 1e-14)
    c = dev.counters()
    assert c["rank"] == 256 and c["truncated"] == 300 - 256
    W, s, V = dev.factors()
    assert np.abs(s - so).max() <= 1e-12 * so[0]
    # 300 updates of 256-column products: the column norms drift by ~eps sqrt(r) per update
    assert np.abs(W.T @ W - np.eye(256)).max() <= 3e-13
    # the spanned subspaces agree (individual vectors of this flat spectrum are
    # ill-conditioned)
    cosines = np.linalg.svd(W.T @ Wo, compute_uv=False)
    assert cosines.min() > 1 - 1e-10


def test_isvd_reorthonormalisation_matches_oracle():
    # perturb W on the device so that its first and last columns are 1e-9 from
    # orthogonal; the next snapshot's update must re-orthonormalise, as the oracle's
    rng = np.random.default_rng(7)
    U = rng.standard_normal((64, 31))
    dev = _stream(U[:, :30], 40, 1e-12, 1e-14, m_max=31)
    r = dev.counters()["rank"]
    with torch.no_grad():
        dev.W_store[r - 1] += 1e-9 * dev.W_store[0]
    torch.cuda.synchronize()
    W0, s0, V0 = dev.factors()
    dev.update(colmajor(U[:, 30:31]))
    torch.cuda.synchronize()
    Wo, so, Vo, ev = oisvd.update(W0, s0, V0, U[:, 30], 1e-12, 1e-14, 40)
    assert ev == "update+qr" and dev.counters()["reorthonormalisations"] == 1
    _compare(dev, Wo, so, Vo, vec_tol=1e-11)


def test_isvd_bases_match_oracle_and_batch_pod():
    # Phi_s, sigma and the temporal bases from the stream equal the oracle's, and
    # equal the oracle's batch POD to the truncation level
    prob = C.problem("c1")
    U = C.snapshots("c1")
    n_s, n_t = C.BASIS_SIZES["c1"]
    nt = np.full(n_s, n_t)
    sc = np.linalg.norm(U, axis=0).max()
    eps = 2.5e-11 * sc
    Wo, so, Vo = oisvd.incremental_svd(U, eps, eps, r_max=256)
    Phi_o, sig_o, Pt_o, rk_o = oisvd.bases(Wo, so, Vo, prob.N_t, len(prob.train_mu), n_s, nt)
    dev = _stream(U, 256, eps, eps)
    Phi, Pt, sig, rk = dev.bases(prob.N_t, len(prob.train_mu), n_s, nt)
    torch.cuda.synchronize()
    assert np.abs(sig.cpu().numpy() - sig_o).max() <= 1e-12 * sig_o[0]
    assert np.abs(Phi.cpu().numpy() - Phi_o).max() <= 1e-9
    assert list(rk.cpu().numpy()) == list(rk_o)
    assert np.abs(Pt.cpu().numpy() - np.concatenate(Pt_o, axis=1)).max() <= 1e-8
    Phi_b, sig_b, V_b = pod.pod(U, n_s)
    assert np.abs(sig.cpu().numpy() - sig_b[:n_s]).max() <= 1e-10 * sig_b[0]
    assert np.abs(Phi.cpu().numpy() - Phi_b).max() <= 1e-8


def test_isvd_many_parameter_stream_matches_oracle():
    # 32 training parameters x 128 steps (4096 snapshots) of the advection-diffusion case
    U = C.snapshots("cb")
    sc = np.linalg.norm(U, axis=0).max()
    eps = 2.5e-11 * sc
    ev = []
    Wo, so, Vo = oisvd.incremental_svd(U, eps, eps, r_max=256, events=ev)
    dev = _stream(U, 256, eps, eps, chunks=4)
    assert dev.counters()["dependent"] == sum(e.startswith("dependent") for e in ev)
    # each of the oracle's 4096 LAPACK decompositions of the middle matrix adds a
    # rounding error of ~eps sigma_1 to its factors; over the stream they reach
    # ~1e-12 sigma_1 (its sigma_1 ends 1.1e-12 sigma_1 below the batch SVD's); the
    # column norms of W drift like a random walk of ~eps per update (the oracle's
    # own W ends 2.3e-13 from orthonormal)
    W, s, V = _compare(dev, Wo, so, Vo, s_tol=4e-12, vec_tol=4e-12, orth_tol=4e-13)
    # the leading singular values, which the truncations barely touch, against the
    # batch SVD of all the snapshots
    sb = np.linalg.svd(U, compute_uv=False)
    assert np.abs(s[:10] - sb[:10]).max() <= 1e-12 * sb[0]


def test_isvd_transport_full_rows_matches_oracle():
    # 2-D transport at its full size (N_s = 49152), the first two parameters'
    # 400 snapshots, thresholds 1e-6 of the largest snapshot norm
    U = C.snapshots("c2")[:, :400]
    sc = np.linalg.norm(U, axis=0).max()
    eps = 1e-6 * sc
    ev = []
    Wo, so, Vo = oisvd.incremental_svd(U, eps, eps, r_max=128, events=ev)
    dev = _stream(U, 128, eps, eps)
    assert dev.counters()["dependent"] == sum(e.startswith("dependent") for e in ev)
    _compare(dev, Wo, so, Vo, vec_tol=1e-11)


def test_isvd_transport_whole_stream_properties():
    # all 8 x 200 snapshots of the 2-D transport case: W stays orthonormal, the
    # leading singular values match the batch SVD's to the truncation level and
    # every sampled snapshot is reproduced to it (each dropped triplet or
    # dependent residual is below eps, so the error is at most their sum)
    U = C.snapshots("c2")
    sc = np.linalg.norm(U, axis=0).max()
    eps = 1e-6 * sc
    dev = _stream(U, 128, eps, eps, chunks=8)
    c = dev.counters()
    assert c["snapshots"] == U.shape[1] and c["refused"] == 0 and c["rank"] < 128
    W, s, V = dev.factors()
    assert np.abs(W.T @ W - np.eye(len(s))).max() <= 1e-12
    drop = (c["dependent"] + c["truncated"]) * eps
    sb = np.sqrt(np.maximum(np.linalg.eigvalsh(U.T @ U)[::-1][:40], 0.0))
    assert np.abs(s[:40] - sb).max() <= drop + 1e-7 * sb[0]
    cols = np.random.default_rng(0).choice(U.shape[1], 64, replace=False)
    err = np.linalg.norm(U[:, cols] - W @ (s[:, None] * V[cols].T), axis=0)
    assert err.max() <= drop
