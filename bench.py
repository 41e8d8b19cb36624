#!/usr/bin/env python3
"""Benchmark of the space-time ROM hot path on one MI355X.

Workload (batched queries): 1-D periodic advection-diffusion, N_s = 256,
N_t = 128, 32 training parameters (snapshot matrix 256 x 4096), n_s = 40
spatial modes with up to 32 temporal modes each, and 4096 test parameters
whose per-mode temporal truncations give reduced systems 400..1200 wide.

One step = one online pass over that batch, with every input already resident
in HBM: a HIP-graph replay of st_solve (assembly, FP32 LU and FP64-residual
refinement of all 4096 reduced systems, FP64 re-solve of any query that does not
converge).  `value` counts the queries whose certified relative error (st_certify,
on the device) is at most 1e-6, per second of step time.  The offline part (POD,
projection, temporal contractions: st_build_bases + st_assemble) is timed on its
own and reported beside it, as are the plain-FP64 solve, the phase durations of
st_solve (HIP events on the solve's stream), the spatial ROM march, the
certificate and the full-order Theorem-3 bound on the same batch.  The CPU
baseline leg times the oracle on a bounded sample of the same workload and
compares its solutions with the device's.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ST-ROM queries/sec (batched FP32+IR vs plain FP64) at rel err<=1e-6; HBM %"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
IR_TOL = 1e-12      # relative residual of the refinement
IR_MAX = 6
CERT_TOL = 1e-6     # a query counts when its certified relative error is at most this (the metric's bound)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--queries", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle baseline leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["batch", "surrogate", "isvd", "c4", "c2"], default="batch",
                    help="batch: the 4096-query batched solve (default); surrogate: train the learned "
                         "surrogate on batched solves of the transport-with-absorber ROM and measure "
                         "surrogate + certificate + fallback against the batched solve; isvd: stream the "
                         "2-D transport snapshots (49152 x 1600) through the incremental SVD; c4: precision at "
                         "scale on the 3-D 128^3 advection-diffusion problem (8000 FP32 snapshots, 8000^2 Gram "
                         "in three arithmetics, n_s = 100 x 30, 3000-wide reduced solves); c2: the plain FP64 "
                         "ST-ROM of the 2-D transport problem (64^2 x 12, N_t = 200, n_s = 40, n_t = 20)")
    ap.add_argument("--surrogate-train", type=int, default=20000)
    ap.add_argument("--surrogate-steps", type=int, default=6000)
    ap.add_argument("--no-isvd", action="store_true",
                    help="skip the incremental-SVD stream of the batch snapshots (e.g. for hardware-counter runs "
                         "that only need the assembly and LU kernels)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="before the steps, copy a buffer of this size once (device to device) so that a "
                         "hardware-counter run can scale byte counters against a kernel of known traffic")
    return ap.parse_args()


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1910_01260_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(queries would shard across GPUs with no communication between them)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "isvd":
        return bench_isvd(args)
    if args.workload == "c4":
        return bench_c4(args)
    if args.workload == "c2":
        return bench_c2(args)

    import numpy as np
    import torch

    from paper_1910_01260_amd import strom
    from paper_1910_01260_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    strom.lib()  # fail loudly if the HIP library is missing

    # ------------------------------------------------------------- inputs
    t0 = time.time()
    prob = W.advdiff1d(n_train=32)
    n_s, n_t_max = 40, 32
    U = W.snapshots(prob)
    n_mu = len(prob.train_mu)
    nq = args.queries
    mus = W.sample_params(prob, nq)
    nt = W.ragged_profiles(nq, n_s)
    widths = nt.astype(np.int64).sum(axis=1)
    tA, tf, t0_ = prob.thetas(mus)
    print(f"[bench] inputs ready in {time.time() - t0:.1f}s: U {U.shape}, {nq} queries, widths "
          f"{widths.min()}..{widths.max()}", file=sys.stderr, flush=True)

    dev = "cuda"
    Ud = torch.tensor(np.ascontiguousarray(U.T), device=dev).T
    dt = torch.tensor(prob.dt, device=dev)
    csr = [strom.csr_to_device(*W.csr_arrays(A)) for A in prob.terms]
    u0 = torch.tensor(np.ascontiguousarray(prob.u0.T), device=dev).T
    dA = torch.tensor(tA, device=dev)
    d0 = torch.tensor(t0_, device=dev)
    ntd = torch.tensor(nt, device=dev)
    desc = strom.RomDesc([n_t_max] * n_s, prob.N_t, prob.Q, prob.Qf, prob.Q0)
    b32 = strom.SolveBuffers(desc, nq, widths, strom.ST_F32, dev)
    b64 = strom.SolveBuffers(desc, nq, widths, strom.ST_F64, dev)
    torch.cuda.synchronize()

    if args.copy_calibration_gib > 0:
        n_cal = int(args.copy_calibration_gib * (1 << 30)) // 4
        src = torch.ones(n_cal, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {4 * n_cal} bytes read, {4 * n_cal} bytes written", file=sys.stderr,
              flush=True)
        del src, dst

    state = {}

    def offline():
        Phi_s, Phi_t, sigma, rank = strom.st_build_bases(Ud, prob.N_t, n_mu, n_s, [n_t_max] * n_s)
        rom = strom.st_assemble(desc, Phi_s, Phi_t, dt, [c[0] for c in csr], None, None, u0)
        state.update(Phi_s=Phi_s, Phi_t=Phi_t, sigma=sigma, rom=rom)

    def online(prec, bufs):
        strom.st_solve(desc, state["rom"], dA, None, d0, ntd, lu_prec=prec,
                       ir_tol=IR_TOL if prec == strom.ST_F32 else 0.0,
                       ir_max=IR_MAX if prec == strom.ST_F32 else 0, bufs=bufs)

    # ------------------------------------------------------------- offline part (timed on its own)
    offline()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    off_ts = []
    for _ in range(max(3, min(args.steps, 5))):
        ev0.record()
        offline()
        ev1.record()
        torch.cuda.synchronize()
        off_ts.append(ev0.elapsed_time(ev1))
    off_ms = float(np.median(off_ts))
    print(f"[bench] offline (POD + projection + temporal contractions): {off_ms:.2f} ms", file=sys.stderr, flush=True)

    # ------------------------------------------------------------- LU autotuning (once, before the steps)
    tune = {}
    for name, prec, bufs in (("fp32", strom.ST_F32, b32), ("fp64", strom.ST_F64, b64)):
        choice, ms = strom.st_autotune(desc, state["rom"], dA, None, d0, ntd, prec, bufs=bufs)
        tune[name] = {"choice": choice, "lu_ms_per_variant": ms}
    print(f"[bench] LU autotune: {json.dumps(tune)}", file=sys.stderr, flush=True)

    # ------------------------------------------------------------- phase durations (eager runs, HIP events on
    # the solve's stream, the source of the roofline's kernel times)
    def phases(prec, bufs, reps):
        strom.st_timing_enable(True)
        online(prec, bufs)
        torch.cuda.synchronize()
        acc = {k: [] for k in strom.TIMING_PHASES}
        for _ in range(reps):
            online(prec, bufs)
            torch.cuda.synchronize()
            for k, v in strom.st_timing_read().items():
                acc[k].append(v)
        strom.st_timing_enable(False)
        return {k: float(np.median(v)) for k, v in acc.items()}

    ph32 = phases(strom.ST_F32, b32, max(3, args.steps // 2))
    ph64 = phases(strom.ST_F64, b64, max(3, args.steps // 2))
    print(f"[bench] phases fp32+IR {json.dumps({k: round(v, 3) for k, v in ph32.items()})}", file=sys.stderr,
          flush=True)

    # ------------------------------------------------------------- the timed steps: graph replays of st_solve
    strom.st_graph_enable(True)

    def timed_steps(prec, bufs):
        for _ in range(max(1, args.warmup)):
            online(prec, bufs)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for a, b in evs:
            a.record()
            online(prec, bufs)
            b.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        return 1e3 * wall / args.steps, float(np.median([a.elapsed_time(b) for a, b in evs]))

    ms_per_step, med32 = timed_steps(strom.ST_F32, b32)
    _, med64 = timed_steps(strom.ST_F64, b64)
    strom.st_graph_enable(False)
    strom.st_graph_reset()
    K = args.steps

    # ------------------------------------------------------------- certification on the device
    info32 = b32.info.cpu().numpy()[:nq]
    relres32 = b32.relres.cpu().numpy()[:nq]
    iters32 = b32.iters.cpu().numpy()[:nq]
    gamma = strom.st_coercivity_floor(prob.N_t)
    _, cert32 = strom.st_certify(desc, state["rom"], dA, None, d0, b32.coeff, ntd, gamma=gamma)
    _, cert64 = strom.st_certify(desc, state["rom"], dA, None, d0, b64.coeff, ntd, gamma=gamma)
    torch.cuda.synchronize()
    cert32 = cert32.cpu().numpy()
    cert64 = cert64.cpu().numpy()
    info64 = b64.info.cpu().numpy()[:nq]
    ok32 = int(np.sum(((info32 == 0) | (info32 == -6)) & (cert32 <= CERT_TOL)))
    ok64 = int(np.sum((info64 == 0) & (cert64 <= CERT_TOL)))
    value = ok32 / (ms_per_step * 1e-3)
    print(f"[bench] {K} graph-replayed steps: {ms_per_step:.2f} ms/step (median {med32:.2f} ms), {ok32}/{nq} "
          f"certified <= {CERT_TOL:g}: {value:.0f} queries/s; plain FP64 {med64:.2f} ms ({ok64} certified)",
          file=sys.stderr, flush=True)
    c32 = b32.coeff.cpu().numpy()
    c64 = b64.coeff.cpu().numpy()
    off = b32.coeff_off.cpu().numpy()
    d3264 = max(float(np.linalg.norm(c32[off[q]:off[q + 1]] - c64[off[q]:off[q + 1]]) /
                      np.linalg.norm(c64[off[q]:off[q + 1]])) for q in range(nq))

    # ------------------------------------------------------------- the other device paths on the same batch
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_call(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            ev2.record()
            fn()
            ev3.record()
            torch.cuda.synchronize()
            ts.append(ev2.elapsed_time(ev3))
        return float(np.median(ts))

    g_dev = None
    ms_spatial = time_call(lambda: strom.st_spatial_march(desc, state["rom"], dA, None, d0, g_dev, None))
    ms_certify = time_call(lambda: strom.st_certify(desc, state["rom"], dA, None, d0, b32.coeff, ntd, gamma=gamma))
    ms_fombound = time_call(lambda: strom.st_fom_bound(desc, state["rom"], state["Phi_s"], [c[0] for c in csr], None,
                                                       None, u0, dA, None, d0, b32.coeff, ntd))
    _, _, fb = strom.st_fom_bound(desc, state["rom"], state["Phi_s"], [c[0] for c in csr], None, None, u0, dA, None,
                                  d0, b32.coeff, ntd)
    fb = fb.cpu().numpy()
    print(f"[bench] spatial ROM march {ms_spatial:.2f} ms, certificate {ms_certify:.2f} ms, full-order "
          f"Theorem-3 bound {ms_fombound:.2f} ms", file=sys.stderr, flush=True)

    # the streaming alternative to the offline POD: the same snapshots through the
    # incremental SVD, then its bases against the batch POD's
    isvd = None
    if not args.no_isvd:
        isvd = isvd_stream(strom, Ud, U, prob.N_t, n_mu, n_s, [n_t_max] * n_s, r_max=128, rel_eps=2.5e-11)
        # (the stream keeps only the triplets above its thresholds: its rank can be below n_s, and
        # the vectors near the truncation level are ill-conditioned, so the leading 20 are compared)
        isvd["max_abs_diff_phi_s_1_to_20_vs_batch_pod"] = float((isvd.pop("Phi_s")[:, :20]
                                                                 - state["Phi_s"][:, :20]).abs().max())
        kk = min(isvd["counters"]["rank"], n_s)
        isvd["max_rel_diff_sigma_vs_batch_pod"] = float(((isvd.pop("sigma")[:kk] - state["sigma"][:kk]).abs().max()
                                                         / state["sigma"][0]))
        print(f"[bench] incremental SVD of the {U.shape[1]} snapshots: {isvd['stream_ms']:.1f} ms "
              f"({isvd['us_per_snapshot']:.1f} us/snapshot), rank {isvd['counters']['rank']}", file=sys.stderr,
              flush=True)

    # ------------------------------------------------------------- roofline of the dominant kernel
    lu_ms = ph32["lu"]
    lu_flops = float(np.sum(2.0 / 3.0 * widths.astype(np.float64) ** 3))
    form_ms = ph32["form"]
    form_bytes = float(np.sum(widths.astype(np.float64) ** 2) * 4 + np.sum(widths) * 8)
    lu_tflops = lu_flops / (lu_ms * 1e-3) / 1e12
    form_gbs = form_bytes / (form_ms * 1e-3) / 1e9

    def counter_traffic(fname, src):
        """HBM bytes per launch from the committed byte-counter summary, if the kernel source
        is unchanged since the counters were taken."""
        path = os.path.join(ROOT, "profiles", fname)
        if not os.path.exists(path):
            return None
        with open(path) as f:
            tr = json.load(f)
        return tr.get("bytes_per_launch") if tr.get("source_hash") == source_hash(src) else None

    traffic = counter_traffic("lu_f32_cb4096_traffic.json", "k_lu.hip")
    form_traffic = counter_traffic("form_f32_cb4096_traffic.json", "k_query.hip")

    # ------------------------------------------------------------- CPU baseline (the oracle, bounded sample)
    cpu = None
    accuracy = {"certified": f"info in (0, -6) and st_certify bound <= {CERT_TOL:g}: relative error against the "
                             "exact reduced solution <= e/(1-e), e = ||b - A c|| / (gamma ||c||), "
                             "gamma = 1 - cos(pi/(N_t+1)) <= lambda_min(sym Ahat_st) since sym(A) <= 0",
                "ir_tol": IR_TOL, "gamma": gamma,
                "fp32ir_cert_max": float(np.nanmax(cert32)), "fp64_cert_max": float(np.nanmax(cert64)),
                "fp32ir_vs_fp64_max_rel_diff": d3264,
                "fp32ir_max_relres": float(np.nanmax(relres32)),
                "fp32ir_iters_max": int(iters32.max()),
                "fp64_resolved_queries": int(np.sum(info32 == -6)),
                "full_order_theorem3_bound": {"p50": float(np.median(fb)), "max": float(np.max(fb))}}
    if not args.no_cpu_baseline:
        cpu, sample_err = cpu_baseline(prob, U, n_s, n_t_max, mus, nt, tA, t0_, args.cpu_seconds, state, c32, off)
        accuracy["oracle_sample_max_rel_err_fp32ir"] = sample_err

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 LU + f64 residual/refinement; f64 POD and operators",
        "data": "synthetic (seeded 1-D advection-diffusion snapshots and parameters)",
        "config": {
            "workload": "batched queries: 1-D periodic advection-diffusion, N_s=256, N_t=128, 32 training mu, "
                        "n_s=40, per-mode n_t 8..32, 4096 ragged queries (reduced widths 400..1200)",
            "queries": nq, "n_s": n_s, "n_t_max": n_t_max, "N_s": int(prob.N_s), "N_t": int(prob.N_t),
            "step": "one HIP-graph replay of st_solve over the batch: assembly, FP32 LU, FP64-residual "
                    "refinement (FP64 re-solve of any query that does not converge); offline part separate",
        },
        "roofline": {
            "bound": "mfma", "kernel": "lu_kernel<float> (batched FP32 LU, one launch per step)",
            "achieved": lu_tflops, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": lu_tflops / FP32_PEAK_TFLOPS,
            "traffic": traffic, "algorithmic_flops_per_launch": lu_flops, "avg_launch_ms": lu_ms,
        },
        "assembly": {"kernel": "form_kernel<float>", "bound": "hbm", "achieved": form_gbs, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": form_gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": form_bytes,
                     "avg_launch_ms": form_ms, "traffic": form_traffic},
        "online_median_ms": {"fp32_ir": med32, "fp64": med64},
        "online_qps": {"fp32_ir": ok32 / (med32 * 1e-3), "fp64": ok64 / (med64 * 1e-3)},
        "offline_ms": off_ms,
        "full_step": {"ms": off_ms + med32, "queries_per_s": ok32 / ((off_ms + med32) * 1e-3),
                      "what": "offline (POD + projection + temporal contractions) + one online solve"},
        "breakdown_ms": {"st_solve_phases_fp32": ph32, "st_solve_phases_fp64": ph64},
        "other_paths_ms": {"spatial_rom_march_4096": ms_spatial, "certify_4096": ms_certify,
                           "full_order_bound_4096": ms_fombound},
        "incremental_svd": isvd,
        "lu_autotune": tune,
        "accuracy": accuracy,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


_CPU = {}


def _cpu_worker_init(shared):
    """Pool worker set-up: one BLAS thread, the oracle's offline data kept per worker."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    _CPU.update(shared)


def _cpu_worker(task):
    """One oracle query (assembly by the block formulas + LAPACK gesv), timed."""
    import numpy as np

    from oracle import rom
    ntq, tAq, t0q = task
    d = _CPU
    t1 = time.perf_counter()
    Pt = [d["Phi_t"][i][:, :ntq[i]] for i in range(len(ntq))]
    M, b = rom.reduced_system(d["Ahat"], tAq, np.zeros((d["u0hat"].shape[0], 0)), np.zeros(0), d["g"], d["u0hat"],
                              t0q, Pt, d["dt"])
    c = rom.solve(M, b)
    return time.perf_counter() - t1, c


def cpu_baseline(prob, U, n_s, n_t_max, mus, nt, tA, t0_, budget_s, state, c32, off):
    """Time the oracle (CPU, FP64) on a bounded sample of the same workload: its
    offline phase once, one query on one core (the paper's online solves ran on one
    core), then a process pool with one BLAS thread per worker over the cores until
    the budget is spent; the pool's rate is extrapolated to the 4096-query batch.
    The sample also checks the device solutions: the oracle's reconstructed
    space-time trajectories against the device's."""
    import multiprocessing as mp
    import platform

    import numpy as np

    from oracle import pod, rom

    nproc = os.cpu_count() or 1
    workers = max(1, min(16, nproc))
    cpu_model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    t0 = time.perf_counter()
    Phi_s, s, V = pod.pod(U, n_s)
    Phi_t, _ = pod.temporal_bases(V, prob.N_t, len(prob.train_mu), np.full(n_s, n_t_max))
    Ahat = [rom.spatial_operator(Phi_s, A) for A in prob.terms]
    u0hat = rom.reduced_vector(Phi_s, prob.u0)
    t_off = time.perf_counter() - t0
    nq = len(mus)
    rng = np.random.default_rng(5)
    order = rng.permutation(nq)

    shared = {"Ahat": Ahat, "Phi_t": Phi_t, "u0hat": u0hat, "g": prob.g, "dt": prob.dt}

    def task(q):
        return (nt[q].copy(), tA[q], t0_[q])

    # one core
    _cpu_worker_init(shared)
    t1q, _ = _cpu_worker(task(int(order[0])))
    # the pool (fresh interpreters: the workers never touch the GPU)
    ctx = mp.get_context("spawn")
    done, results = 0, []
    pool = ctx.Pool(workers, initializer=_cpu_worker_init, initargs=(shared,))
    pool.map(_cpu_worker, [task(int(order[0]))] * workers)     # workers started and warm
    t_pool0 = time.perf_counter()
    with pool:
        while time.perf_counter() - t_pool0 < budget_s and done < nq:
            batch = [int(q) for q in order[done:done + 4 * workers]]
            res = pool.map(_cpu_worker, [task(q) for q in batch])
            results += list(zip(batch, res))
            done += len(batch)
    t_pool = time.perf_counter() - t_pool0
    rate = nq / (t_off + nq * t_pool / done)
    Phi_s_d = state["Phi_s"].cpu().numpy()
    Pt_d = state["Phi_t"].cpu().numpy()
    worst = 0.0
    for q, (_, c) in results[:64]:
        Pt = [Phi_t[i][:, :nt[q, i]] for i in range(n_s)]
        ref = rom.reconstruct(Phi_s, Pt, c)
        Ptd = [Pt_d[:, i * n_t_max: i * n_t_max + nt[q, i]] for i in range(n_s)]
        got = rom.reconstruct(Phi_s_d, Ptd, c32[off[q]:off[q + 1]])
        worst = max(worst, float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    print(f"[bench] cpu oracle: offline {t_off:.2f}s, 1 core {1e3 * t1q:.1f} ms/query, pool of {workers} "
          f"(1 BLAS thread each): {done} queries in {t_pool:.1f}s; sample max rel err (trajectories) {worst:.2e}",
          file=sys.stderr, flush=True)
    return ({"value": rate, "unit": "queries/s", "cores": workers, "kind": "oracle",
             "sample": f"oracle POD once ({t_off:.2f} s) + {done} of {nq} queries on a pool of {workers} processes "
                       f"with one BLAS thread each ({t_pool:.1f} s); rate extrapolated to the {nq}-query batch",
             "single_core_ms_per_query": 1e3 * t1q, "nproc": nproc, "cpu_model": cpu_model}, worst)


def isvd_stream(strom, Ud, U, N_t, n_mu, n_s, n_t, r_max, rel_eps, reps=2):
    """Streams the snapshot columns through st_isvd_update (one call, timed with HIP
    events on the current stream; the last of `reps` runs is kept), then takes the
    bases with st_isvd_bases.  Thresholds eps_svd = eps_sv = rel_eps times the largest
    snapshot norm."""
    import numpy as np
    import torch

    sc = float(np.linalg.norm(U, axis=0).max())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(reps):
        inc = strom.IncrementalSVD(U.shape[0], r_max, U.shape[1], rel_eps * sc, rel_eps * sc)
        torch.cuda.synchronize()
        e0.record()
        inc.update(Ud)
        e1.record()
        torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    e0.record()
    Phi_s, Phi_t, sigma, rank = inc.bases(N_t, n_mu, n_s, n_t)
    e1.record()
    torch.cuda.synchronize()
    return {"snapshots": int(U.shape[1]), "N_s": int(U.shape[0]), "r_max": r_max,
            "eps_svd_rel": rel_eps, "eps_sv_rel": rel_eps, "stream_ms": ms,
            "us_per_snapshot": 1e3 * ms / U.shape[1], "bases_ms": e0.elapsed_time(e1),
            "counters": inc.counters(), "Phi_s": Phi_s, "sigma": sigma}


def bench_isvd(args):
    """Incremental SVD (Sec. 4.2, Alg. 1-2) of the 2-D transport snapshots: 8 training
    parameters x 200 steps of N_s = 49152 (64^2 cells x 12 directions), streamed in
    time order through st_isvd_update with r_max = 128 and eps_svd = eps_sv = 1e-6 of
    the largest snapshot norm.  `value` is snapshots per second of the whole stream
    (inputs resident in HBM).  The HBM roofline is taken over the whole stream: the
    bytes a step must move at the least with two Gram-Schmidt passes (W read three
    times and written once, the snapshot and residual vectors, V read and written)
    summed with each step's actual rank, over the stream's time."""
    import numpy as np
    import torch

    from paper_1910_01260_amd import strom
    from paper_1910_01260_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    strom.lib()
    log = lambda m: print(f"[isvd] {m}", file=sys.stderr, flush=True)
    t0 = time.time()
    prob = W.transport2d()
    U = W.snapshots(prob)
    log(f"snapshots {U.shape} in {time.time() - t0:.1f}s")
    Ud = torch.tensor(np.ascontiguousarray(U.T), device="cuda").T
    n_s, n_t = 40, 20
    res = isvd_stream(strom, Ud, U, prob.N_t, len(prob.train_mu), n_s, [n_t] * n_s, r_max=128, rel_eps=1e-6,
                      reps=max(2, args.warmup + 1))
    res.pop("Phi_s")
    sig = res.pop("sigma").cpu().numpy()
    # per-step ranks (an untimed replay of the same stream, one snapshot per call)
    sc = float(np.linalg.norm(U, axis=0).max())
    inc = strom.IncrementalSVD(U.shape[0], 128, U.shape[1], 1e-6 * sc, 1e-6 * sc)
    ranks = []
    for c in range(U.shape[1]):
        r_before = int(inc.state[0].item())
        inc.update(Ud[:, c])
        ranks.append((r_before, int(inc.state[0].item())))
    N_s = U.shape[0]
    step_bytes = [8.0 * (4 * N_s * rb + N_s * ra + 6 * N_s + (k + 1) * (rb + ra)) for k, (rb, ra) in enumerate(ranks)]
    total_bytes = float(np.sum(step_bytes))
    gbs = total_bytes / (res["stream_ms"] * 1e-3) / 1e9
    sb = np.sqrt(np.maximum(np.linalg.eigvalsh(U.T @ U)[::-1][:n_s], 0.0))
    out = {
        "metric": "incremental SVD snapshots/s (Sec. 4.2, Alg. 1-2)",
        "value": U.shape[1] / (res["stream_ms"] * 1e-3),
        "unit": "snapshots/s",
        "n_gpus": 1,
        "steps": U.shape[1],
        "warmup": args.warmup,
        "ms_per_step": res["stream_ms"] / U.shape[1],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded 2-D transport snapshots)",
        "config": {"workload": "incremental SVD: 2-D discrete-ordinates transport, 64x64 cells x 12 directions "
                               "(N_s=49152), 8 training mu x 200 steps streamed in time order, r_max=128, "
                               "eps_svd=eps_sv=1e-6 x max snapshot norm",
                   "step": "one snapshot through st_isvd_update (9 launches, no host synchronisation)"},
        "roofline": {"bound": "hbm", "kernel": "whole stream (dots, sub1, sub2, apply_w, apply_v and the "
                                               "one-workgroup reductions, bordered SVD and commit)",
                     "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes": total_bytes},
        "isvd": res,
        "accuracy": {"sigma_1_to_40_max_rel_diff_vs_batch_gram": float(np.max(np.abs(sig - sb)) / sb[0])},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the oracle's stream (oracle.isvd, NumPy/LAPACK) on the first parameter's snapshots
        from oracle import isvd as oisvd
        m_cpu = 200
        t1 = time.perf_counter()
        oisvd.incremental_svd(U[:, :m_cpu], 1e-6 * sc, 1e-6 * sc, r_max=128)
        dt_cpu = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": m_cpu / dt_cpu, "unit": "snapshots/s", "cores": os.cpu_count(),
                               "kind": "oracle",
                               "sample": f"the first {m_cpu} snapshots (one parameter's trajectory) through "
                                         "oracle.isvd.incremental_svd; cores = the host's CPUs available to "
                                         "its BLAS"}
    print(json.dumps(out))


def bench_c4(args):
    """Precision at scale: 3-D periodic advection-diffusion on 128^3 cells (N_s = 2,097,152),
    16 training parameters x 500 steps = 8000 snapshots generated on the GPU and kept there in
    FP32 (67 GB); the 8000 x 8000 snapshot Gram in FP64, FP32 and split-BF16 (errors against
    FP64 and the MFMA roofline of each); the POD (n_s = 100) from each Gram; the ROM with 30
    temporal vectors per mode (n = 3000) assembled and a batch of queries solved with the FP64 LU
    and the FP32 LU + FP64 refinement.  `value` = certified (<= 1e-6) queries/s of the FP32+IR
    solve on that batch; the dominant kernel is the FP64 Gram."""
    import numpy as np
    import torch

    from paper_1910_01260_amd import strom
    from paper_1910_01260_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    strom.lib()
    log = lambda m: print(f"[c4] {m}", file=sys.stderr, flush=True)
    N3, NT, NMU, NS, NTM = 128, 500, 16, 100, 30
    # 256 queries: at n = 3000 the LU runs one query per workgroup of 512 threads, one workgroup
    # per CU, so 256 queries occupy every CU once (128 would leave half of them idle)
    nq = min(args.queries, 256)
    prob = W.advdiff3d(n=N3, N_t=NT, n_train=NMU)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        ev0.record()
        r = fn()
        ev1.record()
        torch.cuda.synchronize()
        return r, ev0.elapsed_time(ev1)

    U, gen_ms = timed(lambda: W.periodic_snapshots_device(prob, N3))
    K, m = U.shape
    log(f"snapshots {tuple(U.shape)} FP32 generated in {gen_ms:.0f} ms")
    gram_flops = float(K) * m * (m + 1)  # the lower triangle: m(m+1)/2 entries of 2K flops
    peaks = {strom.ST_F64: FP64_PEAK_TFLOPS, strom.ST_F32: FP32_PEAK_TFLOPS, strom.ST_BF16X3: 2500.0 / 3.0}
    names = {strom.ST_F64: "f64", strom.ST_F32: "f32", strom.ST_BF16X3: "bf16x3"}
    grams, G64 = {}, None
    for prec in (strom.ST_F64, strom.ST_F32, strom.ST_BF16X3):
        strom.st_gram(U, prec)  # warm
        G, ms = timed(lambda: strom.st_gram(U, prec))
        tf = gram_flops / (ms * 1e-3) / 1e12
        grams[names[prec]] = {"ms": ms, "tflops": tf, "peak_tflops": peaks[prec], "frac": tf / peaks[prec]}
        if prec == strom.ST_F64:
            G64 = G
        else:
            grams[names[prec]]["max_abs_err_rel_to_max_f64"] = float((G - G64).abs().max() / G64.abs().max())
        del G
        log(f"Gram {names[prec]}: {ms:.0f} ms, {tf:.1f} TFLOP/s")
    del G64
    pods, bases = {}, None
    for prec in (strom.ST_F64, strom.ST_F32, strom.ST_BF16X3):
        (Phi_s, Phi_t, sig, rank), ms = timed(lambda: strom.st_build_bases(U, NT, NMU, NS, [NTM] * NS,
                                                                            gram_prec=prec))
        pods[names[prec]] = {"ms": ms, "sigma": sig.cpu().numpy()}
        if prec == strom.ST_F64:
            bases = (Phi_s, Phi_t)
        log(f"POD {names[prec]}: {ms:.0f} ms")
    s64 = pods["f64"]["sigma"]
    for k in ("f32", "bf16x3"):
        d = np.abs(pods[k].pop("sigma") - s64) / s64[0]
        pods[k]["max_rel_sigma_diff_vs_f64_modes_1_20"] = float(d[:20].max())
        pods[k]["max_rel_sigma_diff_vs_f64_all"] = float(d.max())
    pods["f64"].pop("sigma")
    del U
    torch.cuda.empty_cache()
    Phi_s, Phi_t = bases
    desc = strom.RomDesc([NTM] * NS, NT, prob.Q, prob.Qf, prob.Q0)
    csr = [strom.csr_to_device(*W.csr_arrays(A)) for A in prob.terms]
    dt = torch.tensor(prob.dt, device="cuda")
    u0 = torch.tensor(np.ascontiguousarray(prob.u0.T), device="cuda").T
    romb, asm_ms = timed(lambda: strom.st_assemble(desc, Phi_s, Phi_t, dt, [c[0] for c in csr], None, None, u0))
    mus = W.sample_params(prob, nq)
    tA, tf_, t0 = prob.thetas(mus)
    nt = np.full((nq, NS), NTM, dtype=np.int32)
    dA, d0, ntd = (torch.tensor(tA, device="cuda"), torch.tensor(t0, device="cuda"), torch.tensor(nt, device="cuda"))
    widths = nt.astype(np.int64).sum(axis=1)
    b32 = strom.SolveBuffers(desc, nq, widths, strom.ST_F32, "cuda")
    b64 = strom.SolveBuffers(desc, nq, widths, strom.ST_F64, "cuda")
    solve = lambda prec, bufs: strom.st_solve(desc, romb, dA, None, d0, ntd, lu_prec=prec,
                                              ir_tol=IR_TOL if prec == strom.ST_F32 else 0.0,
                                              ir_max=IR_MAX if prec == strom.ST_F32 else 0, bufs=bufs)
    tune = {}
    for name, prec, bufs in (("fp32", strom.ST_F32, b32), ("fp64", strom.ST_F64, b64)):
        choice, ms = strom.st_autotune(desc, romb, dA, None, d0, ntd, prec, bufs=bufs)
        tune[name] = {"choice": choice, "lu_ms_per_variant": ms}
    for _ in range(max(1, args.warmup)):
        solve(strom.ST_F32, b32)
        solve(strom.ST_F64, b64)
    torch.cuda.synchronize()
    ms32 = float(np.median([timed(lambda: solve(strom.ST_F32, b32))[1] for _ in range(max(1, args.steps // 2))]))
    ms64 = float(np.median([timed(lambda: solve(strom.ST_F64, b64))[1] for _ in range(max(1, args.steps // 2))]))
    gamma = strom.st_coercivity_floor(NT)
    _, cert32 = strom.st_certify(desc, romb, dA, None, d0, b32.coeff, ntd, gamma=gamma)
    torch.cuda.synchronize()
    info32 = b32.info.cpu().numpy()[:nq]
    ok32 = int(np.sum(np.isin(info32, (0, -6)) & (cert32.cpu().numpy() <= CERT_TOL)))
    c32, c64, off = b32.coeff.cpu().numpy(), b64.coeff.cpu().numpy(), b32.coeff_off.cpu().numpy()
    d3264 = max(float(np.linalg.norm(c32[off[q]:off[q + 1]] - c64[off[q]:off[q + 1]])
                      / np.linalg.norm(c64[off[q]:off[q + 1]])) for q in range(nq))
    lu_flops = nq * 2.0 / 3.0 * float(NS * NTM) ** 3
    g = grams["f64"]
    out = {
        "metric": "ST-ROM queries/sec at n = 3000 (FP32 LU + FP64 refinement) at rel err<=1e-6; Gram MFMA %",
        "value": ok32 / (ms32 * 1e-3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": max(1, args.steps // 2),
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 snapshots; Gram f64/f32/bf16x3; f32 LU + f64 refinement",
        "data": "synthetic (3-D advection-diffusion snapshots generated on the GPU)",
        "config": {"workload": "precision at scale: 3-D periodic advection-diffusion 128^3 (N_s=2097152), "
                               "7-point stencil CSR, N_t=500, 16 training mu (8000 FP32 snapshots), n_s=100, "
                               f"n_t=30 (n=3000), {nq} queries",
                   "step": "one st_solve over the batch (FP32 LU + FP64 refinement)"},
        "roofline": {"bound": "mfma", "kernel": "gram_f64_kernel (8000 x 8000 snapshot Gram, FP64 MFMA)",
                     "achieved": g["tflops"], "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": g["frac"], "traffic": None, "algorithmic_flops_per_launch": gram_flops,
                     "avg_launch_ms": g["ms"]},
        "generator_ms": gen_ms,
        "gram": grams,
        "pod": pods,
        "assemble_ms": asm_ms,
        "lu_autotune": tune,
        "solve": {"fp32_ir_ms": ms32, "fp64_ms": ms64, "certified_fp32_ir": ok32, "queries": nq,
                  "lu_tflops_fp32_ir": lu_flops / (ms32 * 1e-3) / 1e12,
                  "fp32ir_vs_fp64_max_rel_diff": d3264},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import rom as orom
        P = Phi_s.cpu().numpy()
        Pt_all = Phi_t.cpu().numpy()
        Pt = [Pt_all[:, i * NTM:(i + 1) * NTM] for i in range(NS)]
        t1 = time.perf_counter()
        Ahat = [orom.spatial_operator(P, A) for A in prob.terms]
        u0hat = orom.reduced_vector(P, prob.u0)
        t_off = time.perf_counter() - t1
        t1 = time.perf_counter()
        M, b = orom.reduced_system(Ahat, tA[0], np.zeros((NS, 0)), tf_[0], prob.g, u0hat, t0[0], Pt, prob.dt)
        c = np.linalg.solve(M, b)
        dt_q = time.perf_counter() - t1
        err = float(np.linalg.norm(c32[off[0]:off[1]] - c) / np.linalg.norm(c))
        out["cpu_baseline"] = {"value": 1.0 / dt_q, "unit": "queries/s", "cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"one query's 3000-wide reduced system assembled by the oracle's block "
                                         f"formulas and solved by LAPACK ({dt_q:.2f} s; the projection of the "
                                         f"operators, {t_off:.1f} s, not counted); its solution agrees with the "
                                         f"device's FP32+IR to {err:.1e}"}
    print(json.dumps(out))


def bench_c2(args):
    """Plain FP64 ST-ROM of the 2-D discrete-ordinates transport problem at its stated size:
    64^2 cells x 12 directions (N_s = 49152), N_t = 200, 8 training parameters (4 total cross
    sections x 2 scattering ratios), n_s = 40 spatial modes x n_t = 20 temporal vectors (n = 800).
    Offline: st_build_bases + st_assemble.  Online: `--queries` parameters drawn in the box,
    solved with the FP64 LU (the configuration's arithmetic; `value` = its certified <= 1e-6
    queries/s) and, beside it, with the FP32 LU + FP64 refinement."""
    import numpy as np
    import torch

    from paper_1910_01260_amd import strom
    from paper_1910_01260_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    strom.lib()
    log = lambda m: print(f"[c2] {m}", file=sys.stderr, flush=True)
    t0 = time.time()
    prob = W.transport2d()
    n_s, n_t = 40, 20
    U = W.snapshots(prob)
    log(f"snapshots {U.shape} in {time.time() - t0:.1f}s")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        ev0.record()
        r = fn()
        ev1.record()
        torch.cuda.synchronize()
        return r, ev0.elapsed_time(ev1)

    Ud = torch.tensor(np.ascontiguousarray(U.T), device="cuda").T
    desc = strom.RomDesc([n_t] * n_s, prob.N_t, prob.Q, prob.Qf, prob.Q0)
    csr = [strom.csr_to_device(*W.csr_arrays(A)) for A in prob.terms]
    dt = torch.tensor(prob.dt, device="cuda")
    Bf = torch.tensor(np.ascontiguousarray(prob.Bf.T), device="cuda").T if prob.Qf else None
    g = torch.tensor(np.ascontiguousarray(prob.g.T), device="cuda").T if prob.Qf else None
    u0 = torch.tensor(np.ascontiguousarray(prob.u0.T), device="cuda").T if prob.Q0 else None

    def offline():
        Phi_s, Phi_t, sigma, rank = strom.st_build_bases(Ud, prob.N_t, len(prob.train_mu), n_s, [n_t] * n_s)
        return Phi_s, Phi_t, strom.st_assemble(desc, Phi_s, Phi_t, dt, [c[0] for c in csr], Bf, g, u0)

    offline()
    (Phi_s, Phi_t, romb), off_ms = timed(offline)
    nq = args.queries
    mus = W.sample_params(prob, nq)
    tA, tf, t0_ = prob.thetas(mus)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), device="cuda") if a.shape[1] else None
    dA, dF, d0 = dev(tA), dev(tf), dev(t0_)
    nt = np.full((nq, n_s), n_t, dtype=np.int32)
    ntd = torch.tensor(nt, device="cuda")
    widths = nt.astype(np.int64).sum(axis=1)
    b64 = strom.SolveBuffers(desc, nq, widths, strom.ST_F64, "cuda")
    b32 = strom.SolveBuffers(desc, nq, widths, strom.ST_F32, "cuda")
    solve = lambda prec, bufs: strom.st_solve(desc, romb, dA, dF, d0, ntd, lu_prec=prec,
                                              ir_tol=IR_TOL if prec == strom.ST_F32 else 0.0,
                                              ir_max=IR_MAX if prec == strom.ST_F32 else 0, bufs=bufs)
    tune = {}
    for name, prec, bufs in (("fp64", strom.ST_F64, b64), ("fp32", strom.ST_F32, b32)):
        choice, ms = strom.st_autotune(desc, romb, dA, dF, d0, ntd, prec, bufs=bufs)
        tune[name] = {"choice": choice, "lu_ms_per_variant": ms}
    log(f"LU autotune: {json.dumps(tune)}")
    strom.st_graph_enable(True)
    for _ in range(max(1, args.warmup)):
        solve(strom.ST_F64, b64)
        solve(strom.ST_F32, b32)
    torch.cuda.synchronize()
    K = args.steps
    ms64 = float(np.median([timed(lambda: solve(strom.ST_F64, b64))[1] for _ in range(K)]))
    ms32 = float(np.median([timed(lambda: solve(strom.ST_F32, b32))[1] for _ in range(K)]))
    strom.st_graph_enable(False)
    strom.st_graph_reset()
    strom.st_timing_enable(True)
    solve(strom.ST_F64, b64)
    torch.cuda.synchronize()
    ph64 = strom.st_timing_read()
    strom.st_timing_enable(False)
    gamma = strom.st_coercivity_floor(prob.N_t)
    _, cert64 = strom.st_certify(desc, romb, dA, dF, d0, b64.coeff, ntd, gamma=gamma)
    _, cert32 = strom.st_certify(desc, romb, dA, dF, d0, b32.coeff, ntd, gamma=gamma)
    torch.cuda.synchronize()
    info64, info32 = b64.info.cpu().numpy()[:nq], b32.info.cpu().numpy()[:nq]
    ok64 = int(np.sum((info64 == 0) & (cert64.cpu().numpy() <= CERT_TOL)))
    ok32 = int(np.sum(np.isin(info32, (0, -6)) & (cert32.cpu().numpy() <= CERT_TOL)))
    lu_flops = float(np.sum(2.0 / 3.0 * widths.astype(np.float64) ** 3))
    lu_tf = lu_flops / (ph64["lu"] * 1e-3) / 1e12
    out = {
        "metric": "ST-ROM queries/sec, plain FP64 (2-D transport, n = 800) at rel err<=1e-6",
        "value": ok64 / (ms64 * 1e-3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded 2-D transport snapshots and parameters)",
        "config": {"workload": "plain ST-ROM, FP64: 2-D discrete-ordinates transport 64x64 x 12 directions "
                               "(N_s=49152), N_t=200, 8 training mu, n_s=40, n_t=20 (n=800), "
                               f"{nq} queries", "step": "one HIP-graph replay of st_solve (FP64 LU)"},
        "roofline": {"bound": "mfma", "kernel": "lu_kernel<double> (batched FP64 LU)", "achieved": lu_tf,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": lu_tf / FP64_PEAK_TFLOPS, "traffic": None,
                     "algorithmic_flops_per_launch": lu_flops, "avg_launch_ms": ph64["lu"]},
        "offline_ms": off_ms,
        "lu_autotune": tune,
        "fp64_phases_ms": ph64,
        "fp32_ir": {"ms": ms32, "certified": ok32, "queries_per_s": ok32 / (ms32 * 1e-3)},
        "certified_fp64": ok64,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        from oracle import rom as orom
        P, Pt_all = Phi_s.cpu().numpy(), Phi_t.cpu().numpy()
        Pt = [Pt_all[:, i * n_t:(i + 1) * n_t] for i in range(n_s)]
        Ahat = [orom.spatial_operator(P, A) for A in prob.terms]
        bhat = orom.reduced_vector(P, prob.Bf) if prob.Qf else np.zeros((n_s, 0))
        u0hat = orom.reduced_vector(P, prob.u0) if prob.Q0 else np.zeros((n_s, 0))
        c64, off = b64.coeff.cpu().numpy(), b64.coeff_off.cpu().numpy()
        n_cpu, worst = 8, 0.0
        t1 = time.perf_counter()
        for q in range(n_cpu):
            M, b = orom.reduced_system(Ahat, tA[q], bhat, tf[q], prob.g, u0hat, t0_[q], Pt, prob.dt)
            c = np.linalg.solve(M, b)
            worst = max(worst, float(np.linalg.norm(c64[off[q]:off[q + 1]] - c) / np.linalg.norm(c)))
        dt_q = (time.perf_counter() - t1) / n_cpu
        out["cpu_baseline"] = {"value": 1.0 / dt_q, "unit": "queries/s", "cores": os.cpu_count(), "kind": "oracle",
                               "sample": f"{n_cpu} queries assembled by the oracle's block formulas and solved by "
                                         f"LAPACK in one process (the projection of the operators not counted); "
                                         f"their solutions agree with the device's FP64 path to {worst:.1e}"}
    print(json.dumps(out))


def bench_surrogate(args):
    """Learned surrogate on the transport-with-absorber ROM (64^2 cells, 12 directions,
    N_t = 200, n_s = 40 modes x 30 temporal vectors = 1200 coefficients, 3 parameters).

    Training data are batched FP64 solves at seeded parameters; the network
    (3 -> 4 x 512 GELU -> 1200) is trained by the library's BF16 kernels.  A fresh
    4096-query batch is then answered (a) by the batched solve alone and (b) by the
    network + FP64 residual certificate, with the rejected queries re-solved, for
    several certificate tolerances."""
    import numpy as np
    import torch

    from paper_1910_01260_amd import strom
    from paper_1910_01260_amd import surrogate as S
    from paper_1910_01260_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    strom.lib()
    dev = "cuda"
    log = lambda m: print(f"[surrogate] {m}", file=sys.stderr, flush=True)
    t0 = time.time()
    prob = W.transport2d_absorber()
    n_s, n_t = 40, 30
    U = W.snapshots(prob)
    log(f"snapshots {U.shape} in {time.time() - t0:.1f}s")
    Ud = torch.tensor(np.ascontiguousarray(U.T), device=dev).T
    Phi_s, Phi_t, sigma, rank = strom.st_build_bases(Ud, prob.N_t, len(prob.train_mu), n_s, [n_t] * n_s)
    desc = strom.RomDesc([n_t] * n_s, prob.N_t, prob.Q, prob.Qf, prob.Q0)
    csr = [strom.csr_to_device(*W.csr_arrays(A)) for A in prob.terms]
    cm = lambda a: torch.tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T), device=dev).T
    rom = strom.st_assemble(desc, Phi_s, Phi_t, torch.tensor(prob.dt, device=dev), [c[0] for c in csr],
                            cm(prob.Bf), cm(prob.g), None)
    torch.cuda.synchronize()
    del Ud
    n = desc.n
    gamma = S.coercivity_floor(prob.N_t)

    def thetas(mus):
        tA, tf, t0_ = prob.thetas(mus)
        dv = lambda a: torch.tensor(np.ascontiguousarray(a), device=dev) if a.shape[1] else None
        return dv(tA), dv(tf), dv(t0_)

    # ---- training data: batched FP64 solves
    n_train = args.surrogate_train
    mus_tr = W.sample_params(prob, n_train, seed=191001261)
    C = np.empty((n_train, n))
    chunk = 2048
    bufs = strom.SolveBuffers(desc, chunk, np.full(chunk, n), strom.ST_F64, dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for a in range(0, n_train, chunk):
        b = min(n_train, a + chunk)
        dA, df, d0 = thetas(mus_tr[a:b])
        if b - a < chunk:
            bufs = strom.SolveBuffers(desc, b - a, np.full(b - a, n), strom.ST_F64, dev)
        strom.st_solve(desc, rom, dA, df, d0, None, strom.ST_F64, bufs=bufs)
        C[a:b] = bufs.coeff[: (b - a) * n].view(b - a, n).cpu().numpy()
    data_s = time.perf_counter() - t1
    del bufs
    log(f"{n_train} training solves in {data_s:.2f}s")

    # ---- training
    X = S.scaled_inputs(prob.box_lo, prob.box_hi, mus_tr)
    net = S.Surrogate(X.shape[1], n, width=512, n_hidden=4, seed=191001263)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    hist = net.fit(X, C, steps=args.surrogate_steps, batch=1024, lr=1e-3, lr_final=1e-5, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t2
    log(f"trained {args.surrogate_steps} steps in {train_s:.1f}s; final val loss {hist[-1][2]:.3e}")

    # ---- test batch
    nq = args.queries
    mus = W.sample_params(prob, nq, seed=191001265)
    dA, df, d0 = thetas(mus)
    Xt = torch.tensor(S.scaled_inputs(prob.box_lo, prob.box_hi, mus), device=dev)
    widths = np.full(nq, n)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            ev[0].record()
            fn()
            ev[1].record()
            torch.cuda.synchronize()
            ts.append(ev[0].elapsed_time(ev[1]))
        return float(np.median(ts))

    b64 = strom.SolveBuffers(desc, nq, widths, strom.ST_F64, dev)
    b32 = strom.SolveBuffers(desc, nq, widths, strom.ST_F32, dev)
    ms64 = timed(lambda: strom.st_solve(desc, rom, dA, df, d0, None, strom.ST_F64, bufs=b64))
    ms32 = timed(lambda: strom.st_solve(desc, rom, dA, df, d0, None, strom.ST_F32, 1e-12, 6, bufs=b32))
    ref = b64.coeff.cpu().numpy().reshape(nq, n)
    ok32 = int(np.sum((b32.info.cpu().numpy()[:nq] == 0) & (b32.relres.cpu().numpy()[:nq] <= 1e-12)))
    ms_pred = timed(lambda: net.predict(Xt))
    Y = net.predict(Xt)
    coeff = torch.empty(nq * n, dtype=torch.float64, device=dev)
    ms_check = timed(lambda: net.check(desc, rom, dA, df, d0, Y, gamma, 0.0, coeff))
    cert, acc = net.check(desc, rom, dA, df, d0, Y, gamma, 0.0, coeff)
    torch.cuda.synchronize()
    pred = coeff.cpu().numpy().reshape(nq, n)
    rel = np.linalg.norm(pred - ref, axis=1) / np.linalg.norm(ref, axis=1)
    certs = cert.cpu().numpy()
    sound = bool(np.all(rel <= certs * (1 + 1e-9) + 1e-15))
    tols = [1e-6, 1e-4, 1e-2, 1e-1, 1.0]
    rows = []
    for tol in tols:
        bs = strom.SolveBuffers(desc, nq, widths, strom.ST_F32, dev)

        def run(tol=tol, bs=bs):
            net.solve(desc, rom, dA, df, d0, Xt, gamma, tol, bs, strom.ST_F32, 1e-12, 6)

        ms = timed(run)
        acc_t = int(np.sum(certs <= tol))
        rows.append({"tol": tol, "accepted": acc_t, "ms": ms, "queries_per_s": nq / (ms * 1e-3),
                     "vs_batched_fp32ir": ms32 / ms})
        log(f"tol {tol:g}: accepted {acc_t}/{nq}, {ms:.2f} ms ({ms32 / ms:.2f}x the batched FP32+IR solve)")
        del bs
    out = {
        "metric": "surrogate-with-fallback ST-ROM queries/s at certified rel err <= tol",
        "workload": "2-D transport with central absorber, 64^2 x 12 directions, N_t=200, 3 parameters, "
                    "n_s=40 x n_t=30 = 1200 coefficients; MLP 3->4x512->1200 (GELU, BF16 products)",
        "data": "synthetic (seeded)", "n_gpus": 1,
        "train": {"queries": n_train, "solve_s": data_s, "steps": args.surrogate_steps, "batch": 1024,
                  "train_s": train_s, "ms_per_step": 1e3 * train_s / max(1, args.surrogate_steps),
                  "val_loss_first": hist[0][2], "val_loss_last": hist[-1][2]},
        "test_queries": nq,
        "batched_fp64_ms": ms64, "batched_fp32ir_ms": ms32, "batched_fp32ir_certified": ok32,
        "batched_fp32ir_queries_per_s": ok32 / (ms32 * 1e-3),
        "predict_ms": ms_pred, "certificate_ms": ms_check,
        "prediction_rel_err": {"p50": float(np.median(rel)), "p90": float(np.quantile(rel, 0.9)),
                               "max": float(rel.max())},
        "certificate": {"gamma": gamma, "p50": float(np.median(certs)), "finite": int(np.isfinite(certs).sum()),
                        "bounds_true_error": sound},
        "by_tolerance": rows,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
