#!/usr/bin/env python3
"""Benchmark of the batched spectral point-mass filter on one MI355X.

Workload (the batched configuration the throughput target is quoted on):
4096 independent 2-D filters, each with its own seeded A (real eigenvalues in
[-1, 0]) and Q (diagonal in [0.05, 1]), grid N x N with N drawn uniformly from
{32, 48, 64, 96, 128}, linear-Gaussian measurements, exact integrator, FP32
densities with FP64 reductions; one step = predict(T = 0.05) + update(z) of every
filter = a planning kernel and one fused launch (a workgroup per group of same-size
filters).

Prints ONE JSON line.  `value` = grid points carried through one full cycle per
second (whole job, inputs resident in HBM).  Also reported: the fused kernel's
duration from HIP events and its HBM roofline fraction, the CPU oracle on the
host cores, p50/p99 step latency, the L1 error of sampled filters against the
FP64 oracle, and the plain single-filter FP64 GPU path.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-point FPE updates/sec at stated L1 error vs FP64; p50/p99 update latency"
HBM_PEAK_GBS = 8000.0
HBM_TARGET_FRAC = 0.60
# FP32 vector arithmetic without packed instructions (the build disables them):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) per clock at 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def fused_flops_per_point(n: int) -> float:
    """Algorithmic FP32 flops of one fused cycle per grid point of an n x n filter:
    real 2-D FFT forward + inverse 5 log2(n^2) (the standard 2.5 m log2 m per real
    transform of m points), spectral gain 4, likelihood 6, moment sums 5, cubic
    Lagrange regrid 62 (2 coordinates, 2 x 10 for the weights, 16 + 4 FMAs),
    renormalising sum 1."""
    return 10.0 * math.log2(n) + 78.0
# VALU issue: 256 CUs x 4 SIMDs x 16 lanes per clock (a wave64 instruction every
# 4 clocks per SIMD; packed FP32 is not used) at 2.4 GHz
VALU_PEAK_LANE_INSTR = 256 * 64 * 2.4e9
BYTES_PER_POINT = 8            # FP32 density read once + written once per cycle
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_batch_4096_traffic.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# sources the fused batched kernel is compiled from: a traffic figure measured on
# another version of them is stale and not reported
FUSED_SOURCES = ("paper_2412_07240_amd/csrc/batch.hip", "paper_2412_07240_amd/csrc/api_internal.h",
                 "paper_2412_07240_amd/csrc/pmf_internal.h", "include/pmf.h")


def source_hash() -> str:
    h = hashlib.sha256()
    for f in FUSED_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# ------------------------------------------------------------------ CPU baseline

def _cpu_worker(args):
    idxs, budget, nfilters = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        import oracle
        import workloads as W
        pts, busy = 0, 0.0
        t_end = time.perf_counter() + budget
        for i in idxs:
            if time.perf_counter() > t_end:
                break
            sc = W.batched_filter(i, K=1)
            m = sc.model.with_(precision=W.FP64)
            st = oracle.create(m, sc.prior)
            t0 = time.perf_counter()
            st, _ = oracle.predict(m, st, sc.T)
            oracle.update(m, st, sc.z[0])
            busy += time.perf_counter() - t0
            pts += m.N[0] * m.N[1]
        return pts, busy


def cpu_baseline(seconds: float, nfilters: int):
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16)
    per = [list(range(w, nfilters, cores)) for w in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(p, seconds, nfilters) for p in per])
    wall = time.perf_counter() - t0
    pts = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": pts / busy if busy > 0 else None, "unit": "grid-point updates/s", "cores": cores,
            "kind": "oracle", "host_cpu": model, "nproc": os.cpu_count(),
            "sample": f"FP64 oracle predict+update cycles of the batched workload's filters "
                      f"(same N mix), {cores} processes x 1 BLAS thread, ~{seconds:.0f} s each; "
                      f"{pts} points in {busy:.1f} s busy ({wall:.1f} s wall incl. start-up)"}


# ------------------------------------------------------------------ main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--filters", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip latency / L1 / plain-path legs")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched: keep the default fused schedules instead of timing the variants per size")
    ap.add_argument("--sched-cache", type=str, default=None,
                    help="batched: JSON schedule cache (read when its device/runtime/build key matches)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also launch a plain device copy of known size (counter scaling)")
    ap.add_argument("--workload", choices=("batched", "cheb3d", "serve", "single", "convergence", "ct4d"),
                    default="batched",
                    help="batched: the headline batched workload (default); cheb3d: one 3-D "
                         "Chebyshev filter on a 64^3 grid (RK4 on MFMA, range measurement); serve: "
                         "many live tracks fed by Poisson arrivals through the serving runtime; single: "
                         "per-op latency of one 1-D (N 64, FP64) and one 2-D (128^2, FP64 and FP32) filter; "
                         "convergence: spectral vs finite-difference time update against the heat kernel; "
                         "ct4d: the 4-D coordinated turn with terrain measurements, N_pa = 34, Monte Carlo "
                         "RMSE / ASTD")
    ap.add_argument("--mc", type=int, default=20, help="ct4d: Monte-Carlo runs")
    ap.add_argument("--tracks", type=int, default=10000, help="serve: live tracks")
    ap.add_argument("--rates", type=str, default="1000,2000,5000,10000,20000,50000",
                    help="serve: offered request rates (requests/s; one request = predict + update)")
    ap.add_argument("--serve-seconds", type=float, default=2.0, help="serve: arrival window per rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(independent filters would be partitioned across processes); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "cheb3d":
        return run_cheb3d(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "single":
        return run_single(args)
    if args.workload == "convergence":
        return run_convergence(args)
    if args.workload == "ct4d":
        return run_ct4d(args)
    return run_batched(args)


def run_batched(args):
    import numpy as np
    import torch
    import workloads as W
    from paper_2412_07240_amd import binding as B

    nf = args.filters
    n_lat = 0 if args.no_extras else 30
    K = args.warmup + args.steps + n_lat + 2
    log(f"bench: generating {nf} filters x {K} measurements")
    scs = W.batched_workload(nf, K=K)
    T = scs[0].T
    pts = int(sum(sc.model.N[0] * sc.model.N[1] for sc in scs))
    Z = np.zeros((K, nf, 2))
    for i, sc in enumerate(scs):
        Z[:, i, :] = sc.z
    ctx = B.pmf_ctx_create(0)
    sched_report = None
    if not args.no_autotune:
        # per-size schedule of the fused kernel, timed on synthetic filters of each
        # size (about the count of that size in this batch), before the timed region
        log("bench: autotuning the fused kernel's schedules for this batch's mix of sizes")
        mix = {N: sum(1 for sc in scs if sc.model.N[0] == N) for N in W.BATCH_SIZES}
        sched_report = B.pmf_autotune(ctx, mix, 10, args.sched_cache)
        for line in sched_report.strip().splitlines():
            log("  " + line)
    schedules = {f"{N}x{N}": B.pmf_get_schedule(ctx, 2, N) for N in W.BATCH_SIZES}
    log("bench: creating filters")
    fs = [B.pmf_create(ctx, sc.model, sc.prior) for sc in scs]
    fa = B.FilterArray(fs)

    log(f"bench: warmup {args.warmup} steps")
    k = 0
    for _ in range(args.warmup):
        B.pmf_batch_step(ctx, fa, T, Z[k])
        k += 1
    B.pmf_stream_sync()
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        B.pmf_batch_step(ctx, fa, T, Z[k])
        k += 1
    B.pmf_stream_sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the fused kernel's own duration: HIP events around it on its stream
    B.pmf_batch_profile(ctx, True)
    for _ in range(args.steps):
        B.pmf_batch_step(ctx, fa, T, Z[k % K])
        k += 1
    kms, nl = B.pmf_batch_kernel_time(ctx)
    B.pmf_batch_profile(ctx, False)
    k = args.warmup + args.steps
    ms_per_step = 1e3 * elapsed / args.steps
    value = pts * args.steps / elapsed
    kavg_ms = kms / max(nl, 1)
    achieved = BYTES_PER_POINT * pts / (kavg_ms * 1e-3) / 1e9
    log(f"bench: {ms_per_step:.3f} ms/step, kernel {kavg_ms:.3f} ms, {value:.3e} pt/s")

    out = {
        "metric": METRIC, "value": value, "unit": "grid-point updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched: {nf} independent 2-D filters, N x N with N uniform in "
                               "{32,48,64,96,128}, exact integrator, linear-Gaussian update, "
                               "planning kernel + one fused launch per step (a workgroup per group of same-size filters)",
                   "filters": nf, "points_per_step": pts, "T": T, "reductions": "f64",
                   "schedules": schedules,
                   "autotune": None if args.no_autotune else
                   "pmf_autotune on a synthetic batch with this batch's mix of sizes: coordinate descent "
                   "over sizes, 10 timed steps x 3 rounds per variant, kept if >= 1 % faster"},
    }
    traffic = None
    valu = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("source_hash") == source_hash() and tr.get("points_per_step") == pts:
            traffic = tr.get("bytes_per_launch")
            valu = tr.get("valu_wave_instr_per_launch")
    # The fused cycle is bound by VALU issue (the HBM roofline is priced beside it):
    # algorithmic FP32 flops per launch over the live kernel time, against the
    # non-packed FP32 vector peak
    flops = float(sum(sc.model.N[0] * sc.model.N[1] * fused_flops_per_point(sc.model.N[0]) for sc in scs))
    tflops = flops / (kavg_ms * 1e-3) / 1e12
    out["roofline"] = {"bound": "alu", "achieved": tflops, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": tflops / FP32_VALU_PEAK_TFLOPS, "traffic": traffic,
                       "kernel": "pmf::k_fused", "kernel_ms": kavg_ms,
                       "algorithmic_flops_per_launch": flops,
                       "why": "VALU issue limits the fused cycle (hbm frac well below its valu_issue frac)"}
    out["hbm"] = {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                  "target_frac": HBM_TARGET_FRAC, "gap_to_target": HBM_TARGET_FRAC / (achieved / HBM_PEAK_GBS),
                  "algorithmic_bytes_per_launch": BYTES_PER_POINT * pts, "traffic": traffic}
    if valu:
        # what actually bounds the fused cycle: VALU issue (SQ_INSTS_VALU of the
        # same sources from the counter run, over the live kernel time)
        lane = 64.0 * valu
        out["valu_issue"] = {"lane_instr_per_point": lane / pts,
                             "achieved": lane / (kavg_ms * 1e-3), "peak": VALU_PEAK_LANE_INSTR,
                             "unit": "lane-instructions/s", "frac": lane / (kavg_ms * 1e-3) / VALU_PEAK_LANE_INSTR}

    sampled = None
    if not args.no_extras:
        # p50/p99 latency of a step (submit -> results on the host)
        lat = []
        lls = None
        for _ in range(n_lat):
            t1 = time.perf_counter()
            lls = B.pmf_batch_step(ctx, fa, T, Z[k], want_loglik=True)
            lat.append(1e3 * (time.perf_counter() - t1))
            k += 1
        out["latency_ms"] = {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "what": "one batched step, submit to log-likelihoods on the host"}
        # one step of 8 sampled filters, kept for the oracle check of the CPU leg
        rng = np.random.default_rng(7)
        sample = sorted(rng.choice(nf, size=8, replace=False).tolist())
        before = [B.pmf_get_state(fs[i])[1:] for i in sample]
        lls = B.pmf_batch_step(ctx, fa, T, Z[k], want_loglik=True)
        after = [B.pmf_get_state(fs[i])[1:] for i in sample]
        sampled = (sample, before, after, Z[k].copy())
        k += 1
        # 8 steps per call through one captured graph (pmf_batch_run), synchronous,
        # beside the plain per-step launches of the timed region
        Kg, reps = 8, 5
        zg = np.stack([Z[(k + j) % K] for j in range(Kg)])
        B.pmf_batch_run(ctx, fa, T, zg)        # capture + first replay
        tg = []
        for _ in range(reps):
            t1 = time.perf_counter()
            B.pmf_batch_run(ctx, fa, T, zg)
            tg.append(1e3 * (time.perf_counter() - t1) / Kg)
        out["graph_run"] = {"ms_per_step": float(np.median(tg)), "steps_per_call": Kg,
                            "plain_ms_per_step": ms_per_step,
                            "what": "pmf_batch_run: 8 steps captured into one HIP graph, replayed (z upload, "
                                    "log-likelihoods back and a host synchronisation per call), median of 5 calls"}
        log(f"bench: graph of {Kg} steps {np.median(tg):.3f} ms/step vs plain {ms_per_step:.3f} ms/step")
        # plain single-filter FP64 GPU path on a sample of the same filters
        sub = scs[:64]
        ff = [B.pmf_create(ctx, sc.model.with_(precision=W.FP64), sc.prior) for sc in sub]
        ppts = sum(sc.model.N[0] * sc.model.N[1] for sc in sub)
        for f, sc in zip(ff, sub):
            B.pmf_predict(f, T)
            B.pmf_update(f, sc.z[0])
        B.pmf_stream_sync()
        t1 = time.perf_counter()
        reps = 3
        for r in range(reps):
            for f, sc in zip(ff, sub):
                B.pmf_predict(f, T)
                B.pmf_update(f, sc.z[1 + r])
        B.pmf_stream_sync()
        dtp = time.perf_counter() - t1
        plain = ppts * reps / dtp
        out["plain_fp64_gpu"] = {"value": plain, "unit": "grid-point updates/s",
                                 "what": "64 of the same filters, FP64, one filter at a time through "
                                         "pmf_predict + pmf_update (generic kernels)",
                                 "speedup_of_value": value / plain}
        for f in ff:
            B.pmf_destroy(f)
        out["equal_accuracy"] = equal_accuracy(B, ctx, scs, W, np)
        log(f"bench: L1 vs the exact Kalman posterior: batched FP32 {out['equal_accuracy']['batched_fp32']['l1_max']:.2e}, "
            f"plain FP64 {out['equal_accuracy']['plain_fp64']['l1_max']:.2e}")

    if args.copy_probe:
        a = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": a.numel() * 4, "write": a.numel() * 4}

    for f in fs:
        B.pmf_destroy(f)
    B.pmf_ctx_destroy(ctx)

    if not args.no_cpu:
        # the CPU leg: the oracle (checker and baseline) and the CPU-FFT reference
        if sampled is not None:
            out["l1_vs_fp64_oracle"] = sampled_oracle_l1(scs, T, *sampled)
            log(f"bench: sampled L1 vs oracle {out['l1_vs_fp64_oracle']['max']:.2e}")
        log(f"bench: CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, nf)
        log(f"bench: CPU-FFT reference (~{args.cpu_seconds:.0f} s)")
        out["cpu_fft_reference"] = cpu_fft_baseline(args.cpu_seconds, nf)
        out["cpu_fft_reference"]["gpu_over_cpu"] = value / out["cpu_fft_reference"]["value"]
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def kalman_posteriors(sc, K):
    """Exact Kalman filter of a linear-Gaussian scenario: posterior (mean, cov)
    after each of K cycles (discretisation e^{AT}, e^{AT} W(T) e^{A^T T}; W by
    Van Loan's block exponential)."""
    import numpy as np
    import scipy.linalg
    m = sc.model
    A = np.asarray(m.A, float)[:2, :2]
    D = np.asarray(m.D, float)[:2, :2]
    C = np.zeros((4, 4))
    C[:2, :2], C[:2, 2:], C[2:, 2:] = A, D, -A.T
    E = scipy.linalg.expm(C * sc.T)
    Phi = E[:2, :2]
    Qd = E[:2, 2:] @ Phi.T                       # e^{AT} W(T) e^{A^T T}
    H = np.asarray(m.H, float)[:m.nz, :2]
    R = np.asarray(m.noise_cov, float)[0][:m.nz, :m.nz]
    mu = np.asarray(sc.prior.mean, float)[0][:2]
    P = np.asarray(sc.prior.cov, float)[0][:2, :2]
    out = []
    for k in range(K):
        mu, P = Phi @ mu, Phi @ P @ Phi.T + Qd
        G = P @ H.T @ np.linalg.inv(H @ P @ H.T + R)
        mu = mu + G @ (np.asarray(sc.z[k], float)[:m.nz] - H @ mu)
        P = (np.eye(2) - G @ H) @ P
        out.append((mu.copy(), 0.5 * (P + P.T)))
    return out


def kalman_l1(sc, c, M, P, mean, cov):
    """L1 of a grid density against N(mean, cov) on the same nodes (normalised
    with the grid's cell volume)."""
    import numpy as np
    N0, N1 = sc.model.N[0], sc.model.N[1]
    U0, U1 = np.meshgrid(np.arange(N0) - N0 // 2, np.arange(N1) - N1 // 2, indexing="ij")
    X = np.stack([c[0] + M[0, 0] * U0 + M[0, 1] * U1, c[1] + M[1, 0] * U0 + M[1, 1] * U1], axis=-1)
    r = X - mean
    Ci = np.linalg.inv(cov)
    g = np.exp(-0.5 * np.einsum("...i,ij,...j->...", r, Ci, r))
    vol = abs(np.linalg.det(M))
    g /= vol * g.sum()
    return float(vol * np.abs(np.asarray(P, float).reshape(N0, N1) - g).sum())


def equal_accuracy(B, ctx, scs, W, np, nfil=8, K=10):
    """Both GPU paths, batched FP32 and plain single-filter FP64, over the same K
    cycles of the same nfil filters (one of each grid size at least), each
    measured against the exact Kalman posterior of the linear-Gaussian model."""
    pick, seen = [], set()
    for i, sc in enumerate(scs):
        if sc.model.N[0] not in seen or len(pick) < nfil:
            pick.append(i)
            seen.add(sc.model.N[0])
        if len(pick) >= nfil and len(seen) >= 5:
            break
    sub = [scs[i] for i in pick]
    fb = [B.pmf_create(ctx, sc.model, sc.prior) for sc in sub]
    fp = [B.pmf_create(ctx, sc.model.with_(precision=W.FP64), sc.prior) for sc in sub]
    kfs = [kalman_posteriors(sc, K) for sc in sub]
    eb, ep, dpp = [], [], []
    try:
        for k in range(K):
            B.pmf_batch_step(ctx, fb, sub[0].T, np.array([sc.z[k] for sc in sub]))
            for f, sc in zip(fp, sub):
                B.pmf_predict(f, sc.T)
                B.pmf_update(f, sc.z[k])
            for j, sc in enumerate(sub):
                _, c1, M1, _, P1 = B.pmf_get_state(fb[j])
                _, c2, M2, _, P2 = B.pmf_get_state(fp[j])
                eb.append(kalman_l1(sc, c1, M1, P1, *kfs[j][k]))
                ep.append(kalman_l1(sc, c2, M2, P2, *kfs[j][k]))
                dpp.append(abs(eb[-1] - ep[-1]))
    finally:
        for f in fb + fp:
            B.pmf_destroy(f)
    return {"what": f"{len(sub)} filters (N in {sorted(seen)}), {K} cycles each, L1 of the grid density "
                    "against the exact Kalman posterior on its own grid (linear-Gaussian models)",
            "batched_fp32": {"l1_max": max(eb), "l1_mean": float(np.mean(eb))},
            "plain_fp64": {"l1_max": max(ep), "l1_mean": float(np.mean(ep))},
            "largest_difference_of_the_two": max(dpp)}


def sampled_oracle_l1(scs, T, sample, before, after, z):
    """L1 and pointwise error of the sampled filters' batched step against the
    FP64 oracle's step from the same pre-step state (CPU leg)."""
    import numpy as np
    import oracle
    worst, worst_pt = 0.0, 0.0
    for j, i in enumerate(sample):
        c, M, t, P = before[j]
        st = oracle.State(np.array(c), np.array(M), t, np.asarray(P, float))
        st, _ = oracle.predict(scs[i].model, st, T)
        st, ll_o, status, _, _ = oracle.update(scs[i].model, st, z[i])
        c2, M2, _, P2 = after[j]
        mapped = oracle.interpolate(scs[i].model, oracle.State(c2, M2, st.t, np.asarray(P2, float)), st.c, st.M)
        q = oracle.quadrature_weights(scs[i].model, st.M)
        worst = max(worst, float(np.sum(q * np.abs(mapped - st.P))))
        worst_pt = max(worst_pt, float(np.abs(mapped - st.P).max() / np.abs(st.P).max()))
    return {"max": worst, "pointwise_max": worst_pt, "filters": len(sample), "tolerance": 1e-5}


def _cpu_fft_worker(args):
    idxs, budget = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        import oracle
        import workloads as W
        from oracle import cpu_fft
        pts, busy = 0, 0.0
        t_end = time.perf_counter() + budget
        for i in idxs:
            if time.perf_counter() > t_end:
                break
            sc = W.batched_filter(i, K=4)
            f = cpu_fft.Filter(sc.model, sc.T)
            st = oracle.create(sc.model, sc.prior)
            t0 = time.perf_counter()
            for k in range(4):
                st = f.predict(st)
                st, _ = f.update(st, sc.z[k])
            busy += time.perf_counter() - t0
            pts += 4 * sc.model.N[0] * sc.model.N[1]
        return pts, busy


def cpu_fft_baseline(seconds: float, nfilters: int):
    """The CPU-FFT reference (scipy.fft real transforms, FP64) on the host cores:
    one single-threaded process per core over the batched workload's filters."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16)
    per = [list(range(w, nfilters, cores)) for w in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_cpu_fft_worker, [(p, seconds) for p in per])
    wall = time.perf_counter() - t0
    pts = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": pts / busy if busy > 0 else None, "unit": "grid-point updates/s", "cores": cores,
            "kind": "scipy.fft CPU reference (FP64, not the oracle)",
            "sample": f"4 predict+update cycles per filter of the batched workload's filters, {cores} processes x "
                      f"1 thread, ~{seconds:.0f} s each; {pts} points in {busy:.1f} s busy ({wall:.1f} s wall)"}


# ------------------------------------------------------------------ 3-D Chebyshev

MFMA_FP32_PEAK_TFLOPS = 157.3
CHEB_PRODUCTS_PER_STAGE = 7   # line products per RK4 stage in 3-D


def _cheb_cpu_worker(args):
    N, frac = args
    from threadpoolctl import threadpool_limits
    import oracle
    import workloads as W
    sc = W.config3(K=1, N=N, precision=W.FP64)
    m = sc.model
    st = oracle.create(m, sc.prior)
    l_full = oracle.substeps(m, st, sc.T)
    Ts = sc.T * frac
    t0 = time.perf_counter()
    st2, l = oracle.predict(m, st, Ts)
    tp = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.update(m, st2, sc.z[0])
    tu = time.perf_counter() - t0
    return l_full, l, tp, tu


def cheb_cpu_baseline(N: int, frac: float):
    """The oracle on a bounded sample of one cycle: a predict over a fraction of
    the interval (its substeps cost the same each) and one full update; the cycle
    time is the sample's predict time scaled to the full substep count plus the
    update time.  Multi-threaded BLAS on all host cores, as the oracle runs."""
    l_full, l, tp, tu = _cheb_cpu_worker((N, frac))
    cycle = tp * l_full / max(l, 1) + tu
    cores = os.cpu_count() or 1
    return {"value": N ** 3 / cycle, "unit": "grid-point updates/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle, one {N}^3 predict over {frac:.2f} T ({l} of {l_full} substeps, "
                      f"{tp:.1f} s) scaled to the full interval, plus one update ({tu:.1f} s); "
                      f"NumPy BLAS on {cores} host threads"}


def run_cheb3d(args):
    import numpy as np
    import torch
    import workloads as W
    from paper_2412_07240_amd import binding as B

    N = 64
    K = args.warmup + args.steps + 2
    sc = W.config3(K=K, N=N, precision=W.FP32)
    pts = N ** 3
    ctx = B.pmf_ctx_create(0)
    f = B.pmf_create(ctx, sc.model, sc.prior)
    log(f"bench cheb3d: warmup {args.warmup} cycles")
    k = 0
    for _ in range(args.warmup):
        B.pmf_predict(f, sc.T)
        B.pmf_update(f, sc.z[k])
        k += 1
    B.pmf_stream_sync()
    torch.cuda.synchronize()
    # predict duration from HIP events on the stream the passes run on (the null
    # stream, which is also torch's default stream here)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    subs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        B.pmf_predict(f, sc.T)
        ev[i][1].record()
        subs.append(B.pmf_last_substeps(f))
        B.pmf_update(f, sc.z[k])
        k += 1
    B.pmf_stream_sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pred_ms = [a.elapsed_time(b) for a, b in ev]
    ms_per_step = 1e3 * elapsed / args.steps
    value = pts * args.steps / elapsed
    lsum = sum(subs)
    flops = 4.0 * lsum * CHEB_PRODUCTS_PER_STAGE * 2.0 * N * pts
    achieved = flops / (sum(pred_ms) * 1e-3) / 1e12
    log(f"bench cheb3d: {ms_per_step:.2f} ms/cycle, substeps {subs}, {achieved:.2f} TFLOP/s")
    out = {
        "metric": METRIC, "value": value, "unit": "grid-point updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "one 3-D filter, 64^3 Chebyshev grid, RK4 method of lines on MFMA, "
                               "range measurement; one step = predict(T = 0.05) + update",
                   "points": pts, "T": sc.T, "substeps": subs, "reductions": "f64"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / MFMA_FP32_PEAK_TFLOPS, "traffic": None,
                     "kernel": "pmf::k_cheb_plane + pmf::k_cheb_pass (all passes of a predict)",
                     "predict_ms": float(np.mean(pred_ms)),
                     "us_per_substep": 1e3 * sum(pred_ms) / lsum,
                     "algorithmic_flops_per_predict": flops / args.steps},
    }
    pair = None
    if not args.no_extras:
        # one predict against the FP64 GPU path (parity-tested against the oracle)
        f64 = B.pmf_create(ctx, sc.model.with_(precision=W.FP64), sc.prior)
        _, c0, M0, t0_, P0 = B.pmf_get_state(f)
        B.pmf_set_state(f64, c0, M0, t0_, P0, W.CHEBYSHEV, W.FP64)
        B.pmf_predict(f, sc.T)
        B.pmf_predict(f64, sc.T)
        _, _, M1, _, P1 = B.pmf_get_state(f)
        _, _, M2, _, P2 = B.pmf_get_state(f64)
        pair = (M2, P1, P2)
        B.pmf_destroy(f64)
    B.pmf_destroy(f)
    B.pmf_ctx_destroy(ctx)
    if not args.no_cpu and pair is not None:
        # CPU leg: the Clenshaw-Curtis quadrature of the oracle for the L1 of the two GPU paths
        import oracle
        M2, P1, P2 = pair
        q = oracle.quadrature_weights(sc.model, np.asarray(M2))
        out["l1_vs_fp64"] = {"value": float(np.sum(q * np.abs(np.asarray(P1, float) - np.asarray(P2, float)))),
                             "what": "one predict, FP32 MFMA path vs the FP64 GPU path from the same state",
                             "tolerance": 1e-5}
    if not args.no_cpu:
        log("bench cheb3d: CPU oracle baseline")
        out["cpu_baseline"] = cheb_cpu_baseline(N, 0.2)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ serving

def run_serve(args):
    import numpy as np
    import torch
    import workloads as W
    from paper_2412_07240_amd import binding as B

    rates = [float(r) for r in args.rates.split(",") if r]
    ntr = args.tracks
    n_req = [int(r * args.serve_seconds) for r in rates]
    K = 8 + int(2 * sum(n_req) / ntr)            # measurements per track, with margin
    log(f"bench serve: generating {ntr} tracks")
    scs = [W.serving_track(i, K=K) for i in range(ntr)]
    pts = np.array([int(np.prod(sc.model.N[:sc.model.nx])) for sc in scs])
    cls = np.array([sc.model.nx for sc in scs])
    ctx = B.pmf_ctx_create(0)
    srv = B.pmf_server_create(ctx, 64 << 30, ntr)
    log("bench serve: creating tracks")
    ids = [B.pmf_server_add_track(srv, sc.model, sc.prior) for sc in scs]
    st0 = B.pmf_server_stats_get(srv)
    nextk = np.zeros(ntr, dtype=int)
    rng = np.random.default_rng(np.random.SeedSequence([241207240, 7]))
    # warm every track once (first fused use uploads its constants)
    tag = 0
    for i in range(ntr):
        B.pmf_server_submit_cycle(srv, ids[i], scs[i].T, scs[i].z[nextk[i]], tag=tag)
        nextk[i] += 1
        tag += 2
    B.pmf_server_drain(srv)
    B.pmf_server_poll(srv, cap=2 * tag + 16)
    torch.cuda.synchronize()
    results = []
    for rate, n in zip(rates, n_req):
        arr = W.poisson_arrivals(rate, n, seed_index=int(rate))
        who = rng.integers(ntr, size=n)
        tag0 = tag
        log(f"bench serve: {rate:.0f} req/s, {n} requests")
        t0 = time.perf_counter()
        for j in range(n):
            target = t0 + arr[j]
            while time.perf_counter() < target:
                pass
            i = int(who[j])
            B.pmf_server_submit_cycle(srv, ids[i], scs[i].T, scs[i].z[nextk[i] % K], tag=tag)
            nextk[i] += 1
            tag += 2
        t_sub = time.perf_counter() - t0
        B.pmf_server_drain(srv)
        t_all = time.perf_counter() - t0
        done = B.pmf_server_poll(srv, cap=2 * (tag - tag0) + 16)
        upd = [c for c in done if c["op"] == B.PMF_OP_UPDATE]
        lat = np.array([c["latency_us"] for c in upd]) / 1e3
        tr = np.array([c["track"] for c in upd])
        fused = np.mean([c["fused"] for c in upd]) if upd else 0.0
        rec = {"offered_req_s": rate, "requests": n, "achieved_req_s": len(upd) / t_all,
               "points_per_s": float(pts[tr].sum() / t_all), "submit_window_s": t_sub,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "fused_fraction": float(fused)}
        for nx in (1, 2, 3):
            sel = cls[tr] == nx
            if sel.any():
                rec[f"p50_ms_{nx}d"] = float(np.percentile(lat[sel], 50))
                rec[f"p99_ms_{nx}d"] = float(np.percentile(lat[sel], 99))
        results.append(rec)
        log(f"bench serve: {json.dumps(rec)}")
    stats = B.pmf_server_stats_get(srv)
    B.pmf_server_destroy(srv)
    # plain path: FP64 copies of a sample of the tracks, one op at a time
    sub = scs[:200]
    ff = [B.pmf_create(ctx, sc.model.with_(precision=W.FP64), sc.prior) for sc in sub]
    for f, sc in zip(ff, sub):
        B.pmf_predict(f, sc.T)
        B.pmf_update(f, sc.z[0])
    B.pmf_stream_sync()
    t1 = time.perf_counter()
    for f, sc in zip(ff, sub):
        B.pmf_predict(f, sc.T)
        B.pmf_update(f, sc.z[1])
    B.pmf_stream_sync()
    dtp = time.perf_counter() - t1
    plain = float(pts[:200].sum() / dtp)
    for f in ff:
        B.pmf_destroy(f)
    B.pmf_ctx_destroy(ctx)
    best = max(results, key=lambda r: r["points_per_s"])
    out = {
        "metric": METRIC, "value": best["points_per_s"], "unit": "grid-point updates/s", "n_gpus": 1,
        "steps": len(rates), "warmup": 1, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serving: {ntr} live tracks (50% 1-D N 64-256, 40% 2-D N 32-128, "
                               "10% 3-D N 32-64), Poisson arrivals, one request = predict(T = 0.05) + "
                               "update, per-track FIFO",
                   "tracks": ntr, "device_bytes": st0["used_bytes"], "rates": rates,
                   "seconds_per_rate": args.serve_seconds},
        "serving": results,
        "server_stats": stats,
        "plain_fp64_gpu": {"value": plain, "unit": "grid-point updates/s",
                           "what": "200 of the same tracks in FP64, one op at a time through "
                                   "pmf_predict + pmf_update"},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ single filters

def run_single(args):
    """Latency-bound single filters: every op is followed by a host synchronisation
    (the host needs the result before the next measurement), as a tracker would."""
    import numpy as np
    import workloads as W
    from paper_2412_07240_amd import binding as B

    checks = []
    cases = [("1-D N=64 FP64, RK4 (>= 10 substeps), T = 0.1", W.config1(K=200)),
             ("2-D 128^2 FP64, RK4, cubic measurement, T = 0.05", W.config2(K=200, precision=W.FP64)),
             ("2-D 128^2 FP32, RK4, cubic measurement, T = 0.05", W.config2(K=200, precision=W.FP32))]
    ctx = B.pmf_ctx_create(0)
    res = []
    n_cyc = args.steps * 5
    for name, sc in cases:
        m = sc.model
        pts = int(np.prod(m.N[:m.nx]))
        f = B.pmf_create(ctx, m, sc.prior)
        k = 0
        for _ in range(args.warmup):
            B.pmf_predict(f, sc.T)
            B.pmf_update(f, sc.z[k])
            k += 1
        B.pmf_stream_sync()
        tp, tu = [], []
        t0 = time.perf_counter()
        for _ in range(n_cyc):
            a = time.perf_counter()
            B.pmf_predict(f, sc.T)
            B.pmf_stream_sync()
            b = time.perf_counter()
            B.pmf_update(f, sc.z[k], want_loglik=True)   # synchronises to read the log-likelihood
            c = time.perf_counter()
            tp.append(b - a)
            tu.append(c - b)
            k += 1
        el = time.perf_counter() - t0
        # the last cycle, kept for the oracle check of the CPU leg
        _, c0, M0, t_, P0 = B.pmf_get_state(f)
        B.pmf_predict(f, sc.T)
        B.pmf_update(f, sc.z[k])
        _, c1, M1, _, P1 = B.pmf_get_state(f)
        B.pmf_destroy(f)
        res.append({"case": name, "points": pts, "cycles": n_cyc, "points_per_s": pts * n_cyc / el,
                    "predict_p50_ms": 1e3 * float(np.percentile(tp, 50)),
                    "predict_p99_ms": 1e3 * float(np.percentile(tp, 99)),
                    "update_p50_ms": 1e3 * float(np.percentile(tu, 50)),
                    "update_p99_ms": 1e3 * float(np.percentile(tu, 99))})
        checks.append((sc, k, (c0, M0, t_, P0), (c1, M1, P1)))
        log(f"bench single: {json.dumps(res[-1])}")
    B.pmf_ctx_destroy(ctx)
    if not args.no_cpu:
        # CPU leg: the last cycle of each case against the oracle from the same pre-cycle state
        import oracle
        for r, (sc, k, (c0, M0, t_, P0), (c1, M1, P1)) in zip(res, checks):
            m = sc.model
            st = oracle.State(np.array(c0), np.array(M0), t_, np.asarray(P0, float))
            st, _ = oracle.predict(m, st, sc.T)
            st, _, _, _, _ = oracle.update(m, st, sc.z[k])
            mapped = oracle.interpolate(m, oracle.State(np.array(c1), np.array(M1), st.t, np.asarray(P1, float)),
                                        st.c, st.M)
            r["l1_vs_fp64_oracle_one_cycle"] = float(np.sum(oracle.quadrature_weights(m, st.M) * np.abs(mapped - st.P)))
    out = {
        "metric": METRIC, "value": res[1]["points_per_s"], "unit": "grid-point updates/s", "n_gpus": 1,
        "steps": n_cyc, "warmup": args.warmup,
        "ms_per_step": res[1]["predict_p50_ms"] + res[1]["update_p50_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "single filters, one op at a time with a host synchronisation after each; "
                               "value is the 2-D 128^2 FP64 case"},
        "single": res, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ convergence study

# N even with 2 (N + 1) also of the form 2^a 3^b 5^c 7^d 11^e 13^f 17^g (the fast sine
# transform of the finite differences is an FFT of that length; the spectral
# updates use N-point FFTs)
CONV_N = (16, 20, 24, 26, 32, 34, 44, 48, 50, 54, 64, 80, 84, 90, 98, 104, 120, 168, 220, 224, 242)


def _gm_density(x, w, mu, var):
    import numpy as np
    return np.sum(w * np.exp(-0.5 * (x[:, None] - mu) ** 2 / var) / np.sqrt(2.0 * np.pi * var), axis=1)


def run_convergence(args):
    """One time update of a 1-D density without advection (A = 0, D = 1, T = 0.05)
    on the GPU, for N over a sweep, by the spectral integrators (exact in time;
    its sine-series variant, exact in time; implicit Euler with 10 and 100
    substeps, the paper's Algorithm; RK4) and by
    the finite-difference baseline (sine-transform route; substeps at the
    stability limit, and at a quarter of it), each against the heat kernel
    solution at the nodes.  Densities: one Gaussian and a three-component
    Gaussian mixture; grid half-widths of 5 and 8 standard deviations."""
    import numpy as np
    import workloads as W
    from paper_2412_07240_amd import binding as B

    T = 0.05
    dens = {"gaussian": (np.array([1.0]), np.array([0.0]), np.array([0.3])),
            "mixture3": (np.array([0.3, 0.4, 0.3]), np.array([-1.2, 0.3, 1.5]), np.array([0.15, 0.1, 0.2]))}
    methods = {"sd_exact": (W.INT_EXACT, 1), "sd_sine": (W.INT_SINE, 1), "sd_euler_l10": (W.INT_EULER, 10),
               "sd_euler_l100": (W.INT_EULER, 100), "sd_rk4": (W.INT_RK4, 1), "fdm_dst": (W.INT_FDM, 1),
               "fdm_dst_r025": (W.INT_FDM, 0)}
    ctx = B.pmf_ctx_create(0)
    rows = []
    for dname, (w, mu, var) in dens.items():
        prior = W.PriorSpec(w, mu[:, None], var[:, None, None])
        for span in (5.0, 8.0):
            for N in CONV_N:
                for mname, (integ, lmin) in methods.items():
                    m = W.ModelSpec(nx=1, A=np.zeros((1, 1)), Q=np.ones((1, 1)), N=(N,), span_sigmas=span,
                                    t_nominal=T, integrator=integ, substeps=lmin, precision=W.FP64,
                                    meas_kind=W.H_LINEAR, nz=1, H=np.ones((1, 1)), **W.gaussian_noise([[0.01]]))
                    if lmin == 0:
                        # finite differences at the mesh ratio h D / delta^2 = 1/4 (time error
                        # below the spatial one) instead of the stability limit 1
                        f = B.pmf_create(ctx, m.with_(substeps=1), prior)
                        _, _, M0, _, _ = B.pmf_get_state(f)
                        B.pmf_destroy(f)
                        m = m.with_(substeps=int(np.ceil(4.0 * T / M0[0][0] ** 2)))
                    f = B.pmf_create(ctx, m, prior)
                    B.pmf_predict(f, T)
                    l = B.pmf_last_substeps(f)
                    _, c, M, _, P = B.pmf_get_state(f)
                    # time per predict of the same filter (the host waits for each)
                    reps = []
                    for _ in range(5):
                        t0 = time.perf_counter()
                        B.pmf_predict(f, T)
                        B.pmf_stream_sync()
                        reps.append(time.perf_counter() - t0)
                    B.pmf_destroy(f)
                    x = c[0] + M[0][0] * (np.arange(N) - N // 2)
                    ex = _gm_density(x, w, mu, var + T)
                    err = np.asarray(P, float) - ex
                    rows.append({"density": dname, "span": span, "N": N, "method": mname, "substeps": l,
                                 "max_rel_err": float(np.max(np.abs(err)) / np.max(ex)),
                                 "l1_err": float(abs(M[0][0]) * np.sum(np.abs(err))),
                                 "us_per_predict": 1e6 * float(np.median(reps))})
    B.pmf_ctx_destroy(ctx)
    # slope of log(error) against log(N) for the finite differences (second order: -2)
    slopes = {}
    for dname in dens:
        for span in (5.0, 8.0):
            for meth in ("fdm_dst", "fdm_dst_r025"):
                sel = [r for r in rows if r["density"] == dname and r["span"] == span and r["method"] == meth
                       and r["N"] >= 100]
                sl = np.polyfit(np.log([r["N"] for r in sel]), np.log([r["max_rel_err"] for r in sel]), 1)[0]
                slopes[f"{dname}_span{span:g}_{meth}"] = float(sl)
    at = {f"{r['density']}_span{r['span']:g}_{r['method']}_N{r['N']}": r["max_rel_err"]
          for r in rows if r["N"] in (80, 224)}
    # time per predict, FDM (fast sine transform) against the spectral exact update
    tcmp = {}
    for N in CONV_N:
        sel = {r["method"]: r["us_per_predict"] for r in rows if r["N"] == N and r["density"] == "gaussian"
               and r["span"] == 8.0}
        tcmp[str(N)] = {"fdm_dst_us": sel["fdm_dst"], "sd_exact_us": sel["sd_exact"], "sd_sine_us": sel["sd_sine"]}
    out = {"metric": "max relative error of one time update vs the heat kernel", "value": None,
           "unit": "relative error", "n_gpus": 1, "steps": len(rows), "warmup": 0, "ms_per_step": None,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "1-D, A = 0, D = 1, T = 0.05; Gaussian N(0, 0.3) and mixture "
                                  "0.3 N(-1.2, 0.15) + 0.4 N(0.3, 0.1) + 0.3 N(1.5, 0.2); spans 5 and 8 sigma",
                      "N": list(CONV_N)},
           "fdm_slope_N100_up": slopes, "at_N80_N224": at, "us_per_predict": tcmp, "rows": rows,
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ 4-D coordinated turn

def run_ct4d(args):
    """The paper's numerical illustration at one-GPU scale: coordinated turn with
    known turn rate, N_pa = 34 (34^4 = 1,336,336 points), the synthetic terrain in
    place of the SRTM map, mixture measurement noise; RMSE and ASTD per state
    component over Monte-Carlo runs (steps k = 0..K, the filtering estimate after
    each update, the prior at k = 0), and the time per predict + update."""
    import numpy as np
    import workloads as W
    from paper_2412_07240_amd import binding as B

    K = args.steps
    N = 34
    ctx = B.pmf_ctx_create(0)
    se = np.zeros(4)
    var = np.zeros(4)
    cnt = 0
    times = []
    status_bits = 0
    for mc in range(args.mc):
        sc = W.config6(K=K, N=N, precision=W.FP32, mc=mc)
        f = B.pmf_create(ctx, sc.model, sc.prior)
        m0 = sc.prior.mean[0]
        se += (sc.truth[0] - m0) ** 2
        var += np.diag(sc.prior.cov[0])
        cnt += 1
        for k in range(K):
            B.pmf_stream_sync()
            t0 = time.perf_counter()
            B.pmf_predict(f, sc.T)
            B.pmf_update(f, sc.z[k], want_loglik=True)
            times.append(time.perf_counter() - t0)
            mean, cov, st = B.pmf_moments(f, 4)
            status_bits |= int(st)
            se += (sc.truth[k + 1] - mean) ** 2
            var += np.diag(cov)
            cnt += 1
        B.pmf_destroy(f)
        log(f"bench ct4d: run {mc} done, {1e3 * np.median(times):.2f} ms per cycle")
    B.pmf_ctx_destroy(ctx)
    pts = N ** 4
    warm = times[args.warmup:] if len(times) > args.warmup else times
    ms = 1e3 * float(np.median(warm))
    out = {"metric": METRIC, "value": pts / (ms * 1e-3), "unit": "grid-point updates/s", "n_gpus": 1,
           "steps": len(warm), "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "4-D coordinated turn (turn rate 30 deg/s, D = diag(0,1,0,1), T_s = 1), "
                                  "N_pa = 34 (1,336,336 points), synthetic terrain measurement, noise "
                                  "0.5 N(0,1) + 0.5 N(20,1); one step = predict + update",
                      "mc_runs": args.mc, "steps_per_run": K},
           "rmse": {"p_x": float(np.sqrt(se[0] / cnt)), "v_x": float(np.sqrt(se[1] / cnt)),
                    "p_y": float(np.sqrt(se[2] / cnt)), "v_y": float(np.sqrt(se[3] / cnt))},
           "astd": {"p_x": float(np.sqrt(var[0] / cnt)), "v_x": float(np.sqrt(var[1] / cnt)),
                    "p_y": float(np.sqrt(var[2] / cnt)), "v_y": float(np.sqrt(var[3] / cnt))},
           "status_bits": status_bits, "p99_ms_per_step": 1e3 * float(np.percentile(warm, 99)),
           "roofline": None, "cpu_baseline": None}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
