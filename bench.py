#!/usr/bin/env python
"""Newton-Raphson multinomial-logit fits per second on one MI355X.

One step = one whole fit (fused pass, block Hessian, Cholesky solve, halving
line search, repeated until ||g||_2 <= 1e-8) of the largest single-GPU
workload: 400,000 individuals, 100 alternatives, 51 individual-specific
columns (incl. intercept, equicorrelated features) and 5 generic
alternative-varying variables (5,054 coefficients), data already resident
in HBM, started from theta = 0, FP64 throughout.

    python bench.py [--steps K] [--warmup W] [--prec fp64|fp32|bf16]
                    [--config c3]

Prints one JSON line.  Besides the fit rate it reports the beta-beta
Hessian MFMA kernel's rate against the MFMA peak of its dtype (HIP events
around every launch, on the stream it runs on), the fused pass kernel's HBM
rate, the p50/p99 fit latency, the FP32- and BF16-Hessian fits of the same
workload (iterations, coefficient difference to the FP64 fit), the
100,000-individual workload against the oracle's recorded optimum, the
500-alternative near-separable workload (iterations, line-search
backtracks, stop reason), the FP64 CPU oracle timed on the host cores over
a bounded sample, and the continuous-batching server on a stream of uneven
fits: saturated fits/s (mixed-precision and FP64 Hessians), p50/p99 latency
under Poisson arrivals, and a batch of 1024 small fits.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("NR fits/sec at 1e-8 grad tol + Hessian TFLOP/s (% MFMA peak); "
          "p50/p99 fit latency")
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
HBM_GBPS = 8000.0
GTOL = 1e-8


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def hess_kernel_flops(pr):
    """Useful flops of the beta-beta Hessian kernel per launch: 2 N per
    unique entry of the (K-1)K/2 blocks of p(p+1)/2 unique entries."""
    N, K, p = pr.N, pr.K, pr.p
    return 2.0 * N * ((K - 1) * K // 2) * (p * (p + 1) // 2)


def hess_total_flops(pr):
    """Useful flops of the whole Hessian (all blocks, unique entries)."""
    N, K, p, g, a = pr.N, pr.K, pr.p, pr.g, pr.a
    u = ((K - 1) * K // 2 * (p * (p + 1) // 2) + (K - 1) * p * K * a +
         K * (K - 1) // 2 * a * a + K * (a * (a + 1) // 2) +
         (K - 1) * p * g + K * a * g + g * (g + 1) // 2)
    return 2.0 * N * u


def pass_bytes(pr):
    """Algorithmic HBM bytes of one fused pass: read X, Y, Z, choice (and
    weights), write P and Ybar."""
    N, K, p, g, a = pr.N, pr.K, pr.p, pr.g, pr.a
    b = N * (p + K * g + K * a) * 8 + 4 * N + N * K * 8 + N * g * 8
    if pr.w is not None:
        b += 8 * N
    return float(b)


def predict_bytes(pr):
    """Algorithmic HBM bytes of one prediction: read X, Y, Z, write P."""
    N, K, p, g, a = pr.N, pr.K, pr.p, pr.g, pr.a
    return float(N * (p + K * g + K * a) * 8 + N * K * 8)


def fitted_methods(ctx, pr, dp, theta, reps=5):
    """Time the collinearity check (Gram products and ordered
    elimination), predict (one fused pass without choices) and the
    summary's standard errors (FP64 Hessian + factorisation with identity
    rows) at the fitted theta; compare the standard errors with the
    oracle's recorded table when one exists for this workload."""
    import numpy as np
    import torch

    import paper_1404_3177_amd as mnl
    X, Y, Z, _, w = dp._refs
    dq = mnl.Problem(X, Y, Z, None, w)
    ctx.predict(dq, theta)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
        enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.predict(dq, theta)
    e1.record()
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1) / reps
    se = ctx.summary(dq, theta)[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        se = ctx.summary(dq, theta)[0]
    torch.cuda.synchronize()
    sms = (time.perf_counter() - t0) / reps * 1e3
    ctx.collinear(dq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        keep = ctx.collinear(dq)
    cms = (time.perf_counter() - t0) / reps * 1e3
    # Wald test of one alternative's beta chunk (covariance block and a
    # quadratic form) and the score test of alpha at theta
    from paper_1404_3177_amd import hypothesis as hyp
    idx = list(range(pr.p))
    hyp.waldtest(ctx, dq, theta, idx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        wald = hyp.waldtest(ctx, dq, theta, idx)
    wms = (time.perf_counter() - t0) / reps * 1e3
    t0 = time.perf_counter()
    for _ in range(reps):
        score = hyp.scoretest(ctx, dp, theta, pr.g)
    scms = (time.perf_counter() - t0) / reps * 1e3
    # Hessian-vector product H(theta) v: the pass at theta, then the pass
    # of v in Hessian-vector mode (reads X, Y, Z, w and P)
    v = torch.ones(pr.n_params, dtype=torch.float64, device=theta.device)
    ctx.hessvec(dq, theta, v)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.hessvec(dq, theta, v)
    e1.record()
    torch.cuda.synchronize()
    hms = e0.elapsed_time(e1) / reps
    N, K = pr.N, pr.K
    hv_bytes = float(N * (pr.p + K * pr.g + K * pr.a) * 8 + N * K * 8 +
                     (8 * N if pr.w is not None else 0))
    hbytes = pass_bytes(pr) + hv_bytes
    out = {"hessvec": {"ms": hms, "bytes": hbytes,
                       "achieved_gbps": hbytes / hms * 1e-6,
                       "frac": hbytes / hms * 1e-6 / HBM_GBPS},
           "wald_test": {"ms": wms, "df": wald[1], "stat": wald[0]},
           "score_test": {"ms": scms, "df": score[1], "stat": score[0]},
           "collinear": {"ms": cms, "kept": [int(k.sum()) for k in keep],
                         "of": [pr.p, pr.g, pr.a]},
           "predict": {"ms": pms, "bytes": predict_bytes(pr),
                       "achieved_gbps": predict_bytes(pr) / pms * 1e-6,
                       "peak_gbps": HBM_GBPS,
                       "frac": predict_bytes(pr) / pms * 1e-6 / HBM_GBPS},
           "summary": {"ms": sms, "n_params": pr.n_params,
                       "se_rel_err_vs_oracle": None}}
    gold = os.path.join(ROOT, "tests", "golden",
                        f"summary_{pr.name}.npz")
    if os.path.exists(gold):
        ref = np.load(gold)
        th_ref = ref["theta"]
        if np.array_equal(theta.cpu().numpy(), th_ref) or \
                np.linalg.norm(theta.cpu().numpy() - th_ref) <= \
                1e-8 * np.linalg.norm(th_ref):
            sr = ctx.summary(dq, torch.from_numpy(th_ref).cuda())[0]
            out["summary"]["se_rel_err_vs_oracle"] = float(
                np.max(np.abs(sr.cpu().numpy() - ref["se"]) / ref["se"]))
    return out


def time_fits(ctx, dp, steps, warmup, prec, method="newton"):
    import torch
    for _ in range(warmup):
        ctx.fit(dp, gtol=GTOL, ftol=0.0, prec=prec, method=method)
    torch.cuda.synchronize()
    lat, infos = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        t = time.perf_counter()
        theta, info = ctx.fit(dp, gtol=GTOL, ftol=0.0, prec=prec,
                              method=method)
        lat.append(time.perf_counter() - t)
        infos.append(info)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return theta, infos, lat, total


def percentile(xs, q):
    xs = sorted(xs)
    k = (len(xs) - 1) * q
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def kernel_stats(pr, infos, prec):
    hk = sum(i["t_hess_kernel"] for i in infos)
    nh = sum(i["n_hess"] for i in infos)
    pk = sum(i["t_pass_kernel"] for i in infos)
    npass = sum(i["n_pass"] for i in infos)
    hess_ms = hk / max(nh, 1)
    pass_ms = pk / max(npass, 1)
    tflops = hess_kernel_flops(pr) / (hess_ms * 1e-3) / 1e12
    gbps = pass_bytes(pr) / (pass_ms * 1e-3) / 1e9
    return dict(hess_ms=hess_ms, n_hess=nh, pass_ms=pass_ms, n_pass=npass,
                tflops=tflops, gbps=gbps,
                peak=PEAK_TFLOPS[prec])


def _oracle_iteration_seconds(pr, n_obs):
    """Wall time of one oracle Newton iteration at theta = 0 on the first
    n_obs observations: log-likelihood + gradient, Hessian of Eq. 10 block
    by block, Cholesky solve, one line-search evaluation."""
    import numpy as np
    from oracle import mnl_ref as R
    sl = slice(0, n_obs)
    X, Y, Z, ch = pr.X[sl], pr.Y[sl], pr.Z[sl], pr.choice[sl]
    w = None if pr.w is None else pr.w[sl]
    th = np.zeros(pr.n_params)
    t0 = time.perf_counter()
    R.loglik(th, X, Y, Z, ch, w)
    g0 = R.gradient(th, X, Y, Z, ch, w)
    H = R.hessian(th, X, Y, Z, ch, w)
    d = R.newton_direction(H, g0)
    R.loglik(th + d, X, Y, Z, ch, w)
    return time.perf_counter() - t0


def cpu_baseline(pr, iters, target_s=12.0):
    """The FP64 oracle on the host cores over a bounded sample: one Newton
    iteration on the first n_s observations (n_s calibrated so the sample
    takes about target_s), scaled linearly to N (every step of the oracle
    is a sum over observations) and by the fit's iteration count, as
    fits/s."""
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    n_cal = min(pr.N, 2000)
    t_cal = _oracle_iteration_seconds(pr, n_cal)
    n_s = int(min(pr.N, max(n_cal, n_cal * target_s / max(t_cal, 1e-3))))
    t_s = _oracle_iteration_seconds(pr, n_s) if n_s > n_cal else t_cal
    if n_s <= n_cal:
        n_s = n_cal
    t_iter = t_s * pr.N / n_s
    return {"value": 1.0 / (t_iter * max(iters, 1)), "unit": "fits/s",
            "cores": int(threads), "kind": "oracle",
            "sample": (f"one NR iteration at theta=0 (loglik, gradient, Eq. 10 "
                       f"Hessian block by block, Cholesky solve, one "
                       f"line-search pass) on the first {n_s} of {pr.N} "
                       f"observations: {t_s:.1f} s; scaled by N/{n_s} and by "
                       f"the fit's {iters} iterations"),
            "seconds_per_iteration_full_N": t_iter}


STOP_NAMES = {0: "none", 1: "gtol", 2: "ftol", 3: "maxiter", 4: "ls_fail",
              5: "not_pd", 6: "nonfinite"}


def serve_run(hps, slots, prec, arrivals_s=None, graph=0):
    """Run host problems through a fresh continuous-batching server.  With
    arrivals_s (seconds from the start) requests are submitted at those
    times (open loop); without, all at once (closed loop, the saturated
    rate).  Latency = completion (theta in host memory) - arrival."""
    import threading
    import paper_1404_3177_amd as mnl
    srv = mnl.Server(slots=slots)
    n = len(hps)
    res = []

    def collect():
        while len(res) < n:
            res.extend(srv.wait(timeout_ms=200.0))
    th = threading.Thread(target=collect)
    th.start()
    t0 = srv.now_ms() + 20.0
    for i, h in enumerate(hps):
        t_arr = t0 + (arrivals_s[i] * 1e3 if arrivals_s is not None else 0.0)
        while True:
            dt = t_arr - srv.now_ms()
            if dt <= 0:
                break
            time.sleep(min(dt, 2.0) * 1e-3)
        srv.submit(h, gtol=GTOL, ftol=0.0, prec=prec, t_arrival=t_arr,
                   graph=graph)
    th.join()
    st = srv.stats()
    srv.close()
    span = max(r["t_done"] for r in res) - t0
    lat = [r["t_done"] - r["t_arrival"] for r in res]
    stops = {}
    for r in res:
        k = STOP_NAMES.get(r["info"]["stop_reason"], "error") \
            if r["status"] == 0 else f"error{r['status']}"
        stops[k] = stops.get(k, 0) + 1
    conv = sum(1 for r in res if r["status"] == 0 and
               r["info"]["stop_reason"] == 1)
    return {"requests": n, "fits_per_s": n / span * 1e3,
            "converged_fits_per_s": conv / span * 1e3,
            "span_s": span * 1e-3,
            "latency_ms": {"p50": percentile(lat, 0.5),
                           "p99": percentile(lat, 0.99),
                           "max": max(lat)},
            "iters_mean": sum(r["info"]["iters"] for r in res) / n,
            "stop_reasons": stops, "max_running": st["max_running"],
            "peak_footprint_gb": st["peak_in_use"] / 1e9}


def serving(n_req, slots, load):
    """The serving stream (uneven fits, mixed-precision Hessian): saturated
    rate, Poisson arrivals at load x that rate, the FP64 path at saturation
    for comparison, and a batch of 1024 independent small fits."""
    import numpy as np
    import torch
    import paper_1404_3177_amd as mnl
    import synth

    def pinned(shape, dt):
        tdt = {np.dtype(np.float64): torch.float64,
               np.dtype(np.int32): torch.int32}[np.dtype(dt)]
        return torch.empty(shape, dtype=tdt, pin_memory=True).numpy()
    log(f"serving: drawing {n_req} requests")
    t = time.perf_counter()
    reqs = synth.ServingStream(n_req, alloc=pinned).requests()
    hps = [mnl.HostProblem.from_numpy(r) for r in reqs]
    log(f"serving: requests ready in {time.perf_counter() - t:.1f} s")
    out = {"workload": (f"{n_req} requests: N log-uniform in [1e3, 2e5], K in "
                        f"5..60, p = 1 + 5..30, g in 0..5, a = 0; fit to "
                        f"||g||_2<=1e-8 from theta=0"),
           "slots": slots}
    log("serving: closed loop, bf16 Hessian")
    sat = serve_run(hps, slots, "bf16")
    log(f"serving: saturated {sat['fits_per_s']:.1f} fits/s")
    out["bf16_saturated"] = sat
    log("serving: closed loop, fp64 Hessian")
    out["fp64_saturated"] = serve_run(hps, slots, "fp64")
    rate = load * sat["fits_per_s"]
    arr = synth.serving_arrivals(n_req, rate)
    log(f"serving: Poisson arrivals at {rate:.1f} requests/s, bf16 Hessian")
    ol = serve_run(hps, slots, "bf16", arrivals_s=arr)
    ol["arrival_rate"] = rate
    ol["load"] = load
    out["bf16_poisson"] = ol
    out["mixed_vs_fp64_saturated"] = (sat["fits_per_s"] /
                                      out["fp64_saturated"]["fits_per_s"])
    log("serving: 1024 independent c1 fits (fp64)")
    c1 = [synth.make_problem(2000, 10, 6, 1, 0, seed=1000 + i, coef_sd=0.5)
          for i in range(1024)]
    out["c1_batch_1024_fp64"] = serve_run(
        [mnl.HostProblem.from_numpy(p, pinned=True) for p in c1], slots,
        "fp64")
    out["c1_batch_1024_fp64"]["path"] = (
        "server: host data, one group of batch-eligible requests per slot "
        "admission, mnl_fit_batch (one workgroup per fit)")
    out["c1_fit_batch_1024_device"] = fit_batch_run(c1)
    return out


def fit_batch_run(probs, reps=3):
    """The same fits through mnl_fit_batch on device-resident data (one
    persistent launch, no host copies): fits/s of the best of reps, and the
    per-fit device phase times of the workgroups."""
    import numpy as np
    import torch
    import paper_1404_3177_amd as mnl
    ctx = mnl.Context(0)
    dps = [mnl.Problem.from_numpy(p) for p in probs]
    s = torch.cuda.Stream()
    best, infos = None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, infos = ctx.fit_batch(dps, opts=dict(gtol=GTOL, ftol=0.0),
                                 stream=s)
        dt = time.perf_counter() - t
        best = dt if best is None else min(best, dt)
    stops = {}
    for i in infos:
        k = STOP_NAMES.get(i["stop_reason"], "error")
        stops[k] = stops.get(k, 0) + 1
    return {"fits": len(probs), "fits_per_s": len(probs) / best,
            "ms_per_batch": best * 1e3,
            "iters_mean": float(np.mean([i["iters"] for i in infos])),
            "stop_reasons": stops,
            "fit_device_ms_mean": {
                k: float(np.mean([i[k] for i in infos]))
                for k in ("t_loglik_grad", "t_hessian", "t_chol", "t_ls")},
            "path": "mnl_fit_batch, device data, one launch"}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_bb_c3_fp64_traffic.md")
HESS_SRC = os.path.join(ROOT, "paper_1404_3177_amd", "csrc", "k_bb.hip")


def source_digest(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per launch of the beta-beta kernel from the committed
    counter profile (FETCH_SIZE / WRITE_SIZE, scaled by a plain copy of
    known size), or None when the kernel source changed since."""
    try:
        txt = open(TRAFFIC_PROFILE).read()
        blk = txt.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(blk)
    except (OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256_16") != source_digest(HESS_SRC):
        return None
    return rec


def traffic_probe(config):
    """Workload of the counter profiles: a 1 GiB device copy (the HBM
    counters' calibration), then one Hessian of the workload in each
    precision (FP64, FP32, BF16; each with its fused pass).  Run under
    rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE, then the SQ counters)."""
    import torch
    import paper_1404_3177_amd as mnl
    import synth
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    x.fill_(1.0)
    torch.cuda.synchronize()
    y = x.clone()   # reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    del x, y
    pr = synth.make_config(config)
    ctx = mnl.Context(0)
    dp = mnl.Problem.from_numpy(pr, device="cuda:0")
    th = torch.from_numpy(0.5 * pr.theta_true).cuda()
    for prec in ("fp64", "fp32", "bf16"):
        ctx.hessian(dp, th, prec=prec)
        torch.cuda.synchronize()
    print(json.dumps({"probe": "done", "config": config,
                      "hessian_source": source_digest(HESS_SRC)}))


def rel_err(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def fit_entry(pr, infos, lat, total, prec):
    """Summary of timed fits: rate, iterations, line search, stop, the
    beta-beta kernel's rate."""
    kv = kernel_stats(pr, infos, prec)
    inf = infos[-1]
    if inf["hess_fallbacks"] > 0:
        # the kernel average mixes this precision's launches with the FP64
        # retries': no rate for the precision itself
        kv = dict(kv, tflops=float("nan"))
    return {"fits_per_s": len(lat) / total, "ms_per_fit": total / len(lat) * 1e3,
            "iters": inf["iters"], "ls_iters": inf["ls_iters"],
            "ls_backtracks": inf["ls_backtracks"],
            "hess_fp64_retries": inf["hess_fallbacks"],
            "stop_reason": STOP_NAMES.get(inf["stop_reason"], "?"),
            "grad_norm": inf["grad_norm"], "loglik": inf["loglik"],
            "bb_kernel_ms": kv["hess_ms"],
            "bb_tflops": kv["tflops"] if kv["tflops"] == kv["tflops"] else None,
            "bb_frac_of_peak": (kv["tflops"] / kv["peak"]
                                if kv["tflops"] == kv["tflops"] else None),
            "peak_tflops": kv["peak"],
            "phase_ms": {k: inf[k] for k in ("t_loglik_grad", "t_hessian",
                                              "t_chol", "t_ls")}}


def golden_theta(name):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"fit_{name}.npz")
    return np.load(path)["theta"] if os.path.exists(path) else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--config", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the serving stream (0: skip serving)")
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the workload of the counter profile")
    ap.add_argument("--batch-probe", action="store_true",
                    help="only run 1024 small fits through mnl_fit_batch "
                         "(the workload of the batched-kernel profile)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the "
              "fit is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    if args.traffic_probe:
        traffic_probe(args.config)
        return
    if args.batch_probe:
        import synth
        c1 = [synth.make_problem(2000, 10, 6, 1, 0, seed=1000 + i,
                                 coef_sd=0.5) for i in range(1024)]
        print(json.dumps(fit_batch_run(c1)), flush=True)
        return

    import numpy as np
    import torch

    import paper_1404_3177_amd as mnl
    import synth

    log(f"generating workload {args.config}")
    pr = synth.make_config(args.config)
    ctx = mnl.Context(0)
    dp = mnl.Problem.from_numpy(pr, device="cuda:0")
    log(f"timing {args.steps} fits ({args.prec} Hessian) after "
        f"{args.warmup} warmup fits")
    theta, infos, lat, total = time_fits(ctx, dp, args.steps, args.warmup,
                                         args.prec)
    info = infos[-1]
    ks = kernel_stats(pr, infos, args.prec)
    log(f"fit: {total / args.steps * 1e3:.2f} ms, iters {info['iters']}, "
        f"beta-beta kernel {ks['hess_ms']:.3f} ms = {ks['tflops']:.2f} TFLOP/s")
    th_main = theta.cpu().numpy()
    gold = golden_theta(args.config)
    coef_err = rel_err(th_main, gold) if gold is not None else None

    variants = {}
    if not args.no_variants and args.prec == "fp64":
        for vp in ("fp32", "bf16"):
            log(f"variant: {vp} Hessian")
            th_v, inf_v, lat_v, tot_v = time_fits(ctx, dp, max(3, args.steps),
                                                  1, vp)
            ent = fit_entry(pr, inf_v, lat_v, tot_v, vp)
            ent["workload"] = args.config
            ent["coef_rel_diff_vs_gpu_fp64_fit"] = rel_err(
                th_v.cpu().numpy(), th_main)
            if gold is not None:
                ent["coef_rel_err_vs_oracle"] = rel_err(th_v.cpu().numpy(),
                                                        gold)
            variants[f"{vp}_hessian"] = ent
        del dp
        torch.cuda.empty_cache()
        # the other workloads: 100,000 individuals (oracle optimum on
        # record), 500 near-separable alternatives, the 2,000-individual
        # single fit
        for name, precs, steps in (("c2", ("fp64", "fp32", "bf16"), 5),
                                   ("c5", ("fp64", "bf16"), 2),
                                   ("c1", ("fp64",), 20)):
            pq = synth.make_config(name)
            dq = mnl.Problem.from_numpy(pq, device="cuda:0")
            gq = golden_theta(name)
            for vp in precs:
                log(f"variant: {name} {vp} Hessian")
                th_q, inf_q, lat_q, tot_q = time_fits(ctx, dq, steps, 1, vp)
                ent = fit_entry(pq, inf_q, lat_q, tot_q, vp)
                ent["workload"] = (f"{name}: N={pq.N} K={pq.K} p={pq.p} "
                                   f"g={pq.g} a={pq.a} (n_p={pq.n_params})")
                ent["latency_ms"] = {"p50": percentile(lat_q, 0.5) * 1e3,
                                     "p99": percentile(lat_q, 0.99) * 1e3}
                if gq is not None:
                    ent["coef_rel_err_vs_oracle"] = rel_err(
                        th_q.cpu().numpy(), gq)
                variants[f"{name}_{vp}"] = ent
                if name == "c2" and vp == "fp64":
                    th_c2, pr_c2, dp_c2 = th_q, pq, dq
            if name == "c2":
                log("variant: c2 inexact Newton (Newton-CG, Hessian-vector "
                    "passes)")
                th_c, inf_c, lat_c, tot_c = time_fits(ctx, dq, 3, 1, "fp64",
                                                      "newton-cg")
                ic = inf_c[-1]
                ent = {"workload": "c2", "fits_per_s": len(lat_c) / tot_c,
                       "ms_per_fit": tot_c / len(lat_c) * 1e3,
                       "iters": ic["iters"], "hessvec_products": ic["cg_iters"],
                       "ms_in_products": ic["t_hessian"],
                       "ms_per_product": ic["t_hessian"] / max(ic["cg_iters"], 1),
                       "grad_norm": ic["grad_norm"],
                       "stop_reason": STOP_NAMES.get(ic["stop_reason"], "?")}
                if gq is not None:
                    ent["coef_rel_err_vs_oracle"] = rel_err(
                        th_c.cpu().numpy(), gq)
                variants["c2_newton_cg"] = ent
                log("fitted-model methods at the c2 optimum")
                methods = fitted_methods(ctx, pq, dq, th_c2)
            del dq
            torch.cuda.empty_cache()
    else:
        methods = None

    serve = None
    if args.serve_requests > 0:
        serve = serving(args.serve_requests, args.serve_slots, args.serve_load)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 CPU oracle (bounded sample)")
        cpu = cpu_baseline(pr, info["iters"])

    value = args.steps / total
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "fits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else f"f64+{args.prec}-hessian",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.config}: N={pr.N} K={pr.K} p={pr.p} g={pr.g} "
                         f"a={pr.a} (n_p={pr.n_params}), NR fit from theta=0 "
                         f"to ||g||_2<=1e-8, {args.prec} Hessian"),
            "N": pr.N, "K": pr.K, "p": pr.p, "g": pr.g, "a": pr.a,
            "n_params": pr.n_params, "gtol": GTOL,
        },
        "roofline": {
            "bound": "mfma",
            "achieved": ks["tflops"],
            "peak": ks["peak"],
            "unit": "TFLOP/s",
            "frac": ks["tflops"] / ks["peak"],
            "traffic": None,
            "traffic_source": None,
            "kernel": (f"k_bb<{ {'fp64': 0, 'fp32': 1, 'bf16': 2}[args.prec] },"
                       f"*> (beta-beta blocks, Khatri-Rao MFMA product)"),
            "kernel_ms": ks["hess_ms"],
            "launches": ks["n_hess"],
            "flops_per_launch": hess_kernel_flops(pr),
        },
        "pass_kernel": {
            "bound": "hbm", "achieved": ks["gbps"], "peak": HBM_GBPS,
            "unit": "GB/s", "frac": ks["gbps"] / HBM_GBPS,
            "kernel_ms": ks["pass_ms"], "launches": ks["n_pass"],
            "bytes_per_launch": pass_bytes(pr),
        },
        "latency_ms": {"p50": percentile(lat, 0.5) * 1e3,
                       "p99": percentile(lat, 0.99) * 1e3},
        "fit": {"iters": info["iters"], "ls_iters": info["ls_iters"],
                "ls_backtracks": info["ls_backtracks"],
                "stop_reason": STOP_NAMES.get(info["stop_reason"], "?"),
                "grad_norm": info["grad_norm"], "loglik": info["loglik"],
                "coef_rel_err_vs_oracle": coef_err,
                "hessian_total_flops": hess_total_flops(pr),
                "phase_ms": {k: info[k] for k in ("t_loglik_grad", "t_hessian",
                                                   "t_chol", "t_ls")}},
        "variants": variants,
        "fitted_methods": methods,
        "serving": serve,
        "cpu_baseline": cpu,
    }
    if args.prec == "fp64":
        rec = recorded_traffic()
        if rec is not None and rec.get("config") == args.config:
            res["roofline"]["traffic"] = rec["hbm_bytes_per_launch"]
            res["roofline"]["traffic_source"] = os.path.relpath(
                TRAFFIC_PROFILE, ROOT)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
