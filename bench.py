#!/usr/bin/env python3
"""Benchmark: elastic-net solves/s at relative KKT residual <= 1e-6 on one MI355X.

Workload: m=500 observations, n=100,000 features in blocks of 50 with Toeplitz
correlation rho=0.6, 20 true nonzeros, SNR 5, alpha=0.5, lambda=0.3*lambda_max,
tol 1e-6 (synthetic, seeded).  One step = one complete SsNAL-EN solve from a
cold start, the design already resident in HBM.  `value` is the mixed-
precision path (design stored in FP32, FP32 accumulation in A^T v and the
Newton matrix, FP64 Cholesky / line search / KKT residual, FP64-accumulated
refresh of A^T y); the plain FP64 path on the same problem is reported beside
it, and BF16 storage as a second mixed variant.  The roofline entry is the
Newton pass w_d = A^T d (k_gemv_t over the FP32 design, FP32 accumulation),
timed live with HIP events around each of its launches on the solve's stream
in every fourth timed solve (the event records leave the GPU idle for a few
microseconds around each timed launch, so timing every solve would slow the
solves being measured).
The CPU baseline is the FP64 oracle on the host's cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Further sections in the same JSON line (each can be skipped): the m=1000,
n=1e6 single solve in FP32/BF16/FP64 (--no-c3); the 100-point SNP-like path
with gcv / e-bic at every point and 10-fold cross validation (--no-path); a
long-column Newton-CG solve, m=20000, n=2e5 (--no-cg, or --cg-only); the
Newton-matrix SYRK at its largest dense shape, m=4096 from r=8192 columns, in
TFLOP/s against the MFMA peak (--no-syrk); the serving stream (--serving 0
skips it).
       python bench.py --profile-syrk K     K launches of that SYRK per storage type
Serving: a stream of requests with the serving workload's distributions (m
log-uniform in [100, 2000], n log-uniform in [1e4, n_max], Gaussian-Toeplitz
or SNP-like designs, FP32 or BF16 storage, tol 1e-6) goes through the
library's serving loop: first closed-loop (all submitted at once) for the
saturated rate, then open-loop with seeded Poisson arrivals at 0.8x that rate;
latency is scheduled arrival -> completion.  The serving designs are drawn on
the GPU (datagen.make_problem_device: same distributions, torch's seeded
generator).  Default: the full stream of 512 requests with n_max = 5e5.
Counter runs (HBM traffic of the A^T v kernel and of a plain copy of the same
byte count, for the calibration factor):
       python bench.py --profile-gemv K     K launches of the FP32 A^T v pass
       python bench.py --profile-copy K     K device copies of m*n*4 bytes
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def _traffic_from_profile(kernel_src, store):
    """HBM bytes per A^T v launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"gemv_t_block_toeplitz_m500_n100000_{store}_pmc.txt")
    if not os.path.exists(path):
        return None
    digest = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != digest:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def large_bench(reps=3):
    """The m=1000, n=1e6 Gaussian single solve with A stored in FP32, BF16 and
    FP64: solves/s and the A^T d bandwidth for each."""
    import torch

    import datagen
    from paper_2006_03970_amd import binding
    from paper_2006_03970_amd.device import design_to_device, vec_to_device

    t0 = time.time()
    p = datagen.make_problem("c3", seed=1, store="f32", want_f64=False)
    print(f"[bench] c3 generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    ctx = binding.Context(0)
    stream = torch.cuda.current_stream()
    b = vec_to_device(p.b)
    out = {"workload": "Gaussian elastic net, m=1000, n=1000000, k=50, snr=3, alpha=0.5, "
                       "c_lambda=0.1, tol=1e-6"}
    for store in ("f32", "bf16", "f64"):
        if store == "f32":
            A = design_to_device(p.AT, "f32")
        elif store == "bf16":
            A = design_to_device(datagen.f32_to_bf16_bits(p.AT), "bf16")
        else:
            A = design_to_device(p.AT.astype("float64"), "f64")
        opts = binding.make_opts(timing=1)
        x = torch.empty(p.n, dtype=torch.float64, device=A.device)
        binding.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, x_out=x, opts=opts, stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = []
        for _ in range(reps):
            _, info = binding.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, x_out=x, opts=opts,
                                             stream=stream)
            infos.append(info)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t) / reps
        s_a = {"f32": 4, "bf16": 2, "f64": 8}[store]
        atd_s = sum(i["atd_ms"] for i in infos) / sum(i["atd_launches"] for i in infos) / 1e3
        out[store] = {"solves_per_s": 1.0 / el, "ms_per_solve": el * 1e3,
                      "eta": infos[-1]["kkt_rel"], "status": infos[-1]["status"],
                      "iterations": [infos[-1]["outer_iters"], infos[-1]["newton_iters"]],
                      "nnz": infos[-1]["nnz"],
                      "atd_gbs": float(p.m) * p.n * s_a / atd_s / 1e9, "atd_us": atd_s * 1e6}
        print(f"[bench] c3 {store}: {out[store]['ms_per_solve']:.1f} ms/solve", file=sys.stderr, flush=True)
        del A
        torch.cuda.empty_cache()
    return out


def path_bench(reps=2):
    """The warm-started path of the SNP-like workload (m=500, n=2e5, alpha=0.7,
    100 points c_lambda 1 -> 0.01, FP32 storage, tol 1e-6): points/s of the
    path, then gcv / e-bic at every point (degrees of freedom, least squares
    on the selected features), 10-fold cross validation over the same grid,
    and the point each criterion selects."""
    import numpy as np
    import torch

    import datagen
    from paper_2006_03970_amd import binding
    from paper_2006_03970_amd.device import design_to_device, vec_to_device

    p = datagen.make_problem("c4", seed=1, store="f32", want_f64=False)
    ctx = binding.Context(0)
    stream = torch.cuda.current_stream()
    A = design_to_device(p.AT, "f32")
    b = vec_to_device(p.b)
    alpha = 0.7
    cl = datagen.path_grid(100)
    X, infos, status = binding.ssnal_en_path(ctx, A, b, alpha, cl, tol=1e-6, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        X, infos, status = binding.ssnal_en_path(ctx, A, b, alpha, cl, tol=1e-6, X_out=X, stream=stream)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / reps
    lam_max = float(torch.max(torch.abs(binding.ssnal_gemv_t(ctx, A, b, acc64=True)))) / alpha
    torch.cuda.synchronize()
    t = time.perf_counter()
    sel = []
    for k in range(len(cl)):
        l2 = (1 - alpha) * cl[k] * lam_max
        sel.append(binding.ssnal_en_model_select(ctx, A, b, X[k], l2, stream=stream))
    torch.cuda.synchronize()
    el_sel = time.perf_counter() - t
    gcv = [s["gcv"] if s["status"] == 0 else np.inf for s in sel]
    ebic = [s["ebic"] if s["status"] == 0 else np.inf for s in sel]
    kg, ke = int(np.argmin(gcv)), int(np.argmin(ebic))
    # 10-fold cross validation over the same grid: ten warm-started paths on the
    # training rows of each fold, validation error at every point
    fold = torch.from_numpy(np.random.default_rng(5).permutation(np.arange(p.m) % 10).astype(np.int32))
    fold = fold.to(A.device)
    torch.cuda.synchronize()
    t = time.perf_counter()
    E, _, cv_status = binding.ssnal_en_cv(ctx, A, b, fold, 10, alpha, cl, tol=1e-6, stream=stream)
    el_cv = time.perf_counter() - t
    kc = int(np.argmin(E.mean(axis=0)))
    out = {"workload": "SNP-like elastic-net path, m=500, n=200000, k=30, snr=5, alpha=0.7, "
                       "100 points c_lambda 1 -> 0.01, FP32 storage, tol 1e-6",
           "status": status, "points_per_s": len(cl) / el, "ms_per_path": el * 1e3,
           "newton_iters": int(sum(i["newton_iters"] for i in infos)),
           "model_select_ms_per_point": el_sel / len(cl) * 1e3,
           "gcv_point": kg, "gcv_nnz": sel[kg]["r"], "ebic_point": ke, "ebic_nnz": sel[ke]["r"],
           "cv10_status": cv_status, "cv10_ms": el_cv * 1e3, "cv10_point": kc,
           "cv10_nnz": int(torch.count_nonzero(X[kc]))}
    print(f"[bench] path: {out['ms_per_path']:.1f} ms/path, model selection "
          f"{out['model_select_ms_per_point']:.2f} ms/point, 10-fold cv {out['cv10_ms']:.0f} ms",
          file=sys.stderr, flush=True)
    return out


def cg_bench(reps=2, r_fixed=16000):
    """Newton-CG on long columns: Gaussian design m=20000, n=200000 (FP32
    storage, 16 GB, drawn on the device), alpha=0.5, lambda = 0.005 lambda_max,
    tol 1e-6, where the active set and m both exceed 4096 for most Newton
    steps, so the directions come from conjugate gradients.  Reports the solve,
    then the CG iteration rate at a fixed r = 16000 (random columns): two
    gathered passes over A_J (2 m r 4 bytes) per iteration against HBM peak."""
    import torch

    import datagen
    from paper_2006_03970_amd import binding

    m, n = 20000, 200000
    cfg = dict(m=m, n=n, design="gauss", k=50, snr=5.0, alpha=0.5, c_lam=0.005)
    dev = torch.device("cuda:0")
    p = datagen.make_problem_device(cfg, seed=1, store="f32", device=dev)
    ctx = binding.Context(0)
    stream = torch.cuda.current_stream()
    x, info = binding.ssnal_en_solve(ctx, p["AT"], p["b"], p["lam1"], p["lam2"], tol=1e-6, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        x, info = binding.ssnal_en_solve(ctx, p["AT"], p["b"], p["lam1"], p["lam2"], tol=1e-6,
                                         x_out=x, stream=stream)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / reps
    g = torch.randn(m, generator=torch.Generator(device=dev).manual_seed(5), device=dev,
                    dtype=torch.float64)
    perm = torch.randperm(n, generator=torch.Generator(device=dev).manual_seed(6), device=dev)
    J = torch.sort(perm[:r_fixed])[0].to(torch.int32)
    best = float("inf")
    iters = 0
    for _ in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, iters = binding.ssnal_newton_cg(ctx, p["AT"], J, 5e-4, g, 0.0, maxit=40, stream=stream)
        best = min(best, (time.perf_counter() - t) / max(iters, 1))
    gbs = 2.0 * m * r_fixed * 4 / best / 1e9
    out = {"workload": "Gaussian elastic net, m=20000, n=200000, k=50, snr=5, alpha=0.5, "
                       "c_lambda=0.005, FP32 storage, tol 1e-6 (Newton-CG directions)",
           "status": info["status"], "ms_per_solve": el * 1e3, "newton_iters": info["newton_iters"],
           "cg_iters": info["cg_iters"], "nnz": info["nnz"], "eta": info["kkt_rel"],
           "cg_iteration": {"r": r_fixed, "iterations": iters, "us_per_iter": best * 1e6,
                            "alg_bytes_per_iter": 2 * m * r_fixed * 4, "alg_gbs": gbs,
                            "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}}
    print(f"[bench] newton-cg: {out['ms_per_solve']:.0f} ms/solve, {info['cg_iters']} CG iterations; "
          f"{best * 1e6:.0f} us per CG iteration at r={r_fixed} ({gbs:.0f} GB/s)", file=sys.stderr, flush=True)
    del p, x
    torch.cuda.empty_cache()
    return out


SYRK_M, SYRK_R = 4096, 8192  # the largest dense Newton matrix: m x m from r columns
MFMA_PEAK_TFS = {"f64": 78.6, "f32": 157.3}  # MI355X dense MFMA, published


def syrk_bench(reps=5, launches=0):
    """The Newton matrix I + kappa A_J A_J^T at its largest dense shape (m =
    4096 rows, r = 8192 active columns; FP64 storage on FP64 MFMA, FP32
    storage on FP32 MFMA): TFLOP/s of the m (m + 1) r flops of the lower
    triangle against the dense MFMA peak.  launches > 0: only that many calls
    per storage type (a short run for rocprofv3 counters)."""
    import torch

    from paper_2006_03970_amd import binding

    m, r = SYRK_M, SYRK_R
    dev = torch.device("cuda:0")
    ctx = binding.Context(0)
    gen = torch.Generator(device=dev).manual_seed(11)
    J = torch.arange(r, dtype=torch.int32, device=dev)
    out = {}
    for store, dt in (("f64", torch.float64), ("f32", torch.float32)):
        A = torch.randn((r, m), generator=gen, device=dev, dtype=dt)
        A /= torch.linalg.vector_norm(A, dim=1, keepdim=True)
        if launches:
            for k in range(launches):
                binding.ssnal_newton_matrix(ctx, A, J, 0.5, 0)
                print(f"[bench] syrk {store} launch {k}", file=sys.stderr, flush=True)
            continue
        binding.ssnal_newton_matrix(ctx, A, J, 0.5, 0)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            binding.ssnal_newton_matrix(ctx, A, J, 0.5, 0)
        el = (time.perf_counter() - t) / reps
        tfs = m * (m + 1) * r / el / 1e12
        out[store] = {"ms": el * 1e3, "tflops": tfs, "peak_tflops": MFMA_PEAK_TFS[store],
                      "frac": tfs / MFMA_PEAK_TFS[store]}
        print(f"[bench] syrk {store}: {el * 1e3:.2f} ms, {tfs:.1f} TFLOP/s", file=sys.stderr, flush=True)
        del A
    if launches:
        return None
    out["shape"] = {"m": m, "r": r, "flops": m * (m + 1) * r}
    return out


def serving_bench(nreq, nmax, slots, seed=7):
    """p50/p99 latency and solves/s of the serving loop over a request stream."""
    import numpy as np
    import torch

    import datagen
    from paper_2006_03970_amd import binding
    from paper_2006_03970_amd.device import design_to_device, vec_to_device

    reqs = datagen.serving_requests(nreq, seed=seed, n_range=(10_000, int(nmax)))
    t0 = time.time()
    probs = []
    dev = torch.device("cuda:0")
    for q in reqs:
        p = datagen.make_problem_device(q, seed=q["seed"], store=q["store"], device=dev)
        x = torch.empty(p["n"], dtype=torch.float64, device=dev)
        probs.append(dict(A=p["AT"], b=p["b"], l1=p["lam1"], l2=p["lam2"], x=x, m=p["m"], n=p["n"],
                          store=p["store"]))
    torch.cuda.synchronize()
    print(f"[bench] serving: generated and uploaded {nreq} requests in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    srv = binding.Server(0, hbm_budget=64 << 30, max_slots=slots)
    try:
        # alone: one request at a time (also the warm-up)
        alone = []
        for q in probs[: min(8, nreq)]:
            t = time.perf_counter()
            info = srv.wait(srv.submit(q["A"], q["b"], q["l1"], q["l2"], 1e-6, q["x"]))
            alone.append(time.perf_counter() - t)
            assert info["status"] == 0, info
        # closed loop: everything submitted at once
        t = time.perf_counter()
        tickets = [srv.submit(q["A"], q["b"], q["l1"], q["l2"], 1e-6, q["x"]) for q in probs]
        infos = [srv.wait(tk) for tk in tickets]
        sat = nreq / (time.perf_counter() - t)
        bad = [i["status"] for i in infos if i["status"] != 0]
        # open loop: Poisson arrivals at 0.8x the saturated rate
        rate = 0.8 * sat
        gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=nreq)
        arrive = np.cumsum(gaps) - gaps[0]
        lat = np.zeros(nreq)
        pending = {}
        start = time.perf_counter()
        nxt = 0
        while nxt < nreq or pending:
            now = time.perf_counter() - start
            while nxt < nreq and arrive[nxt] <= now:
                q = probs[nxt]
                pending[srv.submit(q["A"], q["b"], q["l1"], q["l2"], 1e-6, q["x"])] = nxt
                nxt += 1
            for tk in list(pending):
                info = srv.poll(tk)
                if info is not None:
                    k = pending.pop(tk)
                    lat[k] = time.perf_counter() - start - arrive[k]
                    if info["status"] != 0:
                        bad.append(info["status"])
            time.sleep(5e-5)
        span = time.perf_counter() - start
    finally:
        srv.close()
    ms = np.array([q["m"] for q in probs])
    ns = np.array([q["n"] for q in probs])
    return {
        "requests": nreq, "slots": slots, "n_range": [10_000, int(nmax)], "m_range": [100, 2000],
        "mean_m": float(ms.mean()), "mean_n": float(ns.mean()),
        "stores": {s: sum(1 for q in probs if q["store"] == s) for s in ("f32", "bf16")},
        "saturated_solves_per_s": sat,
        "poisson_rate_per_s": rate,
        "solves_per_s": nreq / span,
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_latency_ms": float(lat.mean() * 1e3),
        "alone_latency_ms_mean": float(np.mean(alone) * 1e3),
        "nonzero_status": bad,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c3", action="store_true", help="skip the m=1000, n=1e6 single-solve section")
    ap.add_argument("--no-path", action="store_true", help="skip the path + model selection section")
    ap.add_argument("--no-cg", action="store_true", help="skip the Newton-CG (m=20000) section")
    ap.add_argument("--cg-only", action="store_true", help="run only the Newton-CG section")
    ap.add_argument("--serving", type=int, default=512, help="requests in the serving stream (0 = off)")
    ap.add_argument("--serving-nmax", type=float, default=5e5)
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--profile-gemv", type=int, default=0)
    ap.add_argument("--profile-copy", type=int, default=0)
    ap.add_argument("--profile-syrk", type=int, default=0,
                    help="only K launches of the m=4096, r=8192 Newton-matrix SYRK per storage type")
    ap.add_argument("--no-syrk", action="store_true", help="skip the Newton-matrix SYRK section")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the solver has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    from paper_2006_03970_amd import binding
    from paper_2006_03970_amd.device import design_to_device, vec_to_device

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.cg_only:
        print(json.dumps({"newton_cg": cg_bench()}), flush=True)
        return
    if args.profile_syrk:
        syrk_bench(launches=args.profile_syrk)
        return
    cfg = datagen.CONFIGS["c2"]
    t0 = time.time()
    p64 = datagen.make_problem("c2", seed=args.seed, store="f64")
    AT32 = p64.AT.astype(np.float32)
    print(f"[bench] generated m={p64.m} n={p64.n} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    A32 = design_to_device(AT32, "f32")
    b = vec_to_device(p64.b)
    ctx = binding.Context(0)
    stream = torch.cuda.current_stream()
    if args.profile_gemv or args.profile_copy:
        # short runs for rocprofv3 counter collection, nothing else
        if args.profile_gemv:
            w = torch.empty(p64.n, dtype=torch.float64, device=dev)
            for k in range(args.profile_gemv):
                binding.ssnal_gemv_t(ctx, A32, b, w, acc64=False, stream=stream)
                print(f"[bench] A^T v launch {k}", file=sys.stderr, flush=True)
        else:
            src_t = torch.ones(p64.m * p64.n, dtype=torch.float32, device=dev)
            dst_t = torch.empty_like(src_t)
            for k in range(args.profile_copy):
                dst_t.copy_(src_t)
                torch.cuda.synchronize()
                print(f"[bench] copy launch {k}", file=sys.stderr, flush=True)
        return
    A64 = design_to_device(p64.AT, "f64")
    Abf = design_to_device(datagen.f32_to_bf16_bits(AT32), "bf16")

    TIME_EVERY = 4  # solves of the timed region whose A^T d launches carry HIP events

    def run(A, steps, timing):
        opts_t = binding.make_opts(timing=1)
        opts_n = binding.make_opts(timing=0)
        infos = []
        x = torch.empty(p64.n, dtype=torch.float64, device=dev)
        for k in range(steps):
            opts = opts_t if timing and k % TIME_EVERY == 0 else opts_n
            _, info = binding.ssnal_en_solve(ctx, A, b, p64.lam1, p64.lam2, tol=p64.tol, x_out=x,
                                             opts=opts, stream=stream)
            if info["status"] != 0:
                raise RuntimeError(f"solve did not converge: {info}")
            infos.append(info)
        return infos, x

    def timed(A, label):
        run(A, args.warmup, True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos, x = run(A, args.steps, True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        print(f"[bench] {label}: {args.steps} solves in {el:.3f}s", file=sys.stderr, flush=True)
        return el, infos, x

    el32, inf32, x32 = timed(A32, "mixed f32")
    el64, inf64, x64 = timed(A64, "fp64")
    elbf, infbf, _ = timed(Abf, "mixed bf16")

    def atd_stats(infos, s_a):
        """Average duration of the Newton A^T d launches (HIP events, in the
        timed solves that carried them)."""
        timed_infos = [i for i in infos if i["atd_launches"] > 0]
        calls = sum(i["atd_launches"] for i in timed_infos)
        ms = sum(i["atd_ms"] for i in timed_infos)
        avg_s = ms / calls / 1e3
        bytes_per_launch = float(p64.m) * p64.n * s_a
        return avg_s, bytes_per_launch, calls / len(timed_infos)

    avg32, bpl32, calls32 = atd_stats(inf32, 4)
    avg64, bpl64, calls64 = atd_stats(inf64, 8)
    avgbf, bplbf, _ = atd_stats(infbf, 2)
    achieved = bpl32 / avg32 / 1e9
    traffic = _traffic_from_profile(os.path.join(ROOT, "paper_2006_03970_amd", "csrc", "k_gemv.hip"), "f32")

    out = {
        "metric": "EN solves/s at KKT<=1e-6 (mixed FP32 storage)",
        "value": args.steps / el32,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el32 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "block-Toeplitz elastic net, m=500, n=100000, rho=0.6, blocks of 50, "
                        "k=20, snr=5, alpha=0.5, c_lambda=0.3, tol=1e-6",
            "m": p64.m, "n": p64.n, "precision": "A in FP32 (FP32 accumulation in A^T v and "
            "A_J A_J^T); FP64 Cholesky, line search, KKT residual, FP64-accumulated A^T y refresh",
            "parallelism": "single GPU",
        },
        "fp64_solves_per_s": args.steps / el64,
        "fp64_ms_per_step": el64 / args.steps * 1e3,
        "mixed_over_fp64": (args.steps / el32) / (args.steps / el64),
        "bf16_solves_per_s": args.steps / elbf,
        "eta": {"mixed_f32": inf32[-1]["kkt_rel"], "fp64": inf64[-1]["kkt_rel"],
                "mixed_bf16": infbf[-1]["kkt_rel"]},
        "iterations": {"mixed_f32": [inf32[-1]["outer_iters"], inf32[-1]["newton_iters"]],
                       "fp64": [inf64[-1]["outer_iters"], inf64[-1]["newton_iters"]],
                       "mixed_bf16": [infbf[-1]["outer_iters"], infbf[-1]["newton_iters"]]},
        "atd_launches_per_solve": {"mixed_f32": calls32, "fp64": calls64},
        "atd_gbs": {"mixed_f32": achieved, "fp64": bpl64 / avg64 / 1e9,
                    "mixed_bf16": bplbf / avgbf / 1e9},
        "roofline": {
            "bound": "hbm",
            "kernel": "Newton pass w_d = A^T d: k_gemv_t<float, float, 2> (FP32 design, FP32 accumulation)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": bpl32, "avg_launch_us": avg32 * 1e6,
        },
    }

    if not args.no_c3:
        out["large_single_solve"] = large_bench()
    if not args.no_path:
        out["path"] = path_bench()
    if not args.no_cg:
        out["newton_cg"] = cg_bench()
    if not args.no_syrk:
        out["newton_matrix_syrk"] = syrk_bench()
    if args.serving > 0:
        out["serving"] = serving_bench(args.serving, args.serving_nmax, args.serving_slots)

    if not args.no_cpu_baseline:
        import oracle
        if not os.path.exists(oracle.LIB_PATH):
            oracle.build()
        nsolve = 0
        t = time.perf_counter()
        while True:
            oracle.en_solve(p64.AT, p64.b, p64.lam1, p64.lam2, tol=p64.tol)
            nsolve += 1
            if time.perf_counter() - t > 10.0 or nsolve >= 12:
                break
        el = time.perf_counter() - t
        out["cpu_baseline"] = {
            "value": nsolve / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{nsolve} complete FP64 oracle solves of the same problem (tol 1e-6), "
                      "single thread",
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
