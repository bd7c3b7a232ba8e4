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
Beside `value` the line carries: FP64 and BF16 solves/s on the same problem;
`roofline_chol`, the FP64 Cholesky factor + solve of the Newton systems
inside the timed solves (sum of N^3/3 over their duration from HIP events)
against the FP64 peak; `concurrent`, 64 copies of the same solve through
the batch entry on 4 and 8 workers (aggregate solves/s of independent
solves sharing the GPU, FP32 and FP64 storage; --no-concurrent); and
further sections (each can be skipped): the
m=100, n=2000 single solve, alone (in one workgroup, and on the
multi-kernel path) and batched B in {1, 64, 1024}, batches as one launch
with one workgroup a problem and, beside it, on the batch entry's 8
workers with the multi-kernel path (--no-c1, or --c1-only); the
m=1000, n=1e6 single solve in
FP32/BF16/FP64 (--no-c3, or --c3-only); the 100-point SNP-like path with
gcv / e-bic at every point and 10-fold cross validation (--no-path); a
long-column Newton-CG solve, m=20000, n=2e5 (--no-cg, or --cg-only); the
Newton-matrix SYRK at its largest dense shape, m=4096 from r=8192 columns,
and at the first Newton step of the m=1000, n=1e6 solve, m=1000 from
r=520000 columns, in TFLOP/s against the MFMA peak (--no-syrk); the serving stream (--serving 0
skips it).
       python bench.py --profile-syrk K     K launches of that SYRK per storage type
Serving: a stream of requests with the serving workload's distributions (m
log-uniform in [100, 2000], n log-uniform in [1e4, n_max], Gaussian-Toeplitz
or SNP-like designs, FP32 or BF16 storage, tol 1e-6) goes through the
library's serving loop with the designs in HBM: every request alone (its
service time), then closed-loop (all submitted at once) for the saturated
rate, then open-loop with seeded Poisson arrivals at 0.8x that rate; latency
is scheduled arrival -> completion, slowdown is latency over the request's
time alone.  The first --serving-host requests are then served again from
pinned host memory (uploaded on admission; latency includes the upload), and
the first 128 in FP64 beside their mixed solves.  The serving designs are
drawn on the GPU (datagen.make_problem_device: same distributions, torch's
seeded generator).  Default: the full stream of 512 requests with n_max =
5e5.
The CPU-baseline leg times the FP64 oracle on one and on all host threads
and reports, with the oracle: every C2 solve's error (objective against a
tight oracle solve on the stored and the original design, support
difference, eta on both) and a seeded sample of served requests (eta on the
stored design and the duality-gap bound of the objective error).
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


def _traffic_from_profile(kernel_srcs, store):
    """HBM bytes per A^T v launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel sources (the kernel file and the
    device helpers it includes; else None)."""
    path = os.path.join(ROOT, "profiles", f"gemv_t_block_toeplitz_m500_n100000_{store}_pmc.txt")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for src in kernel_srcs:
        h.update(open(src, "rb").read())
    digest = h.hexdigest()
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256") != digest:
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


def c1_bench(single_reps=200, batches=(1, 64, 1024)):
    """The single-solve workload (m=100, n=2000 Gaussian, FP64, tol 1e-10):
    back-to-back single solves of one problem on one stream (in one
    workgroup: its n-vectors fit in LDS; and on the multi-kernel path with
    opts.no_small for comparison), then batches of B independent problems
    (B seeds) through ssnal_en_solve_batch:
    one launch, one workgroup a problem (the default; B = 1 is the same
    problem in one workgroup), and on 8 concurrent workers with the
    multi-kernel path (opts.no_small).  Latency-bound: the design (1.6 MB)
    lives in the caches, so solves/s is the figure, not bandwidth."""
    import torch

    import datagen
    from paper_2006_03970_amd import binding
    from paper_2006_03970_amd.device import design_to_device, vec_to_device

    ctx = binding.Context(0)
    stream = torch.cuda.current_stream()
    nmax = max(batches)
    t0 = time.time()
    probs = []
    for s in range(nmax):
        p = datagen.make_problem("c1", seed=1000 + s)
        A, b = design_to_device(p.AT, "f64"), vec_to_device(p.b)
        probs.append(dict(A=A, b=b, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol,
                          x_out=torch.empty(p.n, dtype=torch.float64, device=A.device)))
    torch.cuda.synchronize()
    print(f"[bench] c1: {nmax} problems generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    q = probs[0]
    for _ in range(5):
        binding.ssnal_en_solve(ctx, q["A"], q["b"], q["lambda1"], q["lambda2"], tol=q["tol"],
                               x_out=q["x_out"], stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(single_reps):
        _, info = binding.ssnal_en_solve(ctx, q["A"], q["b"], q["lambda1"], q["lambda2"], tol=q["tol"],
                                         x_out=q["x_out"], stream=stream)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / single_reps
    out = {"workload": "Gaussian elastic net, m=100, n=2000, k=10, snr=5, alpha=0.5, c_lambda=0.5, "
                       "FP64, tol 1e-10",
           "single": {"solves_per_s": 1.0 / el, "ms_per_solve": el * 1e3, "status": info["status"],
                      "iterations": [info["outer_iters"], info["newton_iters"]], "eta": info["kkt_rel"],
                      "one_workgroup": info["one_workgroup"]},
           "batched": {}}
    print(f"[bench] c1 single: {1.0 / el:.0f} solves/s (one workgroup: {info['one_workgroup']})",
          file=sys.stderr, flush=True)
    multi = binding.make_opts(no_small=1)
    for _ in range(5):
        binding.ssnal_en_solve(ctx, q["A"], q["b"], q["lambda1"], q["lambda2"], tol=q["tol"],
                               x_out=q["x_out"], stream=stream, opts=multi)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(single_reps):
        _, info = binding.ssnal_en_solve(ctx, q["A"], q["b"], q["lambda1"], q["lambda2"], tol=q["tol"],
                                         x_out=q["x_out"], stream=stream, opts=multi)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / single_reps
    out["single_multi_kernel"] = {"solves_per_s": 1.0 / el, "ms_per_solve": el * 1e3, "status": info["status"],
                                  "iterations": [info["outer_iters"], info["newton_iters"]],
                                  "eta": info["kkt_rel"]}
    print(f"[bench] c1 single multi-kernel: {1.0 / el:.0f} solves/s", file=sys.stderr, flush=True)
    binding.ssnal_en_solve_batch(ctx, probs[:64], stream=stream)
    binding.ssnal_en_solve_batch(ctx, probs[:64], stream=stream, opts=binding.make_opts(no_small=1))  # workers
    # the problem descriptors are marshalled before the timed call (host-side
    # preparation, like the upload of the designs); the timed region is the
    # library's batch call
    for B in batches:
        args = binding.batch_args(probs[:B])
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos, rc = binding.solve_batch_args(ctx, args, stream=stream)
        el = time.perf_counter() - t
        out["batched"][str(B)] = {"solves_per_s": B / el, "ms": el * 1e3, "worst_status": rc,
                                  "max_eta": max(infos[i].kkt_rel for i in range(B))}
        print(f"[bench] c1 batch {B}: {B / el:.0f} solves/s", file=sys.stderr, flush=True)
    out["batched"]["launch"] = "one launch, one workgroup per problem"
    out["batched_multi_kernel"] = {}
    for B in batches:
        args = binding.batch_args(probs[:B])
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos, rc = binding.solve_batch_args(ctx, args, stream=stream, opts=binding.make_opts(no_small=1))
        el = time.perf_counter() - t
        out["batched_multi_kernel"][str(B)] = {"solves_per_s": B / el, "ms": el * 1e3, "worst_status": rc}
        print(f"[bench] c1 batch {B} multi-kernel: {B / el:.0f} solves/s", file=sys.stderr, flush=True)
    out["batched_multi_kernel"]["workers"] = 8
    del probs
    torch.cuda.empty_cache()
    return out


def c2_concurrent(ctx, designs, b, p, stream, copies=64, workers=(4, 8)):
    """The same block-Toeplitz solve, `copies` times, through
    ssnal_en_solve_batch on W concurrent workers (own streams): the
    aggregate solves/s when independent solves share the GPU.  One solve is
    latency-bound (its Cholesky steps run on a few CUs), so the single-solve
    rate above is the headline and this is the throughput beside it."""
    import torch

    from paper_2006_03970_amd import binding

    out = {"copies": copies}
    for label, A in designs.items():
        probs = [dict(A=A, b=b, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol,
                      x_out=torch.empty(p.n, dtype=torch.float64, device=A.device)) for _ in range(copies)]
        res = {}
        for w in workers:
            binding.ssnal_en_solve_batch(ctx, probs[:2 * w], stream=stream, workers=w)  # warm the workers
            torch.cuda.synchronize()
            t = time.perf_counter()
            infos, rc = binding.ssnal_en_solve_batch(ctx, probs, stream=stream, workers=w)
            el = time.perf_counter() - t
            res[str(w)] = {"solves_per_s": copies / el, "worst_status": rc,
                           "max_eta": max(i["kkt_rel"] for i in infos)}
            print(f"[bench] c2 concurrent {label} x{w}: {copies / el:.0f} solves/s", file=sys.stderr, flush=True)
        out[label] = res
        del probs
    return out


FP64_PEAK_TFS = 78.6  # MI355X dense FP64 (vector and matrix), published


def chol_roofline(infos, label):
    """FP64 Cholesky factor + solve of the Newton systems inside the timed
    solves that carried events: sum of N^3/3 over the factorisations divided
    by their summed duration, against the FP64 peak."""
    tim = [i for i in infos if i["chol_calls"] > 0]
    calls = sum(i["chol_calls"] for i in tim)
    ms = sum(i["chol_ms"] for i in tim)
    gflop = sum(i["chol_gflop"] for i in tim)
    if not calls or ms <= 0:
        return None
    tfs = gflop / ms  # GFLOP per ms = TFLOP/s
    return {"bound": "fp64", "kernel": f"Cholesky factor + forward/backward solve (k_chol_step x ceil(N/64) "
                                       f"+ k_chol_back) of the Newton systems, {label}",
            "achieved": tfs, "peak": FP64_PEAK_TFS, "unit": "TFLOP/s", "frac": tfs / FP64_PEAK_TFS,
            "calls_per_solve": calls / len(tim), "us_per_call": ms / calls * 1e3,
            "mean_N3_over_3_mflop": gflop / calls * 1e3, "share_of_solve": ms / sum(
                i["solve_ms"] for i in tim)}


SYRK_M, SYRK_R = 4096, 8192  # the largest dense Newton matrix: m x m from r columns
MFMA_PEAK_TFS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}  # MI355X dense MFMA, published


def syrk_bench(reps=5, launches=0):
    """The Newton matrix I + kappa A_J A_J^T at two shapes: the largest dense
    one (m = 4096 rows, r = 8192 active columns) and the first Newton step of
    the m = 1000, n = 1e6 solve (m = 1000 from r = 520000 columns, the
    active set of its first iteration); FP64 storage on FP64 MFMA, FP32 on
    FP32 MFMA, BF16 on BF16 MFMA.  TFLOP/s of the m (m + 1) r flops of the
    triangle against the dense MFMA peak of the storage type.  launches > 0:
    only that many calls per shape and storage type (a short run for
    rocprofv3 counters)."""
    import torch

    from paper_2006_03970_amd import binding

    dev = torch.device("cuda:0")
    ctx = binding.Context(0)
    gen = torch.Generator(device=dev).manual_seed(11)
    out = {}
    for key, (m, r) in (("dense_max", (SYRK_M, SYRK_R)), ("first_newton_step_m1000", (1000, 520000))):
        J = torch.arange(r, dtype=torch.int32, device=dev)
        res = {}
        for store, dt in (("f64", torch.float64), ("f32", torch.float32), ("bf16", torch.bfloat16)):
            A = torch.randn((r, m), generator=gen, device=dev, dtype=torch.float32)
            A = (A / torch.linalg.vector_norm(A, dim=1, keepdim=True)).to(dt)
            if launches:
                for k in range(launches):
                    binding.ssnal_newton_matrix(ctx, A, J, 0.5, 0)
                    print(f"[bench] syrk {key} {store} launch {k}", file=sys.stderr, flush=True)
                del A
                continue
            binding.ssnal_newton_matrix(ctx, A, J, 0.5, 0)
            torch.cuda.synchronize()
            n_rep = reps if m * m * r < 2e11 else 3
            t = time.perf_counter()
            for _ in range(n_rep):
                binding.ssnal_newton_matrix(ctx, A, J, 0.5, 0)
            el = (time.perf_counter() - t) / n_rep
            tfs = m * (m + 1) * r / el / 1e12
            res[store] = {"ms": el * 1e3, "tflops": tfs, "peak_tflops": MFMA_PEAK_TFS[store],
                          "frac": tfs / MFMA_PEAK_TFS[store]}
            print(f"[bench] syrk {key} {store}: {el * 1e3:.2f} ms, {tfs:.1f} TFLOP/s", file=sys.stderr,
                  flush=True)
            del A
        res["shape"] = {"m": m, "r": r, "flops": m * (m + 1) * r}
        out[key] = res
        del J
        torch.cuda.empty_cache()
    return None if launches else out


def _pinned_pool(sizes, chunk=4 << 30):
    """Pinned host buffers for tensors of the given byte sizes, carved out of
    4 GiB pinned chunks (one allocation per chunk; offsets 256-byte aligned).
    Returns a list of uint8 tensors."""
    import torch
    out, cur, off = [], None, 0
    for sz in sizes:
        need = (sz + 255) // 256 * 256
        if cur is None or off + need > cur.numel():
            cur = torch.empty(max(chunk, need), dtype=torch.uint8, pin_memory=True)
            off = 0
        out.append(cur[off:off + sz])
        off += need
    return out


def _latency_stats(lat, alone):
    import numpy as np
    slow = lat / alone
    return {"p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_latency_ms": float(lat.mean() * 1e3),
            "p50_slowdown": float(np.percentile(slow, 50)), "p99_slowdown": float(np.percentile(slow, 99))}


def _open_loop(srv, probs, rate, seed, host):
    """Seeded Poisson arrivals at `rate`; latency = scheduled arrival ->
    completion (for host-resident requests it includes the upload)."""
    import numpy as np
    nreq = len(probs)
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=nreq)
    arrive = np.cumsum(gaps) - gaps[0]
    lat = np.zeros(nreq)
    upload = np.zeros(nreq)
    bad = []
    pending = {}
    start = time.perf_counter()
    nxt = 0
    while nxt < nreq or pending:
        now = time.perf_counter() - start
        while nxt < nreq and arrive[nxt] <= now:
            q = probs[nxt]
            A, b, x = (q["Ah"], q["bh"], q["xh"]) if host else (q["A"], q["b"], q["x"])
            pending[srv.submit(A, b, q["l1"], q["l2"], 1e-6, x)] = nxt
            nxt += 1
        for tk in list(pending):
            info = srv.poll(tk)
            if info is not None:
                k = pending.pop(tk)
                lat[k] = time.perf_counter() - start - arrive[k]
                upload[k] = info["upload_ms"]
                if info["status"] != 0:
                    bad.append(info["status"])
        time.sleep(5e-5)
    return lat, upload, nreq / (time.perf_counter() - start), bad


def serving_bench(nreq, nmax, slots, seed=7, host_requests=128, fp64_subset=128):
    """The serving stream: p50/p99 latency and solves/s of the library's
    serving loop with the designs resident in HBM; then its first
    host_requests requests with their designs in pinned host memory (uploaded
    on admission, latency including the upload), and an FP64 figure on the
    first fp64_subset requests with their stored values upcast exactly.
    Returns (report, state kept for the oracle check of the served results)."""
    import numpy as np
    import torch

    import datagen
    from paper_2006_03970_amd import binding

    reqs = datagen.serving_requests(nreq, seed=seed, n_range=(10_000, int(nmax)))
    t0 = time.time()
    probs = []
    dev = torch.device("cuda:0")
    for q in reqs:
        p = datagen.make_problem_device(q, seed=q["seed"], store=q["store"], device=dev)
        x = torch.empty(p["n"], dtype=torch.float64, device=dev)
        probs.append(dict(A=p["AT"], b=p["b"], l1=p["lam1"], l2=p["lam2"], x=x, m=p["m"], n=p["n"],
                          store=p["store"], design=q["design"]))
    torch.cuda.synchronize()
    print(f"[bench] serving: generated {nreq} requests on the device in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    srv = binding.Server(0, hbm_budget=64 << 30, max_slots=slots)
    out = {"requests": nreq, "slots": slots, "n_range": [10_000, int(nmax)], "m_range": [100, 2000],
           "mean_m": float(np.mean([q["m"] for q in probs])), "mean_n": float(np.mean([q["n"] for q in probs])),
           "stores": {s: sum(1 for q in probs if q["store"] == s) for s in ("f32", "bf16")},
           "admission": "smallest estimated work first among the requests whose footprint fits; "
                        "a request passed over 4 x slots times goes next"}
    try:
        # every request alone (its service time: the slowdown denominators)
        alone = np.zeros(nreq)
        for i, q in enumerate(probs):
            t = time.perf_counter()
            info = srv.wait(srv.submit(q["A"], q["b"], q["l1"], q["l2"], 1e-6, q["x"]))
            alone[i] = time.perf_counter() - t
            assert info["status"] == 0, info
        # closed loop: everything submitted at once
        t = time.perf_counter()
        tickets = [srv.submit(q["A"], q["b"], q["l1"], q["l2"], 1e-6, q["x"]) for q in probs]
        infos = [srv.wait(tk) for tk in tickets]
        sat = nreq / (time.perf_counter() - t)
        bad = [i["status"] for i in infos if i["status"] != 0]
        eta_max = max(i["kkt_rel"] for i in infos)
        lat, _, rate_done, bad2 = _open_loop(srv, probs, 0.8 * sat, seed, host=False)
        out["device_resident"] = {
            "saturated_solves_per_s": sat, "poisson_rate_per_s": 0.8 * sat, "solves_per_s": rate_done,
            **_latency_stats(lat, alone), "alone_latency_ms_mean": float(alone.mean() * 1e3),
            "alone_latency_ms_p50": float(np.percentile(alone, 50) * 1e3),
            "alone_latency_ms_p99": float(np.percentile(alone, 99) * 1e3),
            "max_eta_gpu": eta_max, "nonzero_status": bad + bad2}
        print(f"[bench] serving (HBM-resident): {sat:.0f}/s saturated, p50 "
              f"{out['device_resident']['p50_latency_ms']:.1f} ms p99 {out['device_resident']['p99_latency_ms']:.1f} ms",
              file=sys.stderr, flush=True)
        # served results, kept for the oracle check (the stored bytes go to host memory below)
        xs = [q["x"].cpu() for q in probs]
        if host_requests > 0:
            hp = probs[:host_requests]
            sizes = [q["A"].numel() * q["A"].element_size() for q in hp]
            bufs = _pinned_pool(sizes)
            for q, buf in zip(hp, bufs):
                q["Ah"] = buf.view(q["A"].dtype).view(q["A"].shape)
                q["Ah"].copy_(q["A"])
                q["bh"] = q["b"].cpu().pin_memory()
                q["xh"] = torch.empty(q["n"], dtype=torch.float64).pin_memory()
            torch.cuda.synchronize()
            t = time.perf_counter()
            tickets = [srv.submit(q["Ah"], q["bh"], q["l1"], q["l2"], 1e-6, q["xh"]) for q in hp]
            infos = [srv.wait(tk) for tk in tickets]
            sat_h = len(hp) / (time.perf_counter() - t)
            bad = [i["status"] for i in infos if i["status"] != 0]
            lat, up, rate_done, bad2 = _open_loop(srv, hp, 0.8 * sat_h, seed + 1, host=True)
            same = all(bool(torch.equal(q["xh"], x)) for q, x in zip(hp, xs))
            gb = sum(sizes) / 1e9
            out["host_resident"] = {
                "requests": len(hp),
                "saturated_solves_per_s": sat_h, "poisson_rate_per_s": 0.8 * sat_h, "solves_per_s": rate_done,
                **_latency_stats(lat, alone[:len(hp)]),
                "upload_ms_mean": float(up.mean()), "upload_ms_p99": float(np.percentile(up, 99)),
                "upload_gbs": gb / (up.sum() / 1e3), "design_gb_total": gb,
                "x_bitwise_equal_to_hbm_resident": same, "nonzero_status": bad + bad2,
                "note": "latency from scheduled arrival to completion includes the upload of A, b "
                        "(pinned host memory) on the slot's stream; slowdown is against the request "
                        "alone with its design already in HBM"}
            print(f"[bench] serving (host-resident): {sat_h:.0f}/s saturated, upload "
                  f"{out['host_resident']['upload_gbs']:.1f} GB/s", file=sys.stderr, flush=True)
        # FP64 on the first fp64_subset requests (stored values upcast exactly) beside the
        # mixed solves of the same requests
        sub = probs[:fp64_subset]
        for q in sub:
            q["A64"] = q["A"].to(torch.float64)
            q["Am"] = q["A"]
        torch.cuda.synchronize()
        res = {}
        for key in ("Am", "A64"):
            al = []
            for q in sub:
                t = time.perf_counter()
                info = srv.wait(srv.submit(q[key], q["b"], q["l1"], q["l2"], 1e-6, q["x"]))
                al.append(time.perf_counter() - t)
                assert info["status"] == 0, info
            t = time.perf_counter()
            tk = [srv.submit(q[key], q["b"], q["l1"], q["l2"], 1e-6, q["x"]) for q in sub]
            inf = [srv.wait(k) for k in tk]
            res[key] = {"saturated_solves_per_s": len(sub) / (time.perf_counter() - t),
                        "alone_latency_ms_mean": float(np.mean(al) * 1e3),
                        "max_eta_gpu": max(i["kkt_rel"] for i in inf)}
        out["fp64_vs_mixed_subset"] = {"requests": len(sub), "mixed": res["Am"], "fp64": res["A64"],
                                       "mixed_over_fp64": res["Am"]["saturated_solves_per_s"] /
                                       res["A64"]["saturated_solves_per_s"]}
        for q in sub:
            q.pop("A64")
            q.pop("Am")
        torch.cuda.empty_cache()
    finally:
        srv.close()
    state = {"probs": probs, "xs": xs}
    return out, state


def served_vs_oracle(state, sample, seed=11):
    """Oracle check of served results (part of the CPU-baseline leg): for a
    seeded sample of the served requests that includes m > 1000, n > 3e5 and
    both storage types, the FP64 oracle evaluates on the stored design (the
    exact bytes the GPU read, dequantised) the KKT residual eta of the served
    x, its objective F and the dual objective D at A x - b; F - D bounds the
    objective error (weak duality, lambda2 > 0)."""
    import numpy as np
    import torch

    import oracle

    probs, xs = state["probs"], state["xs"]
    g = np.random.default_rng(seed)
    idx = list(g.choice(len(probs), size=min(sample, len(probs)), replace=False))
    need = [lambda q: q["m"] > 1000, lambda q: q["n"] > 300_000, lambda q: q["store"] == "f32",
            lambda q: q["store"] == "bf16", lambda q: q["m"] > 1000 and q["n"] > 300_000]
    for cond in need:
        if not any(cond(probs[i]) for i in idx):
            cand = [i for i in range(len(probs)) if cond(probs[i]) and i not in idx]
            if cand:
                idx.append(cand[0])
    rows = []
    t0 = time.perf_counter()
    for i in idx:
        q = probs[i]
        AT64 = q["A"].cpu().to(torch.float64).numpy()
        b = q["b"].cpu().numpy()
        x = xs[i].numpy()
        eta = oracle.eta(AT64, b, x, q["l1"], q["l2"])
        F = oracle.primal_obj(AT64, b, x, q["l1"], q["l2"])
        D = oracle.dual_obj(AT64, b, oracle.gemv_n(AT64, x) - b, q["l1"], q["l2"])
        rows.append(dict(i=int(i), m=q["m"], n=q["n"], store=q["store"], eta=eta, rel_gap=(F - D) / abs(D)))
        del AT64
    return {"sample": len(rows), "seconds": time.perf_counter() - t0,
            "max_eta_oracle": max(r["eta"] for r in rows),
            "max_rel_objective_error_bound": max(r["rel_gap"] for r in rows),
            "all_eta_le_tol": all(r["eta"] <= 1e-6 * (1 + 1e-9) for r in rows),
            "largest": max(rows, key=lambda r: r["m"] * r["n"]),
            "covers": {"m_gt_1000": any(r["m"] > 1000 for r in rows),
                       "n_gt_3e5": any(r["n"] > 300_000 for r in rows),
                       "f32": any(r["store"] == "f32" for r in rows),
                       "bf16": any(r["store"] == "bf16" for r in rows)}}


def _host_threads():
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS")
    return max(1, min(n, int(omp))) if omp and omp.isdigit() else n


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(p64, AT32, bits_bf, xs_gpu, serving_state, serving_sample):
    """The FP64 oracle on the host (the CPU baseline), then the oracle's report
    on the GPU's results: per C2 solve, the relative objective error against a
    tight oracle solve (tol 1e-10) on the stored and on the original design,
    the support difference, eta on the stored design and eta on the original;
    and the served-request check."""
    import numpy as np

    import datagen
    import oracle

    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    out = {}
    runs = {}
    for threads, budget, cap in ((1, 10.0, 12), (_host_threads(), 10.0, 64)):
        oracle.set_threads(threads)
        nsolve = 0
        t = time.perf_counter()
        while True:
            oracle.en_solve(p64.AT, p64.b, p64.lam1, p64.lam2, tol=p64.tol)
            nsolve += 1
            if time.perf_counter() - t > budget or nsolve >= cap:
                break
        runs[threads] = (nsolve, time.perf_counter() - t)
        print(f"[bench] oracle on {threads} thread(s): {nsolve / runs[threads][1]:.2f} solves/s",
              file=sys.stderr, flush=True)
    nt = _host_threads()
    n1, e1 = runs[1]
    nn, en = runs[nt]
    out["cpu_baseline"] = {
        "value": nn / en, "unit": "solves/s", "cores": nt, "kind": "oracle",
        "sample": f"{nn} complete FP64 oracle solves of the same problem (tol 1e-6) on {nt} host threads "
                  f"(OpenMP over the A^T y, A x and Newton-matrix loops; every sum in its serial order)",
        "single_thread": {"value": n1 / e1, "cores": 1, "sample": f"{n1} solves on one thread"},
        "cpu_model": _cpu_model()}
    # per-solve parity of the C2 solves
    orig = p64.AT
    stored = {"mixed_f32": AT32.astype(np.float64), "fp64": orig,
              "mixed_bf16": datagen.bf16_bits_to_f64(bits_bf)}
    x_orig, i_orig, _ = oracle.en_solve(orig, p64.b, p64.lam1, p64.lam2, tol=1e-10)
    rep = {}
    for key, x in xs_gpu.items():
        A_s = stored[key]
        if A_s is orig:
            x_s, i_s = x_orig, i_orig
        else:
            x_s, i_s, _ = oracle.en_solve(A_s, p64.b, p64.lam1, p64.lam2, tol=1e-10)
        F_s = oracle.primal_obj(A_s, p64.b, x, p64.lam1, p64.lam2)
        F_o = oracle.primal_obj(orig, p64.b, x, p64.lam1, p64.lam2)
        diff = (x != 0) ^ (x_s != 0)
        rep[key] = {"eta_stored": oracle.eta(A_s, p64.b, x, p64.lam1, p64.lam2),
                    "eta_orig": oracle.eta(orig, p64.b, x, p64.lam1, p64.lam2),
                    "rel_obj_err_stored": abs(F_s - i_s["primal_obj"]) / abs(i_s["primal_obj"]),
                    "rel_obj_err_orig": abs(F_o - i_orig["primal_obj"]) / abs(i_orig["primal_obj"]),
                    "support_diff": int(diff.sum()),
                    "support_diff_above_1e-8": int(np.sum(diff & ((np.abs(x) > 1e-8) | (np.abs(x_s) > 1e-8)))),
                    "nnz": int(np.count_nonzero(x)), "nnz_oracle": int(np.count_nonzero(x_s))}
    out["parity_vs_oracle"] = rep
    if serving_state is not None:
        out["served_vs_oracle"] = served_vs_oracle(serving_state, serving_sample)
    oracle.set_threads(1)
    return out


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
    ap.add_argument("--c3-only", action="store_true", help="run only the m=1000, n=1e6 section")
    ap.add_argument("--no-c1", action="store_true", help="skip the m=100, n=2000 single/batched section")
    ap.add_argument("--c1-only", action="store_true", help="run only the m=100, n=2000 single/batched section")
    ap.add_argument("--c1-reps", type=int, default=200, help="timed single solves of that section")
    ap.add_argument("--serving", type=int, default=512, help="requests in the serving stream (0 = off)")
    ap.add_argument("--serving-host", type=int, default=128,
                    help="requests of the stream (its first ones) also served from pinned host memory (0 = off)")
    ap.add_argument("--serving-oracle-sample", type=int, default=64,
                    help="served requests checked by the oracle in the CPU-baseline leg")
    ap.add_argument("--serving-nmax", type=float, default=5e5)
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--profile-gemv", type=int, default=0)
    ap.add_argument("--profile-copy", type=int, default=0)
    ap.add_argument("--profile-syrk", type=int, default=0,
                    help="only K launches of the m=4096, r=8192 Newton-matrix SYRK per storage type")
    ap.add_argument("--no-syrk", action="store_true", help="skip the Newton-matrix SYRK section")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the concurrent copies of the block-Toeplitz solve")
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
    if args.c3_only:
        print(json.dumps({"large_single_solve": large_bench()}), flush=True)
        return
    if args.c1_only:
        print(json.dumps({"small_single_solve": c1_bench(single_reps=args.c1_reps)}), flush=True)
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
    bits_bf = datagen.f32_to_bf16_bits(AT32)
    Abf = design_to_device(bits_bf, "bf16")

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
    elbf, infbf, xbf = timed(Abf, "mixed bf16")

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

    # measured stream bandwidths on this GPU over the FP32 design's bytes: a
    # read-only stream (torch's sum over the array) and a device-to-device
    # copy (bytes read + bytes written over the copy time)
    src = A32.reshape(-1)
    dst = torch.empty_like(src)
    nbytes = src.numel() * src.element_size()
    nrep = 20

    def stream_rate(fn, moved):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(nrep):
            fn()
        torch.cuda.synchronize()
        return moved * nrep / (time.perf_counter() - t) / 1e9

    stream_gbs = stream_rate(lambda: src.sum(), nbytes)
    copy_gbs = stream_rate(lambda: dst.copy_(src), 2.0 * nbytes)
    del dst

    def solve_gbs(infos, el, s_a):
        """Effective solve bandwidth: full A^T v passes per solve x m n s_A / solve time."""
        passes = sum(i["gemv_calls"] for i in infos) / len(infos)
        return passes * float(p64.m) * p64.n * s_a / (el / args.steps) / 1e9, passes
    csrc = os.path.join(ROOT, "paper_2006_03970_amd", "csrc")
    traffic = _traffic_from_profile([os.path.join(csrc, "k_gemv.hip"), os.path.join(csrc, "common.hpp")], "f32")

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
        "stream_read_gbs": stream_gbs,
        "stream_copy_gbs": copy_gbs,
        "atd_frac_of_stream": {"mixed_f32": achieved / stream_gbs, "fp64": bpl64 / avg64 / 1e9 / stream_gbs,
                               "mixed_bf16": bplbf / avgbf / 1e9 / stream_gbs},
        "effective_solve_gbs": {k: {"gbs": g, "passes_per_solve": ps} for k, (g, ps) in
                                (("mixed_f32", solve_gbs(inf32, el32, 4)), ("fp64", solve_gbs(inf64, el64, 8)),
                                 ("mixed_bf16", solve_gbs(infbf, elbf, 2)))},
        "roofline": {
            "bound": "hbm",
            "kernel": "Newton pass w_d = A^T d: k_gemv_t<float, float, 2> (FP32 design, FP32 accumulation)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": bpl32, "avg_launch_us": avg32 * 1e6,
        },
    }

    out["roofline_chol"] = chol_roofline(inf32, "FP32-stored design (FP64 factor)")
    out["roofline_chol_fp64"] = chol_roofline(inf64, "FP64 design")
    if not args.no_concurrent:
        out["concurrent"] = c2_concurrent(ctx, {"mixed_f32": A32, "fp64": A64}, b, p64, stream)
    xs_gpu = {"mixed_f32": x32.cpu().numpy(), "fp64": x64.cpu().numpy(), "mixed_bf16": xbf.cpu().numpy()}
    del A64, Abf
    torch.cuda.empty_cache()

    if not args.no_c1:
        out["small_single_solve"] = c1_bench(single_reps=args.c1_reps)
    if not args.no_c3:
        out["large_single_solve"] = large_bench()
    if not args.no_path:
        out["path"] = path_bench()
    if not args.no_cg:
        out["newton_cg"] = cg_bench()
    if not args.no_syrk:
        out["newton_matrix_syrk"] = syrk_bench()
    serving_state = None
    if args.serving > 0:
        out["serving"], serving_state = serving_bench(args.serving, args.serving_nmax, args.serving_slots,
                                                      host_requests=args.serving_host)

    if not args.no_cpu_baseline:
        out.update(cpu_baseline_leg(p64, AT32, bits_bf, xs_gpu, serving_state, args.serving_oracle_sample))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
