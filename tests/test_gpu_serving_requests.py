"""Served requests against the FP64 oracle, host-resident requests, warm-started
path points submitted as requests, and the batch entry's workers (the serving
form of the solver; Sec. 3.3 for the warm starts)."""
import math

import numpy as np
import pytest

from tests.certify import check_eta

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu):
    return gpu.Context(0)


def _rel_obj(F, Fr):
    return abs(F - Fr) / abs(Fr)


def _stream_requests():
    """Requests with the serving workload's distributions (Gaussian-Toeplitz or
    SNP-like designs, alpha ~ U[0.2, 0.9], c_lambda ~ U[0.05, 0.8], FP32 or BF16
    storage, tol 1e-6) at sizes the oracle solves in seconds, plus one with
    m > 1000 rows in each storage type."""
    import datagen
    reqs = datagen.serving_requests(8, seed=91, m_range=(100, 600), n_range=(10_000, 60_000))
    big = datagen.serving_requests(2, seed=92, m_range=(1100, 1300), n_range=(30_000, 40_000))
    big[0]["store"], big[1]["store"] = "f32", "bf16"
    return reqs + big


def test_served_requests_vs_oracle(gpu, orc):
    """Ten requests served concurrently on four slots: each served x meets
    eta <= tol in the FP64 oracle's evaluation on the stored (dequantised)
    design, the server's reported eta is the oracle's to rounding, and the
    objective is within 1e-8 (relative) of a tight oracle solve on the same
    stored design."""
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    reqs = _stream_requests()
    probs = []
    for q in reqs:
        p = datagen.make_problem(q, seed=q["seed"], store=q["store"])
        A, b = design_to_device(p.AT, p.store), vec_to_device(p.b)
        x = torch.full((p.n,), float("nan"), dtype=torch.float64, device=A.device)
        probs.append((p, A, b, x))
    _say("served requests vs oracle:", [(p.m, p.n, p.store) for p, *_ in probs])
    srv = gpu.Server(0, hbm_budget=8 << 30, max_slots=4)
    try:
        tickets = [srv.submit(A, b, p.lam1, p.lam2, p.tol, x) for p, A, b, x in probs]
        infos = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    torch.cuda.synchronize()
    worst_eta, worst_rel = 0.0, 0.0
    for (p, A, b, x), info in zip(probs, infos):
        assert info["status"] == 0, info
        xs = x.cpu().numpy()
        # the oracle reads the bytes the GPU consumed, dequantised exactly
        AT64 = A.to(torch.float64).cpu().numpy()
        assert np.array_equal(AT64, p.AT64)
        eta = check_eta(orc, AT64, p.b, xs, p.lam1, p.lam2, p.tol, eta_gpu=info["kkt_rel"])
        xr, ir, _ = orc.en_solve(AT64, p.b, p.lam1, p.lam2, tol=1e-10)
        assert ir["status"] == 0
        rel = _rel_obj(orc.primal_obj(AT64, p.b, xs, p.lam1, p.lam2), ir["primal_obj"])
        assert rel <= 1e-8, (p.m, p.n, p.store, rel)
        worst_eta, worst_rel = max(worst_eta, eta), max(worst_rel, rel)
    print(f"[report] served vs oracle: max eta {worst_eta:.3e}, max rel objective error {worst_rel:.3e}")


def test_server_host_resident_bitwise(gpu, ctx):
    """Host-resident requests (pinned host memory; the server uploads A, b and
    x0 on admission and writes x back) in a mix with device-resident ones on
    three slots give the bits of the same solves run alone on the device, one
    of them warm-started and one with a padded leading dimension."""
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    reqs = datagen.serving_requests(6, seed=93, m_range=(100, 500), n_range=(10_000, 50_000))
    _say("host-resident requests in the mix")
    items = []
    for i, q in enumerate(reqs):
        p = datagen.make_problem(q, seed=q["seed"], store=q["store"])
        lda = p.m + 3 if i == 2 else None
        A, b = design_to_device(p.AT, p.store, lda=lda), vec_to_device(p.b)
        x0 = None
        if i == 4:  # warm start from a perturbed cold solution
            xc, _ = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, m=p.m)
            x0 = (xc * 0.9).contiguous()
        host = i % 2 == 0
        # a host-resident design is uploaded packed (leading dimension m): the
        # reference solve reads the packed design too
        Aref = A[:, :p.m].contiguous() if host else A
        xa, info = gpu.ssnal_en_solve(ctx, Aref, b, p.lam1, p.lam2, x0=x0, tol=p.tol, m=p.m)
        assert info["status"] == 0
        items.append(dict(p=p, A=A, b=b, x0=x0, alone=xa.clone(), host=host))
    torch.cuda.synchronize()
    srv = gpu.Server(0, hbm_budget=8 << 30, max_slots=3)
    try:
        tickets = []
        for it in items:
            p = it["p"]
            if it["host"]:
                A = it["A"].cpu().pin_memory()
                b = it["b"].cpu().pin_memory()
                x0 = None if it["x0"] is None else it["x0"].cpu().pin_memory()
                x = torch.full((p.n,), float("nan"), dtype=torch.float64).pin_memory()
            else:
                A, b, x0 = it["A"], it["b"], it["x0"]
                x = torch.full((p.n,), float("nan"), dtype=torch.float64, device=A.device)
            it["x"] = x
            it["foot"] = gpu.srv_footprint(A, m=p.m)
            tickets.append(srv.submit(A, b, p.lam1, p.lam2, p.tol, x, x0=x0, m=p.m))
        infos = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    torch.cuda.synchronize()
    for it, info in zip(items, infos):
        assert info["status"] == 0, info
        assert bool((it["x"].to(it["alone"].device) == it["alone"]).all())
        assert info["queue_ms"] >= 0.0
        p = it["p"]
        ws = gpu.workspace_bytes(p.m, p.n)
        if it["host"]:
            assert info["upload_ms"] > 0.0
            s_a = {"f64": 8, "f32": 4, "bf16": 2}[p.store]
            assert it["foot"] == ws + p.m * p.n * s_a + (p.m + p.n) * 8
        else:
            assert info["upload_ms"] == 0.0 and it["foot"] == ws


def test_server_path_points_as_requests(gpu, ctx):
    """A warm-started lambda path submitted point by point (x0 = the previous
    point's served x, sigma0 = its final sigma capped as ssnal_en_path caps it)
    while other requests run on the other slots gives the bits of
    ssnal_en_path."""
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    p = datagen.make_problem(dict(m=300, n=40_000, design="snp", k=20, snr=5.0, alpha=0.7, c_lam=1.0,
                                  tol=1e-6), seed=94, store="f32")
    A, b = design_to_device(p.AT, p.store), vec_to_device(p.b)
    alpha = 0.7
    grid = datagen.path_grid(8, lo=0.1)
    _say("path points as served requests")
    X, pinfos, rc = gpu.ssnal_en_path(ctx, A, b, alpha, grid, tol=1e-6)
    assert rc == 0
    amax = float(torch.max(torch.abs(gpu.ssnal_gemv_t(ctx, A, b, acc64=True))))
    lam_max = amax / alpha
    others = datagen.serving_requests(6, seed=95, m_range=(100, 400), n_range=(10_000, 40_000))
    oth = []
    for q in others:
        po = datagen.make_problem(q, seed=q["seed"], store=q["store"])
        oth.append((po, design_to_device(po.AT, po.store), vec_to_device(po.b)))
    torch.cuda.synchronize()
    srv = gpu.Server(0, hbm_budget=8 << 30, max_slots=3)
    try:
        xs, x0, sig, cap = [], None, 0.0, None
        busy = []
        for k, c in enumerate(grid):
            # keep the other slots busy while the point runs
            po, Ao, bo = oth[k % len(oth)]
            xo = torch.empty(po.n, dtype=torch.float64, device=Ao.device)
            busy.append(srv.submit(Ao, bo, po.lam1, po.lam2, po.tol, xo))
            lam = c * lam_max
            x = torch.full((p.n,), float("nan"), dtype=torch.float64, device=A.device)
            info = srv.wait(srv.submit(A, b, alpha * lam, (1.0 - alpha) * lam, 1e-6, x, x0=x0,
                                       sigma0=sig))
            assert info["status"] == 0, (k, info)
            if cap is None:  # the same products as the path's cap, in the same order
                cap = info["sigma0"] * 5.0 * 5.0 * 5.0 * 5.0
            sig = min(info["sigma_final"], cap)
            x0 = x
            xs.append(x)
        for t in busy:
            assert srv.wait(t)["status"] == 0
    finally:
        srv.close()
    torch.cuda.synchronize()
    for k in range(len(grid)):
        assert bool((xs[k] == X[k]).all()), k
        assert pinfos[k]["newton_iters"] >= 0


def test_server_ready_event(gpu):
    """A request whose design and response were written on a side stream is
    submitted without a host synchronisation: the event the binding records
    orders the solve after those writes."""
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    q = datagen.serving_requests(1, seed=96, m_range=(200, 300), n_range=(20_000, 30_000))[0]
    p = datagen.make_problem(q, seed=q["seed"], store=q["store"])
    A0, b0 = design_to_device(p.AT, p.store), vec_to_device(p.b)
    ctx = gpu.Context(0)
    xa, _ = gpu.ssnal_en_solve(ctx, A0, b0, p.lam1, p.lam2, tol=p.tol)
    torch.cuda.synchronize()
    _say("ready event")
    side = torch.cuda.Stream()
    srv = gpu.Server(0, hbm_budget=4 << 30, max_slots=2)
    try:
        with torch.cuda.stream(side):
            A = torch.empty_like(A0)
            b = torch.empty_like(b0)
            A.copy_(A0)
            b.copy_(b0)
            x = torch.full((p.n,), float("nan"), dtype=torch.float64, device=A0.device)
            t = srv.submit(A, b, p.lam1, p.lam2, p.tol, x)
        info = srv.wait(t)
    finally:
        srv.close()
    torch.cuda.synchronize()
    assert info["status"] == 0
    assert bool((x == xa).all())


def test_server_refuses_bad_requests(gpu):
    """Mixed host/device arrays and an oversized host request are refused at
    submission."""
    import torch
    srv = gpu.Server(0, hbm_budget=64 << 20, max_slots=1)
    try:
        A = torch.zeros((100_000, 200), dtype=torch.float32).pin_memory()  # 80 MB > budget
        b = torch.zeros(200, dtype=torch.float64).pin_memory()
        x = torch.zeros(100_000, dtype=torch.float64).pin_memory()
        with pytest.raises(gpu.SsnalError):
            srv.submit(A, b, 0.1, 0.1, 1e-6, x)
        with pytest.raises(AssertionError):
            srv.submit(A[:10], b.cuda(), 0.1, 0.1, 1e-6, x[:10])
    finally:
        srv.close()


@pytest.mark.parametrize("workers", [1, 3, 8])
def test_batch_workers_bitwise(gpu, ctx, workers):
    """The batch entry on 1, 3 and 8 concurrent workers gives the bits of each
    problem solved alone (small Gaussian problems of the single-solve
    workload's shape, two with their own sigma0), on the multi-kernel path
    (opts.no_small; in one workgroup a batch takes no workers)."""
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("batch workers", workers)
    probs, alone = [], []
    for s in range(10):
        p = datagen.make_problem("c1", seed=200 + s)
        A, b = design_to_device(p.AT, "f64"), vec_to_device(p.b)
        sig = 0.05 if s in (3, 7) else 0.0
        opts = gpu.make_opts(sigma0=sig, no_small=1) if sig else gpu.make_opts(no_small=1)
        xa, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, opts=opts)
        assert info["status"] == 0
        alone.append(xa.clone())
        probs.append(dict(A=A, b=b, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol, sigma0=sig,
                          x_out=torch.full((p.n,), float("nan"), dtype=torch.float64, device=A.device)))
    infos, rc = gpu.ssnal_en_solve_batch(ctx, probs, opts=gpu.make_opts(no_small=1), workers=workers)
    torch.cuda.synchronize()
    assert rc == 0
    for q, xa, info in zip(probs, alone, infos):
        assert info["status"] == 0
        assert bool((q["x_out"] == xa).all())
    assert math.isclose(infos[3]["sigma0"], 0.05) and math.isclose(infos[7]["sigma0"], 0.05)
