"""Path, batch and serving entry points through the C ABI (warm starts of
Sec. 3.3; the serving loop's bitwise alone-vs-mix property)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu):
    return gpu.Context(0)


def _upload(p):
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    return design_to_device(p.AT, p.store), vec_to_device(p.b)


def _oracle_path(orc, AT64, b, alpha, grid, tol):
    """Warm-started oracle path over lam_k = c_k * ||A^T b||_inf / alpha, each
    point starting from the previous point's x and final sigma, the sigma
    capped at 5^4 times the cold default 2.5 / mean_j |a_j|^2."""
    lam_max = float(np.max(np.abs(orc.gemv_t(AT64, b)))) / alpha
    cap = 625.0 * 2.5 / float(np.mean(np.sum(np.asarray(AT64, dtype=np.float64) ** 2, axis=1)))
    xs, infos, x0, sig = [], [], None, None
    for c in grid:
        lam = c * lam_max
        kw = {"sigma0": sig} if sig else {}
        x, info, _ = orc.en_solve(AT64, b, alpha * lam, (1 - alpha) * lam, tol=tol, x0=x0, **kw)
        xs.append(x)
        infos.append(info)
        x0, sig = x, min(info["sigma_final"], cap)
    return lam_max, xs, infos


def test_path_small_fp64_vs_oracle(gpu, ctx, orc):
    """SNP-like m=120, n=1500, alpha=0.7, 12 points from c=1 (x=0) down to 0.05,
    tol 1e-10: every point matches the warm-started oracle path."""
    import datagen
    p = datagen.make_problem(dict(m=120, n=1500, design="snp", k=10, snr=5.0, alpha=0.7,
                                  c_lam=1.0, tol=1e-10), seed=5)
    grid = np.geomspace(1.0, 0.05, 12)
    _say("path small fp64")
    A, b = _upload(p)
    X, infos, rc = gpu.ssnal_en_path(ctx, A, b, 0.7, grid, tol=1e-10)
    assert rc == 0, infos
    X = X.cpu().numpy()
    lam_max, xr, ir = _oracle_path(orc, p.AT, p.b, 0.7, grid, 1e-10)
    assert np.count_nonzero(X[0]) == 0  # c = 1 is lambda_max: the zero solution (pin P5)
    for k, c in enumerate(grid):
        lam = c * lam_max
        l1, l2 = 0.7 * lam, 0.3 * lam
        assert infos[k]["status"] == 0, (k, infos[k])
        assert orc.eta(p.AT, p.b, X[k], l1, l2) <= 1e-10, k
        F = orc.primal_obj(p.AT, p.b, X[k], l1, l2)
        Fr = orc.primal_obj(p.AT, p.b, xr[k], l1, l2)
        assert abs(F - Fr) <= 1e-10 * abs(Fr), (k, F, Fr)
        np.testing.assert_allclose(X[k], xr[k], rtol=0, atol=1e-7 * (1 + np.max(np.abs(xr[k]))))


@pytest.mark.parametrize("store,alpha", [("f32", 0.7), ("f64", 0.3)])
def test_path_snp_full_size(gpu, ctx, orc, store, alpha):
    """m=500, n=200000 SNP-like design, 100 points c = 1 .. 0.01 (log), tol 1e-6:
    every point is certified (eta <= 1e-6 with FP64 accumulation over the
    stored design), warm starts keep points to one or two outer iterations,
    and three sampled points match a cold oracle solve."""
    import datagen
    p = datagen.make_problem("c4", seed=2, store=store, alpha=alpha)
    grid = datagen.path_grid(100, 0.01, 1.0)
    _say("path c4", store, "alpha", alpha)
    A, b = _upload(p)
    X, infos, rc = gpu.ssnal_en_path(ctx, A, b, alpha, grid, tol=1e-6)
    assert rc == 0, [i["status"] for i in infos]
    assert all(i["status"] == 0 and i["kkt_rel"] <= 1e-6 for i in infos)
    outer = np.array([i["outer_iters"] for i in infos])
    newton = np.array([i["newton_iters"] for i in infos])
    # warm starts: at most two multiplier updates at the median point and a few
    # Newton steps per point (a cold solve takes 3-5 updates)
    assert np.median(outer[1:]) <= 2, outer
    assert newton.sum() <= 6 * len(grid), newton
    lam_max = float(np.max(np.abs(orc.gemv_t(p.AT64, p.b)))) / alpha
    assert abs(lam_max - p.lam_max) <= 1e-6 * p.lam_max  # FP32 storage moves it slightly
    Xh = X.cpu().numpy()
    for k in (10, 55, 99):
        lam = grid[k] * lam_max
        l1, l2 = alpha * lam, (1 - alpha) * lam
        assert orc.eta(p.AT64, p.b, Xh[k], l1, l2) <= 1e-6, k
        xr, ir, _ = orc.en_solve(p.AT64, p.b, l1, l2, tol=1e-9)
        F = orc.primal_obj(p.AT64, p.b, Xh[k], l1, l2)
        assert abs(F - ir["primal_obj"]) <= 1e-6 * abs(ir["primal_obj"]), (k, F, ir["primal_obj"])


def test_path_truncation_and_errors(gpu, ctx):
    import datagen
    p = datagen.make_problem("c1", seed=3)
    A, b = _upload(p)
    grid = np.geomspace(1.0, 0.01, 20)
    _say("path truncation")
    X, infos, rc = gpu.ssnal_en_path(ctx, A, b, 0.5, grid, tol=1e-8, max_active=5)
    assert rc == 3  # SSNAL_PATH_TRUNCATED
    k = next(i for i, inf in enumerate(infos) if inf["nnz"] > 5)
    assert all(inf["status"] == 3 for inf in infos[k + 1:])
    Xh = X.cpu().numpy()
    assert np.all(Xh[k + 1:] == 0)
    assert np.count_nonzero(Xh[k]) > 5
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_path(ctx, A, b, 1.5, grid)  # alpha outside (0, 1]
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_path(ctx, A, b, 0.5, [1.0, -0.1])


def _problems(gpu, n_prob, seed0=20):
    import datagen
    import torch
    probs, keep = [], []
    for i in range(n_prob):
        # the third (FP64, m = 120, n = 3000) is past the single-solve limits
        # of the one-workgroup path (m n > 2^17, n-vectors too large for LDS)
        cfg = dict(m=80 + 20 * i, n=(1500, 1750, 3000, 2250, 2500, 2750)[i % 6],
                   design=("gauss", "toeplitz", "snp")[i % 3], k=8,
                   snr=5.0, alpha=0.5, c_lam=0.3 + 0.1 * (i % 3), tol=1e-8)
        p = datagen.make_problem(cfg, seed=seed0 + i, store=("f64", "f32")[i % 2])
        A, b = _upload(p)
        x = torch.empty(p.n, dtype=torch.float64, device=A.device)
        probs.append(dict(A=A, b=b, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol, x_out=x))
        keep.append(p)
    return probs, keep


def test_batch_matches_individual_bitwise(gpu, ctx):
    """A batch gives each problem's bits alone when both take the same path
    (FP32 storage and small FP64 problems); an FP64 problem past the
    single-solve limits of the one-workgroup path (m = 120, n = 3000) runs
    in one workgroup only in the batch and agrees to 1e-9."""
    _say("batch vs individual")
    probs, _ = _problems(gpu, 4)
    alone = []
    for q in probs:
        x, info = gpu.ssnal_en_solve(ctx, q["A"], q["b"], q["lambda1"], q["lambda2"], tol=q["tol"])
        assert info["status"] == 0
        alone.append((x.clone(), info["one_workgroup"]))
    infos, rc = gpu.ssnal_en_solve_batch(ctx, probs)
    assert rc == 0
    assert [i["one_workgroup"] for i in infos] == [1, 0, 1, 0]
    assert [ow for _, ow in alone] == [1, 0, 0, 0]
    for q, (xa, ow), info in zip(probs, alone, infos):
        if ow == info["one_workgroup"]:
            assert bool((q["x_out"] == xa).all())
        else:
            assert float((q["x_out"] - xa).abs().max()) <= 1e-9


def test_server_bitwise_alone_vs_mix(gpu, ctx):
    """Six requests of different shapes and storage types in flight on three
    slots give the same bits as each solved alone."""
    import torch
    _say("server mix")
    probs, _ = _problems(gpu, 6, seed0=40)
    alone = []
    for q in probs:
        x, info = gpu.ssnal_en_solve(ctx, q["A"], q["b"], q["lambda1"], q["lambda2"], tol=q["tol"])
        assert info["status"] == 0
        alone.append(x.clone())
        q["x_out"].fill_(float("nan"))
    torch.cuda.synchronize()
    srv = gpu.Server(0, hbm_budget=4 << 30, max_slots=3)
    try:
        tickets = [srv.submit(q["A"], q["b"], q["lambda1"], q["lambda2"], q["tol"], q["x_out"])
                   for q in probs]
        infos = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    torch.cuda.synchronize()
    assert all(i["status"] == 0 for i in infos)
    for q, xa in zip(probs, alone):
        assert bool((q["x_out"] == xa).all())


def test_server_admission_budget(gpu):
    """A budget that fits one request at a time still completes every request
    (they queue); a request larger than the budget is refused at submit."""
    import torch
    _say("server budget")
    probs, _ = _problems(gpu, 3, seed0=60)
    need = max(gpu.workspace_bytes(q["A"].shape[1], q["A"].shape[0]) for q in probs)
    srv = gpu.Server(0, hbm_budget=need + need // 2, max_slots=3)
    try:
        tickets = [srv.submit(q["A"], q["b"], q["lambda1"], q["lambda2"], q["tol"], q["x_out"])
                   for q in probs]
        assert all(srv.wait(t)["status"] == 0 for t in tickets)
        with pytest.raises(gpu.SsnalError):
            srv.wait(tickets[0])  # collected already
    finally:
        srv.close()
    small = gpu.Server(0, hbm_budget=1 << 20, max_slots=1)
    try:
        q = probs[0]
        with pytest.raises(gpu.SsnalError):
            small.submit(q["A"], q["b"], q["lambda1"], q["lambda2"], q["tol"], q["x_out"])
    finally:
        small.close()
    torch.cuda.synchronize()


def test_concurrent_solves_bitwise(gpu):
    """Sixteen requests of the serving workload's shapes solved by four host
    threads at once (own context and stream each) and through a four-slot
    server equal the solves run alone, bit for bit.  Regression test for a
    race in which a Cholesky panel workgroup dispatched late (other streams
    holding the CUs) read a diagonal tile already overwritten by the
    factor."""
    import threading
    import datagen
    import torch
    _say("concurrent solves")
    dev = torch.device("cuda:0")
    reqs = datagen.serving_requests(16, seed=7, m_range=(100, 700), n_range=(20_000, 200_000))
    probs = [datagen.make_problem_device(q, seed=q["seed"], store=q["store"], device=dev) for q in reqs]
    torch.cuda.synchronize()
    ctx = gpu.Context(0)
    alone = []
    for p in probs:
        x, info = gpu.ssnal_en_solve(ctx, p["AT"], p["b"], p["lam1"], p["lam2"], tol=1e-6)
        assert info["status"] == 0, info
        alone.append(x.clone())
    torch.cuda.synchronize()
    outs = [None] * len(probs)
    errs = []
    nxt = [0]
    lock = threading.Lock()

    def worker():
        c = gpu.Context(0)
        st = torch.cuda.Stream(device=dev)
        while True:
            with lock:
                i = nxt[0]
                nxt[0] += 1
            if i >= len(probs):
                return
            p = probs[i]
            with torch.cuda.stream(st):
                x = torch.empty(p["n"], dtype=torch.float64, device=dev)
                try:
                    gpu.ssnal_en_solve(c, p["AT"], p["b"], p["lam1"], p["lam2"], tol=1e-6, x_out=x,
                                       stream=st)
                    st.synchronize()
                    outs[i] = x
                except gpu.SsnalError as e:
                    errs.append((i, str(e)))

    threads = [threading.Thread(target=worker) for _ in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    assert not errs, errs
    for i, xa in enumerate(alone):
        assert bool((outs[i] == xa).all()), i
    xs = [torch.full((p["n"],), float("nan"), dtype=torch.float64, device=dev) for p in probs]
    torch.cuda.synchronize()
    srv = gpu.Server(0, hbm_budget=16 << 30, max_slots=4)
    try:
        tickets = [srv.submit(p["AT"], p["b"], p["lam1"], p["lam2"], 1e-6, x) for p, x in zip(probs, xs)]
        assert all(srv.wait(t)["status"] == 0 for t in tickets)
    finally:
        srv.close()
    torch.cuda.synchronize()
    for i, xa in enumerate(alone):
        assert bool((xs[i] == xa).all()), i


def test_server_long_rows_cg_in_mix(gpu, ctx):
    """A request with m = 5000 > 4096 rows (its first Newton steps take
    conjugate-gradient directions) among small ones on three slots gives the
    same bits as each solved alone."""
    import datagen
    import torch
    _say("server mix with a Newton-CG request")
    probs, _ = _problems(gpu, 4, seed0=70)
    p = datagen.make_problem(dict(m=5000, n=30000, design="gauss", k=20, snr=5.0, alpha=0.5, c_lam=0.05,
                                  tol=1e-6), seed=71, store="f32")
    A, b = _upload(p)
    probs.insert(1, dict(A=A, b=b, lambda1=p.lam1, lambda2=p.lam2, tol=p.tol,
                         x_out=torch.empty(p.n, dtype=torch.float64, device=A.device)))
    alone = []
    for q in probs:
        x, info = gpu.ssnal_en_solve(ctx, q["A"], q["b"], q["lambda1"], q["lambda2"], tol=q["tol"])
        assert info["status"] == 0
        alone.append(x.clone())
        q["x_out"].fill_(float("nan"))
    torch.cuda.synchronize()
    srv = gpu.Server(0, hbm_budget=8 << 30, max_slots=3)
    try:
        tickets = [srv.submit(q["A"], q["b"], q["lambda1"], q["lambda2"], q["tol"], q["x_out"])
                   for q in probs]
        infos = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    torch.cuda.synchronize()
    assert all(i["status"] == 0 for i in infos)
    assert infos[1]["cg_iters"] > 0
    for q, xa in zip(probs, alone):
        assert bool((q["x_out"] == xa).all())
