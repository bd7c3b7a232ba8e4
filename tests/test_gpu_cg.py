"""Newton-CG (Sec. 3.2: conjugate gradients on eq. newton_direction when m and
r are large) through the C ABI against the FP64 oracle: the A^T v pass over
columns longer than one register-resident slice, single CG directions (small,
and long columns with row panels), whole solves with CG forced, and the
automatic switch to CG at m, r > 4096 certified by the oracle's KKT residual
and duality gap."""
import numpy as np
import pytest

from tests.certify import check_eta

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu):
    return gpu.Context(0)


def _design(m, n, store, seed, lda=None):
    """Gaussian columns of squared norm ~m, as stored (FP64 values of the
    stored design); lda > m pads every column with NaN rows."""
    import datagen
    from paper_2006_03970_amd.device import design_to_device
    AT = np.random.default_rng(seed).standard_normal((n, m))
    if store == "f64":
        return design_to_device(AT, "f64", lda=lda), AT
    AT32 = AT.astype(np.float32)
    if store == "f32":
        return design_to_device(AT32, "f32", lda=lda), AT32.astype(np.float64)
    bits = datagen.f32_to_bf16_bits(AT32)
    return design_to_device(bits, "bf16", lda=lda), datagen.bf16_bits_to_f64(bits)


@pytest.mark.parametrize("m,n,store,lda", [(5000, 3000, "f32", None), (5001, 700, "f32", None),
                                           (5001, 900, "f32", 5004), (9000, 2000, "bf16", None),
                                           (3000, 2500, "f64", None), (4100, 1500, "f64", 4102)])
def test_gemv_long_columns(gpu, ctx, orc, m, n, store, lda):
    """Row panels of A^T v (NaN padding rows never reach a result): every
    entry within the accumulation error bound."""
    from paper_2006_03970_amd.device import vec_to_device
    _say("gemv long", m, n, store, lda)
    A, ATs = _design(m, n, store, seed=m + n, lda=lda)
    v = np.random.default_rng(7).standard_normal(m)
    ref = orc.gemv_t(ATs, v)
    mag = np.abs(ATs) @ np.abs(v)
    for acc64 in (False, True):
        w = gpu.ssnal_gemv_t(ctx, A, vec_to_device(v), acc64=acc64, m=m).cpu().numpy()
        u = 2.0 ** -53 if (acc64 or store == "f64") else 2.0 ** -24
        assert np.all(np.abs(w - ref) <= (2 * m + 4) * u * mag), (acc64, np.max(np.abs(w - ref) / mag))


@pytest.mark.parametrize("m,n,r,store,kappa,eps", [
    (300, 2000, 500, "f64", 0.05, 1e-12),
    (300, 2000, 120, "f64", 0.05, 1e-3),
    (5000, 8000, 4500, "f32", 5e-4, 1e-10),
    (4500, 6000, 5000, "f64", 5e-4, 1e-3),
])
def test_cg_direction_vs_oracle(gpu, ctx, orc, m, n, r, store, kappa, eps):
    """Run tight, the direction matches the oracle's; at a loose eps both stop
    within one iteration of each other and the residual meets the test."""
    import torch
    from paper_2006_03970_amd.device import vec_to_device
    _say("cg direction", m, n, r, store, eps)
    A, ATs = _design(m, n, store, seed=3 * m + r)
    rng = np.random.default_rng(m + r)
    J = np.sort(rng.choice(n, r, replace=False)).astype(np.int32)
    g = rng.standard_normal(m)
    d, it = gpu.ssnal_newton_cg(ctx, A, torch.from_numpy(J).cuda(), kappa, vec_to_device(g), eps,
                                maxit=500)
    d = d.cpu().numpy()
    d_ref, it_ref = orc.newton_cg(ATs, J, kappa, g, eps, maxit=500)
    assert it < 500 and it_ref < 500
    if eps < 1e-8:
        assert np.linalg.norm(d - d_ref) <= 1e-8 * np.linalg.norm(d_ref)
    else:
        assert abs(it - it_ref) <= 1
        res = orc.newton_matvec(ATs, J, kappa, d) + g
        assert np.linalg.norm(res) <= eps * np.linalg.norm(g) * (1 + 1e-6)
    assert g @ d < 0


def test_cg_direction_edge_cases(gpu, ctx, orc):
    """r = 0 gives d = -g; maxit = 0 gives d = 0; a single column terminates
    within two iterations (two distinct eigenvalues)."""
    import torch
    from paper_2006_03970_amd.device import vec_to_device
    _say("cg edge cases")
    A, ATs = _design(64, 100, "f64", seed=5)
    g = np.random.default_rng(6).standard_normal(64)
    J0 = torch.zeros(1, dtype=torch.int32, device="cuda")[:0]
    d, it = gpu.ssnal_newton_cg(ctx, A, J0, 0.5, vec_to_device(g), 1e-6)
    assert it == 0 and np.array_equal(d.cpu().numpy(), -g)
    J = torch.tensor([17], dtype=torch.int32, device="cuda")
    d, it = gpu.ssnal_newton_cg(ctx, A, J, 0.5, vec_to_device(g), 1e-6, maxit=0)
    assert it == 0 and np.all(d.cpu().numpy() == 0.0)
    d, it = gpu.ssnal_newton_cg(ctx, A, J, 0.5, vec_to_device(g), 1e-12)
    assert it <= 2
    d_ch = orc.newton_direction(ATs, np.array([17], dtype=np.int32), 0.5, g)
    assert np.linalg.norm(d.cpu().numpy() - d_ch) <= 1e-11 * np.linalg.norm(d_ch)


@pytest.mark.parametrize("seed", [1, 2])
def test_solve_forced_cg_fp64_vs_oracle(gpu, ctx, orc, seed):
    """m=100, n=2000 Gaussian design, tol 1e-10, CG directions on both sides:
    the oracle's objective and support, and the exact-direction solve's."""
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    p = datagen.make_problem("c1", seed=seed)
    _say("forced cg c1 seed", seed)
    A, b = design_to_device(p.AT, "f64"), vec_to_device(p.b)
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, opts=gpu.make_opts(newton_cg=1))
    x = x.cpu().numpy()
    assert info["status"] == 0, info
    assert info["cg_iters"] > 0
    xr, ir, _ = orc.en_solve(p.AT, p.b, p.lam1, p.lam2, tol=p.tol, newton_cg=1)
    assert ir["cg_iters"] > 0
    assert orc.eta(p.AT, p.b, x, p.lam1, p.lam2) <= p.tol
    F = orc.primal_obj(p.AT, p.b, x, p.lam1, p.lam2)
    assert abs(F - ir["primal_obj"]) <= 1e-10 * abs(ir["primal_obj"])
    diff = (x != 0) ^ (xr != 0)
    assert np.all(np.abs(x[diff]) <= 1e-8) and np.all(np.abs(xr[diff]) <= 1e-8)
    xd, infod = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol)
    assert infod["cg_iters"] == 0
    assert np.max(np.abs(x - xd.cpu().numpy())) <= 1e-7
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, opts=gpu.make_opts(newton_cg=1, cg_eta=1.0))


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_solve_forced_cg_mixed_full_size(gpu, ctx, orc, store):
    """The m=500, n=100000 block-Toeplitz workload with FP32 or BF16 storage
    and CG directions: KKT residual <= 1e-6 on the stored design and the
    objective of the factored-direction solve."""
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    p = datagen.make_problem("c2", seed=1, store=store)
    _say("forced cg c2", store)
    A, b = design_to_device(p.AT, store), vec_to_device(p.b)
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, opts=gpu.make_opts(newton_cg=1))
    x = x.cpu().numpy()
    assert info["status"] == 0, info
    assert info["cg_iters"] > 0
    check_eta(orc, p.AT64, p.b, x, p.lam1, p.lam2, p.tol, eta_gpu=info["kkt_rel"])
    xd, infod = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol)
    F = orc.primal_obj(p.AT64, p.b, x, p.lam1, p.lam2)
    Fd = orc.primal_obj(p.AT64, p.b, xd.cpu().numpy(), p.lam1, p.lam2)
    assert abs(F - Fd) <= 1e-6 * abs(Fd)
    print(f"[report] c2 {store} cg: newton {info['newton_iters']} cg {info['cg_iters']} "
          f"ms {info['solve_ms']:.1f} (factored: newton {infod['newton_iters']} ms {infod['solve_ms']:.1f})")


@pytest.mark.parametrize("store", ["f32", "bf16", "f64"])
def test_solve_long_rows_auto_cg(gpu, ctx, orc, store):
    """m=5000 > 4096 rows, n=40000 Gaussian design, lambda = 0.05 lambda_max:
    the first active sets exceed 4096 columns, so the solve switches to CG by
    itself (no dense m x m system exists at this m); certified by the oracle's
    KKT residual and duality gap on the stored design."""
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    cfg = dict(m=5000, n=40000, design="gauss", k=50, snr=5.0, alpha=0.5, c_lam=0.05, tol=1e-6)
    p = datagen.make_problem(cfg, seed=3, store=store, want_f64=True)
    _say("auto cg m=5000", store)
    A, b = design_to_device(p.AT, store), vec_to_device(p.b)
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol)
    del A
    torch.cuda.empty_cache()
    assert info["status"] == 0, info
    assert info["cg_iters"] > 0
    x = x.cpu().numpy()
    eta = check_eta(orc, p.AT64, p.b, x, p.lam1, p.lam2, p.tol, eta_gpu=info["kkt_rel"])
    F = orc.primal_obj(p.AT64, p.b, x, p.lam1, p.lam2)
    y = orc.gemv_n(p.AT64, x) - p.b
    D = orc.dual_obj(p.AT64, p.b, y, p.lam1, p.lam2)
    assert D <= F * (1 + 1e-12)
    assert (F - D) / (1 + abs(F)) <= 1e-5
    print(f"[report] m=5000 {store}: nnz {info['nnz']} newton {info['newton_iters']} "
          f"cg {info['cg_iters']} eta {eta:.2e} ms {info['solve_ms']:.1f}")


def test_path_long_rows(gpu, ctx, orc):
    """A warm-started path at m=5000 > 4096 rows (FP32 storage, 6 points
    c_lambda 1 -> 0.05): x = 0 at lambda_max, every point certified by the
    oracle's KKT residual on the stored design."""
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    cfg = dict(m=5000, n=20000, design="gauss", k=30, snr=5.0, alpha=0.7, c_lam=1.0, tol=1e-6)
    p = datagen.make_problem(cfg, seed=8, store="f32", want_f64=True)
    _say("path m=5000")
    A, b = design_to_device(p.AT, "f32"), vec_to_device(p.b)
    cl = np.geomspace(1.0, 0.05, 6)
    X, infos, status = gpu.ssnal_en_path(ctx, A, b, 0.7, cl, tol=1e-6)
    del A
    torch.cuda.empty_cache()
    assert status == 0, [i["status"] for i in infos]
    X = X.cpu().numpy()
    assert np.all(X[0] == 0.0)
    lam_max = np.max(np.abs(orc.gemv_t(p.AT64, p.b))) / 0.7  # over the stored design, as the path
    for k in range(1, len(cl)):
        lam = cl[k] * lam_max
        check_eta(orc, p.AT64, p.b, X[k], 0.7 * lam, 0.3 * lam, 1e-6, eta_gpu=infos[k]["kkt_rel"])


def test_solve_max_rows(gpu, ctx, orc):
    """The largest m a solve accepts (2^20 rows, n = 64, FP32 storage):
    certified by the oracle's KKT residual; one row more is rejected."""
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    m, n = 1 << 20, 64
    _say("max rows", m, n)
    g = np.random.default_rng(21)
    AT = g.standard_normal((n, m)).astype(np.float32)
    AT /= np.linalg.norm(AT, axis=1, keepdims=True).astype(np.float32)
    x_true = np.zeros(n)
    x_true[[3, 17, 40]] = [2.0, -1.5, 1.0]
    AT64 = AT.astype(np.float64)
    b = orc.gemv_n(AT64, x_true) + 0.01 * g.standard_normal(m)
    lmax = np.max(np.abs(orc.gemv_t(AT64, b)))
    l1, l2 = 0.2 * lmax, 0.1 * lmax
    A = design_to_device(AT, "f32")
    x, info = gpu.ssnal_en_solve(ctx, A, vec_to_device(b), l1, l2, tol=1e-6)
    assert info["status"] == 0, info
    xh = x.cpu().numpy()
    check_eta(orc, AT64, b, xh, l1, l2, 1e-6, eta_gpu=info["kkt_rel"])
    assert set(np.flatnonzero(xh)) >= {3, 17, 40}
    big = torch.zeros((2, m + 1), dtype=torch.float32, device="cuda")
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_solve(ctx, big, vec_to_device(np.ones(m + 1)), 0.1, 0.1)
    del A, big
    torch.cuda.empty_cache()
