"""The Lasso limit lambda2 = 0 (alpha = 1) through the C ABI against the FP64
oracle: small Gaussian problems to tight tolerance, the full-size
block-Toeplitz workload with alpha = 1, a warm-started path, and the
certificates (the dual objective at the scaled feasible point)."""
import numpy as np
import pytest

from tests import pinlib

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu):
    return gpu.Context(0)


@pytest.mark.parametrize("seed", [12, 13])
def test_lasso_small_vs_oracle(gpu, ctx, orc, seed):
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("lasso small", seed)
    A, b, l1, _ = pinlib.gaussian_problem(60, 400, seed, k=8, c_lam=0.3)
    AT = np.ascontiguousarray(A.T)
    xr, ir, _ = orc.en_solve(AT, b, l1, 0.0, tol=1e-10)
    assert ir["status"] == 0
    x, info = gpu.ssnal_en_solve(ctx, design_to_device(AT, "f64"), vec_to_device(b), l1, 0.0,
                                 tol=1e-10)
    assert info["status"] == 0, info
    x = x.cpu().numpy()
    assert orc.eta(AT, b, x, l1, 0.0) <= 1e-10
    F = pinlib.primal_objective(A, b, x, l1, 0.0)
    assert abs(F - ir["primal_obj"]) <= 1e-11 * ir["primal_obj"]
    assert np.max(np.abs(x - xr)) <= 1e-7
    # the certificate: D at the scaled feasible point, gap ~ 0 at the minimiser
    assert info["dual_obj"] <= info["primal_obj"] * (1 + 1e-13)
    assert info["rel_gap"] <= 1e-9
    assert info["dual_obj"] == pytest.approx(orc.dual_obj(AT, b, A @ x - b, l1, 0.0), rel=1e-11)


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_lasso_block_toeplitz(gpu, ctx, orc, store):
    """m=500, n=100000 block-Toeplitz design with alpha = 1 (lambda2 = 0), tol
    1e-6: certified with the oracle's eta on the stored design, objective
    against a tight oracle solve."""
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    p = datagen.make_problem("c2", seed=1, store=store, alpha=1.0)
    assert p.lam2 == 0.0
    _say("lasso c2", store)
    A = design_to_device(p.AT, store)
    x, info = gpu.ssnal_en_solve(ctx, A, vec_to_device(p.b), p.lam1, 0.0, tol=1e-6)
    assert info["status"] == 0, info
    x = x.cpu().numpy()
    assert orc.eta(p.AT64, p.b, x, p.lam1, 0.0) <= 1e-6
    xr, ir, _ = orc.en_solve(p.AT64, p.b, p.lam1, 0.0, tol=1e-10)
    F = orc.primal_obj(p.AT64, p.b, x, p.lam1, 0.0)
    assert abs(F - ir["primal_obj"]) <= 1e-8 * abs(ir["primal_obj"])
    assert info["rel_gap"] <= 1e-5


def test_lasso_path_vs_oracle(gpu, ctx, orc):
    """alpha = 1 path, SNP-like m=120, n=1500, 10 points c = 1 .. 0.05, tol
    1e-10: every point against the warm-started oracle path."""
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    p = datagen.make_problem(dict(m=120, n=1500, design="snp", k=10, snr=5.0, alpha=1.0,
                                  c_lam=1.0, tol=1e-10), seed=5)
    grid = np.geomspace(1.0, 0.05, 10)
    _say("lasso path")
    X, infos, rc = gpu.ssnal_en_path(ctx, design_to_device(p.AT, "f64"), vec_to_device(p.b), 1.0,
                                     grid, tol=1e-10)
    assert rc == 0, [i["status"] for i in infos]
    X = X.cpu().numpy()
    lam_max = float(np.max(np.abs(orc.gemv_t(p.AT, p.b))))
    assert np.count_nonzero(X[0]) == 0
    x0 = None
    for k, c in enumerate(grid):
        l1 = c * lam_max
        xr, ir, _ = orc.en_solve(p.AT, p.b, l1, 0.0, tol=1e-10, x0=x0)
        x0 = xr
        assert orc.eta(p.AT, p.b, X[k], l1, 0.0) <= 1e-10, k
        F = orc.primal_obj(p.AT, p.b, X[k], l1, 0.0)
        assert abs(F - ir["primal_obj"]) <= 1e-10 * abs(ir["primal_obj"]), k


def test_lasso_kkt_entry(gpu, ctx, orc):
    """ssnal_kkt with lambda2 = 0 at an arbitrary point: eta and the scaled dual
    bound against the oracle."""
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("lasso kkt")
    A, b, l1, _ = pinlib.gaussian_problem(50, 300, 3, k=5, c_lam=0.2)
    AT = np.ascontiguousarray(A.T)
    g = np.random.default_rng(2)
    x = np.where(g.random(300) < 0.05, g.standard_normal(300), 0.0)
    res = gpu.ssnal_kkt(ctx, design_to_device(AT, "f64"), vec_to_device(b), vec_to_device(x), l1, 0.0)
    assert res["eta"] == pytest.approx(orc.eta(AT, b, x, l1, 0.0), rel=1e-12)
    assert res["dual_obj"] == pytest.approx(orc.dual_obj(AT, b, A @ x - b, l1, 0.0), rel=1e-12)
    assert res["primal_obj"] == pytest.approx(pinlib.primal_objective(A, b, x, l1, 0.0), rel=1e-12)
