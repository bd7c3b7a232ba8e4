"""k-fold cross validation (Sec. "Parameter tuning") through the C ABI against
the FP64 oracle: validation errors per fold and grid point on the full data's
lambda grid, with the argmin of the mean error, and the input checks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu):
    return gpu.Context(0)


def _fold_dev(fold):
    import torch
    return torch.from_numpy(np.ascontiguousarray(fold, dtype=np.int32)).cuda()


@pytest.mark.parametrize("cfg,store,k,alpha,tol,rtol", [
    (dict(m=120, n=1500, design="gauss", k=10, snr=5.0, alpha=0.5, c_lam=1.0, tol=1e-10), "f64", 4, 0.5,
     1e-10, 1e-7),
    (dict(m=150, n=2000, design="toeplitz", k=10, snr=3.0, alpha=1.0, c_lam=1.0, tol=1e-10), "f64", 3, 1.0,
     1e-10, 1e-7),
    (dict(m=300, n=20000, design="snp", k=20, snr=5.0, alpha=0.7, c_lam=1.0, tol=1e-6), "f32", 5, 0.7,
     1e-6, 1e-4),
])
def test_cv_vs_oracle(gpu, ctx, orc, cfg, store, k, alpha, tol, rtol):
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("cv", cfg["m"], cfg["n"], store, "k", k, "alpha", alpha)
    p = datagen.make_problem(cfg, seed=11, store=store, want_f64=True)
    grid = np.geomspace(2.0, 0.05, 8)
    fold = np.random.default_rng(4).permutation(np.arange(p.m) % k)
    err, infos, rc = gpu.ssnal_en_cv(ctx, design_to_device(p.AT, store), vec_to_device(p.b),
                                     _fold_dev(fold), k, alpha, grid, tol=tol)
    assert rc == 0, rc
    assert all(i["status"] == 0 for row in infos for i in row)
    ref, rc_ref = orc.cv(p.AT64, p.b, fold, k, alpha, grid, tol=1e-10)
    assert rc_ref == 0
    # grid point 0 lies above lambda_max: every fold's error is the mean of b^2 over its rows
    for f in range(k):
        assert err[f, 0] == pytest.approx(np.mean(p.b[fold == f] ** 2), rel=1e-12)
    np.testing.assert_allclose(err, ref, rtol=rtol, atol=0)
    assert int(np.argmin(err.mean(axis=0))) == int(np.argmin(ref.mean(axis=0)))


def test_cv_errors(gpu, ctx):
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("cv errors")
    p = datagen.make_problem(dict(m=40, n=300, design="gauss", k=4, snr=5.0, alpha=0.5, c_lam=1.0,
                                  tol=1e-8), seed=2)
    A, b = design_to_device(p.AT, "f64"), vec_to_device(p.b)
    bad = np.arange(40) % 3
    bad[5] = 7
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_cv(ctx, A, b, _fold_dev(bad), 3, 0.5, [0.5])
    empty = np.zeros(40, dtype=np.int32)  # fold 1 has no rows
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_cv(ctx, A, b, _fold_dev(empty), 2, 0.5, [0.5])
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_cv(ctx, A, b, _fold_dev(np.arange(40) % 2), 1, 0.5, [0.5])
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_cv(ctx, A, b, _fold_dev(np.arange(40) % 2), 2, 0.5, [0.5], slots=0)


def test_cv_slots_bitwise(gpu, ctx):
    """Folds on concurrent workers give the errors of the folds in turn, bit for bit."""
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("cv slots")
    p = datagen.make_problem(dict(m=200, n=4000, design="toeplitz", k=10, snr=4.0, alpha=0.6, c_lam=1.0,
                                  tol=1e-6), seed=6, store="f32")
    A, b = design_to_device(p.AT, "f32"), vec_to_device(p.b)
    fold = _fold_dev(np.random.default_rng(9).permutation(np.arange(200) % 5))
    grid = np.geomspace(1.0, 0.05, 12)
    E1, I1, rc1 = gpu.ssnal_en_cv(ctx, A, b, fold, 5, 0.6, grid, tol=1e-6, slots=1)
    E3, I3, rc3 = gpu.ssnal_en_cv(ctx, A, b, fold, 5, 0.6, grid, tol=1e-6, slots=3)
    E8, I8, rc8 = gpu.ssnal_en_cv(ctx, A, b, fold, 5, 0.6, grid, tol=1e-6, slots=8)
    assert rc1 == rc3 == rc8 == 0
    assert np.array_equal(E1, E3) and np.array_equal(E1, E8)
    assert [i["newton_iters"] for row in I1 for i in row] == [i["newton_iters"] for row in I8 for i in row]


def test_cv_long_rows_composition(gpu, ctx, orc):
    """m=4500 > 4096 rows (FP32 storage): each fold's errors equal the path
    on the fold's training rows copied on the host (full data's grid), with
    the validation residuals taken by the oracle."""
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("cv long rows")
    m, n, k, alpha = 4500, 6000, 3, 0.6
    p = datagen.make_problem(dict(m=m, n=n, design="gauss", k=20, snr=5.0, alpha=alpha, c_lam=1.0,
                                  tol=1e-6), seed=12, store="f32")
    A, b = design_to_device(p.AT, "f32"), vec_to_device(p.b)
    fold = np.random.default_rng(13).permutation(np.arange(m) % k)
    grid = np.geomspace(0.6, 0.1, 4)
    E, infos, rc = gpu.ssnal_en_cv(ctx, A, b, _fold_dev(fold), k, alpha, grid, tol=1e-6, slots=2)
    assert rc == 0
    lam_max = np.max(np.abs(orc.gemv_t(p.AT64, p.b))) / alpha
    ctx2 = gpu.Context(0)
    for f in range(k):
        tr = np.flatnonzero(fold != f)
        At = design_to_device(np.ascontiguousarray(p.AT[:, tr]), "f32")
        # the path on the training rows scales its own grid by ||A_t^T b_t||_inf; rescale
        lam_t = np.max(np.abs(orc.gemv_t(p.AT64[:, tr], p.b[tr]))) / alpha
        X, inf_t, st = gpu.ssnal_en_path(ctx2, At, vec_to_device(p.b[tr]), alpha, grid * lam_max / lam_t,
                                         tol=1e-6)
        assert st == 0
        X = X.cpu().numpy()
        va = np.flatnonzero(fold == f)
        for q in range(len(grid)):
            res = orc.gemv_n(p.AT64, X[q]) - p.b
            ref = np.mean(res[va] ** 2)
            assert E[f, q] == pytest.approx(ref, rel=1e-6), (f, q)
