"""Model selection at a solution (gcv / e-bic, Sec. "Parameter tuning", eq.
gcv_bic) through the C ABI against the FP64 oracle: degrees of freedom, the
least-squares (de-biased) fit and the criteria, on synthetic supports that
span one and several 64-row blocks of the dense systems, the r >= m and
singular cases, and along a warm-started path of the SNP-like workload."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu):
    return gpu.Context(0)


def _check(res, ref, tol):
    assert res["status"] == ref["status"], (res, ref)
    assert res["r"] == ref["r"]
    for k in ("nu", "rss_en"):
        assert res[k] == pytest.approx(ref[k], rel=tol, abs=tol), k
    if ref["status"] == 0:
        for k in ("rss", "gcv", "ebic"):
            assert res[k] == pytest.approx(ref[k], rel=tol, abs=tol), k
    else:
        assert np.isnan(res["rss"]) and np.isnan(res["gcv"]) and np.isnan(res["ebic"])


@pytest.mark.parametrize("m,n,r,store", [(300, 5000, 40, "f64"), (300, 5000, 150, "f64"),
                                         (300, 5000, 260, "f64"), (300, 5000, 0, "f64"),
                                         (300, 5000, 1, "f64"), (300, 5000, 64, "f64"),
                                         (300, 5000, 420, "f64"), (257, 3000, 129, "f64"),
                                         (300, 5000, 150, "f32"), (300, 5000, 150, "bf16")])
def test_model_select_vs_oracle(gpu, ctx, orc, m, n, r, store):
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("model_select", m, n, r, store)
    AT, AT64 = datagen.make_design("gauss", m, n, 77 + r, store)
    g = np.random.default_rng(r + 5)
    x = np.zeros(n)
    J = g.choice(n, size=r, replace=False)
    x[J] = g.standard_normal(r)
    b = g.standard_normal(m)
    l2 = 0.4
    ref = orc.model_select(AT64, b, x, l2, want_beta=True)
    A = design_to_device(AT, store)
    res = gpu.ssnal_en_model_select(ctx, A, vec_to_device(b), vec_to_device(x), l2, want_beta=True)
    # FP64 storage: FP64 throughout; FP32/BF16 storage: the Gram matrices
    # accumulate in FP32 (relative error ~ m * 2^-24 per entry)
    tol = 1e-9 if store == "f64" else 2e-4
    _check(res, ref, tol)
    beta = res["beta"].cpu().numpy()
    if ref["status"] == 0:
        scale = max(1.0, np.max(np.abs(ref["beta"])))
        assert np.max(np.abs(beta - ref["beta"])) <= tol * 10 * scale
    else:
        assert np.all(beta == 0.0)


def test_model_select_singular(gpu, ctx, orc):
    """A repeated selected column: A_J^T A_J is singular (status 2)."""
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("model_select singular")
    g = np.random.default_rng(8)
    m, n = 40, 200
    AT = g.standard_normal((n, m))
    AT[3] = 0.0
    AT[3, :4] = 1.0
    AT[5] = AT[3]
    x = np.zeros(n)
    x[[3, 5, 9]] = 1.0
    b = g.standard_normal(m)
    ref = orc.model_select(AT, b, x, 0.5)
    assert ref["status"] == 2
    res = gpu.ssnal_en_model_select(ctx, design_to_device(AT, "f64"), vec_to_device(b),
                                    vec_to_device(x), 0.5)
    _check(res, ref, 1e-9)


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_model_select_on_path(gpu, ctx, orc, store):
    """Criteria along a warm-started path of the SNP-like workload (m=500,
    n=2e5, alpha=0.5): every point against the oracle at the same solution,
    and the minimising points agree."""
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("model_select path", store)
    p = datagen.make_problem("c4", seed=3, store=store, want_f64=True)
    A = design_to_device(p.AT, store)
    b = vec_to_device(p.b)
    cl = np.geomspace(0.9, 0.05, 12)
    X, infos, status = gpu.ssnal_en_path(ctx, A, b, 0.5, cl, tol=1e-6)
    assert status == 0
    lam_max = float(np.max(np.abs(orc.gemv_t(p.AT64, p.b)))) / 0.5
    gcv, gcv_ref = [], []
    for k in range(len(cl)):
        l2 = 0.5 * cl[k] * lam_max
        x = X[k].contiguous()
        res = gpu.ssnal_en_model_select(ctx, A, b, x, l2)
        ref = orc.model_select(p.AT64, p.b, x.cpu().numpy(), l2)
        _check(res, ref, 1e-9 if store == "f64" else 2e-4)
        gcv.append(res["gcv"] if res["status"] == 0 else np.inf)
        gcv_ref.append(ref["gcv"] if ref["status"] == 0 else np.inf)
    assert int(np.argmin(gcv)) == int(np.argmin(gcv_ref))


@pytest.mark.parametrize("m,n,r,store", [(5000, 8000, 120, "f64"), (5000, 8000, 300, "f32")])
def test_model_select_long_rows(gpu, ctx, orc, m, n, r, store):
    """m > 4096 rows with a support of r < 4096 columns: the r x r systems."""
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("model_select long rows", m, n, r, store)
    AT, AT64 = datagen.make_design("gauss", m, n, 91 + r, store)
    g = np.random.default_rng(r + 9)
    x = np.zeros(n)
    x[g.choice(n, size=r, replace=False)] = g.standard_normal(r)
    b = g.standard_normal(m)
    ref = orc.model_select(AT64, b, x, 0.4, want_beta=True)
    res = gpu.ssnal_en_model_select(ctx, design_to_device(AT, store), vec_to_device(b),
                                    vec_to_device(x), 0.4, want_beta=True)
    _check(res, ref, 1e-9 if store == "f64" else 2e-3)


def test_model_select_long_rows_wide_support(gpu, ctx):
    """m > 4096 and a support above 4096 columns: no dense system fits."""
    import datagen
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    _say("model_select long rows, wide support")
    AT, _ = datagen.make_design("gauss", 4200, 5000, 3, "f32")
    x = np.zeros(5000)
    x[:4100] = 1.0
    b = np.ones(4200)
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_model_select(ctx, design_to_device(AT, "f32"), vec_to_device(b), vec_to_device(x), 0.4)
