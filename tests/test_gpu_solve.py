"""Whole-solve parity of the HIP path against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest

from tests import pinlib
from tests.certify import check_eta

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu):
    return gpu.Context(0)


def _upload(p, lda=None):
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    return design_to_device(p.AT, p.store, lda=lda), vec_to_device(p.b)


def _support_ok(x, xr, thr=1e-8):
    """supp(x) and supp(xr) agree apart from coefficients within thr of zero."""
    diff = (x != 0) ^ (xr != 0)
    return np.all(np.abs(x[diff]) <= thr) and np.all(np.abs(xr[diff]) <= thr)


def _rel_obj(F, Fr):
    return abs(F - Fr) / abs(Fr)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_small_workload_fp64_vs_oracle(gpu, ctx, orc, seed):
    """m=100, n=2000 Gaussian design, tol 1e-10: rel. objective 1e-10, same support."""
    import datagen
    p = datagen.make_problem("c1", seed=seed)
    _say("c1 fp64 seed", seed)
    A, b = _upload(p)
    x, info, trace = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, trace_cap=512)
    x = x.cpu().numpy()
    xr, ir, tr = orc.en_solve(p.AT, p.b, p.lam1, p.lam2, tol=p.tol)
    assert info["status"] == 0, info
    assert info["kkt_rel"] <= p.tol
    assert orc.eta(p.AT, p.b, x, p.lam1, p.lam2) <= p.tol
    F = orc.primal_obj(p.AT, p.b, x, p.lam1, p.lam2)
    assert _rel_obj(F, ir["primal_obj"]) <= 1e-10
    assert _support_ok(x, xr)
    # r trajectory of the first Newton steps follows the oracle's
    assert trace[0, 2] == tr[0, 2]


def test_block_toeplitz_fp64_vs_oracle(gpu, ctx, orc):
    """m=500, n=100000 block-Toeplitz design (rho=0.6), FP64, full size, both
    sides to tol 1e-10: relative objective 1e-10 and the same support apart
    from coefficients within 1e-8 of zero."""
    import datagen
    p = datagen.make_problem("c2", seed=1)
    _say("c2 fp64 full size, tol 1e-10")
    A, b = _upload(p)
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10)
    x = x.cpu().numpy()
    xr, ir, _ = orc.en_solve(p.AT, p.b, p.lam1, p.lam2, tol=1e-10)
    assert info["status"] == 0, info
    check_eta(orc, p.AT, p.b, x, p.lam1, p.lam2, 1e-10, eta_gpu=info["kkt_rel"])
    F = orc.primal_obj(p.AT, p.b, x, p.lam1, p.lam2)
    assert _rel_obj(F, ir["primal_obj"]) <= 1e-10
    assert _support_ok(x, xr)
    print(f"[report] c2 fp64 tol 1e-10: relobj {_rel_obj(F, ir['primal_obj']):.2e} "
          f"nnz {info['nnz']} / {ir['nnz']}")


@pytest.mark.parametrize("store", ["f32", "bf16"])
def test_block_toeplitz_mixed(gpu, ctx, orc, store):
    """Reduced-precision storage: KKT residual <= 1e-6 on the stored design
    (FP64 oracle on the dequantised design) and the error to the FP64 oracle
    on the original design reported."""
    import datagen
    p = datagen.make_problem("c2", seed=1, store=store)
    _say("c2 mixed", store)
    A, b = _upload(p)
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol)
    x = x.cpu().numpy()
    assert info["status"] == 0, info
    assert info["kkt_rel"] <= p.tol
    eta_stored = check_eta(orc, p.AT64, p.b, x, p.lam1, p.lam2, p.tol, eta_gpu=info["kkt_rel"])
    xr, ir, _ = orc.en_solve(p.AT64, p.b, p.lam1, p.lam2, tol=1e-10)
    F = orc.primal_obj(p.AT64, p.b, x, p.lam1, p.lam2)
    assert _rel_obj(F, ir["primal_obj"]) <= 1e-8
    print(f"[report] {store}: eta_stored={eta_stored:.3e} relobj_stored={_rel_obj(F, ir['primal_obj']):.3e}")


@pytest.mark.parametrize("no_small", [0, 1])
def test_zero_solution(gpu, ctx, orc, no_small):
    """lambda1 >= ||A^T b||_inf: x = 0 with r = 0 throughout (in one workgroup
    and on the multi-kernel path)."""
    import datagen
    p = datagen.make_problem("c1", seed=4)
    lmax = np.max(np.abs(p.AT @ p.b))
    A, b = _upload(p)
    _say("zero solution", no_small)
    x, info = gpu.ssnal_en_solve(ctx, A, b, lmax * 1.01, 0.3, tol=1e-10, opts=gpu.make_opts(no_small=no_small))
    assert info["one_workgroup"] == 1 - no_small
    assert info["status"] == 0 and info["nnz"] == 0
    assert np.count_nonzero(x.cpu().numpy()) == 0


def test_ridge_limit(gpu, ctx, orc):
    """lambda1 = 0: J is every column (r = n > m), the m x m system every step."""
    A_, b_, _, _ = pinlib.gaussian_problem(60, 900, 9)
    l2 = 0.7
    import torch
    A = torch.from_numpy(np.ascontiguousarray(A_.T)).cuda()
    b = torch.from_numpy(b_).cuda()
    _say("ridge")
    x, info = gpu.ssnal_en_solve(ctx, A, b, 0.0, l2, tol=1e-11)
    ref = A_.T @ np.linalg.solve(A_ @ A_.T + l2 * np.eye(60), b_)
    assert info["status"] == 0
    assert np.max(np.abs(x.cpu().numpy() - ref)) <= 1e-9


@pytest.mark.parametrize("m,n", [(1, 50), (7, 1), (300, 40)])
def test_edge_shapes(gpu, ctx, orc, m, n):
    """m = 1, n = 1, and m > n (orthogonal-ish designs)."""
    import torch
    g = np.random.default_rng(m * 100 + n)
    A_ = g.standard_normal((m, n))
    b_ = g.standard_normal(m)
    l1 = 0.3 * np.max(np.abs(A_.T @ b_))
    l2 = 0.2
    A = torch.from_numpy(np.ascontiguousarray(A_.T)).cuda()
    b = torch.from_numpy(b_).cuda()
    _say("edge", m, n)
    x, info = gpu.ssnal_en_solve(ctx, A, b, l1, l2, tol=1e-11)
    xr, ir, _ = orc.en_solve(np.ascontiguousarray(A_.T), b_, l1, l2, tol=1e-12)
    assert info["status"] == 0, info
    assert np.max(np.abs(x.cpu().numpy() - xr)) <= 1e-8


@pytest.mark.parametrize("no_small", [0, 1])
def test_padded_lda_and_warm_start(gpu, ctx, orc, no_small):
    """lda > m with NaN padding rows; a warm start reaches the same minimiser
    (in one workgroup and on the multi-kernel path)."""
    import datagen
    p = datagen.make_problem("c1", seed=5)
    A, b = _upload(p, lda=p.m + 4)
    o = gpu.make_opts(no_small=no_small)
    _say("padded lda + warm start", no_small)
    x_cold, ic = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10, m=p.m, opts=o)
    x1, _ = gpu.ssnal_en_solve(ctx, A, b, p.lam1 * 1.2, p.lam2 * 1.2, tol=1e-10, m=p.m, opts=o)
    x_warm, iw = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, x0=x1, tol=1e-10, m=p.m, opts=o)
    assert ic["status"] == 0 and iw["status"] == 0
    assert ic["one_workgroup"] == iw["one_workgroup"] == 1 - no_small
    xc, xw = x_cold.cpu().numpy(), x_warm.cpu().numpy()
    xr, ir, _ = orc.en_solve(p.AT, p.b, p.lam1, p.lam2, tol=1e-11)
    assert np.max(np.abs(xc - xr)) <= 1e-8 and np.max(np.abs(xw - xr)) <= 1e-8


@pytest.mark.parametrize("no_small", [0, 1])
def test_errors(gpu, ctx, no_small):
    """Invalid lambdas: SSNAL_EINVAL; non-finite b: SSNAL_ENONFINITE;
    max_outer = 1 at a tight tol: SSNAL_NOT_CONVERGED (in one workgroup and
    on the multi-kernel path)."""
    import datagen
    p = datagen.make_problem("c1", seed=6)
    A, b = _upload(p)
    _say("errors", no_small)
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_en_solve(ctx, A, b, p.lam1, -0.1)  # lambda2 < 0 (0 is the Lasso limit)
    assert e.value.code == -1
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_en_solve(ctx, A, b, -1.0, 0.5)
    assert e.value.code == -1
    bn = b.clone()
    bn[3] = float("nan")
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_en_solve(ctx, A, bn, p.lam1, p.lam2)
    assert e.value.code == -2
    o = gpu.make_opts(max_outer=1, no_small=no_small)
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-14, opts=o)
    assert info["status"] == 1 and info["one_workgroup"] == 1 - no_small


@pytest.mark.parametrize("no_small", [0, 1])
def test_repeat_bitwise(gpu, ctx, no_small):
    """Deterministic reductions: two solves of the same input agree bit for bit
    (in one workgroup and on the multi-kernel path)."""
    import datagen
    p = datagen.make_problem("c1", seed=7)
    A, b = _upload(p)
    o = gpu.make_opts(no_small=no_small)
    _say("repeat", no_small)
    x1, i1 = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10, opts=o)
    x2, _ = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10, opts=o)
    assert i1["one_workgroup"] == 1 - no_small
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
