"""Full-size single solve: m=1000, n=1,000,000 Gaussian design (alpha=0.5,
lambda=0.1 lambda_max, SNR 3, tol 1e-6) with A stored in FP32 (4 GB), BF16
(2 GB) and FP64 (8 GB).  A full FP64 oracle solve at this size takes far too
long on the host, so each GPU solution is certified independently instead:
the oracle's KKT residual eta (FP64 over the stored design) and duality gap,
sampled columns of A^T v against the oracle, and agreement of the three
solutions' objectives."""
import numpy as np
import pytest

from tests.certify import check_eta

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def c3():
    import datagen
    _say("c3 generate")
    return datagen.make_problem("c3", seed=1, store="f32", want_f64=True)


@pytest.fixture(scope="module")
def ctx(gpu):
    return gpu.Context(0)


def test_c3_fp32_storage(gpu, ctx, orc, c3):
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    p = c3
    _say("c3 fp32 upload")
    A = design_to_device(p.AT, "f32")
    b = vec_to_device(p.b)
    # sampled columns of A^T v against the oracle (FP32 accumulation bound)
    v = np.random.default_rng(3).standard_normal(p.m)
    w = gpu.ssnal_gemv_t(ctx, A, vec_to_device(v)).cpu().numpy()
    cols = np.random.default_rng(4).choice(p.n, size=4096, replace=False)
    wr = orc.gemv_t(np.ascontiguousarray(p.AT64[cols]), v)
    bound = (2 * p.m * 2.0 ** -24 + 2.0 ** -24) * (np.abs(p.AT64[cols]) @ np.abs(v))
    assert np.all(np.abs(w[cols] - wr) <= bound)
    _say("c3 fp32 solve")
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol)
    assert info["status"] == 0, info
    xh = x.cpu().numpy()
    del A
    torch.cuda.empty_cache()
    eta = check_eta(orc, p.AT64, p.b, xh, p.lam1, p.lam2, p.tol, eta_gpu=info["kkt_rel"])
    _say("c3 fp32 eta", eta, "nnz", info["nnz"], "iters", info["outer_iters"], info["newton_iters"])
    F = orc.primal_obj(p.AT64, p.b, xh, p.lam1, p.lam2)
    y = orc.gemv_n(p.AT64, xh) - p.b  # y = A x - b
    D = orc.dual_obj(p.AT64, p.b, y, p.lam1, p.lam2)
    assert D <= F * (1 + 1e-12)
    assert (F - D) / (1 + abs(F)) <= 1e-5  # duality gap at an eta <= 1e-6 point
    c3.x32, c3.F32 = xh, F


def test_c3_bf16_storage(gpu, ctx, orc, c3):
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    p = c3
    bits = datagen.f32_to_bf16_bits(p.AT)
    ATb = datagen.bf16_bits_to_f64(bits)
    _say("c3 bf16 upload")
    A = design_to_device(bits, "bf16")
    b = vec_to_device(p.b)
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol)
    del A
    torch.cuda.empty_cache()
    assert info["status"] == 0, info
    xh = x.cpu().numpy()
    eta = check_eta(orc, ATb, p.b, xh, p.lam1, p.lam2, p.tol, eta_gpu=info["kkt_rel"])
    eta32 = orc.eta(p.AT64, p.b, xh, p.lam1, p.lam2)  # against the FP32 design, reported
    _say("c3 bf16 eta", eta, "eta on the fp32 design", eta32, "nnz", info["nnz"])


def test_c3_fp64_storage(gpu, ctx, orc, c3):
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    p = c3
    _say("c3 fp64 upload")
    A = design_to_device(p.AT64, "f64")
    b = vec_to_device(p.b)
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol)
    del A
    torch.cuda.empty_cache()
    assert info["status"] == 0, info
    xh = x.cpu().numpy()
    eta = check_eta(orc, p.AT64, p.b, xh, p.lam1, p.lam2, p.tol, eta_gpu=info["kkt_rel"])
    F = orc.primal_obj(p.AT64, p.b, xh, p.lam1, p.lam2)
    _say("c3 fp64 eta", eta, "F", F)
    if hasattr(c3, "F32"):
        # the FP32-storage and FP64 solutions of the same (FP32-representable)
        # design agree to the accuracy eta <= 1e-6 allows
        assert abs(F - c3.F32) <= 1e-6 * abs(F)
