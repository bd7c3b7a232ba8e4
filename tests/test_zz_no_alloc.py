"""The no-allocation solve entry point (for callers that cannot allocate)
against ssnal_en_solve, through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


def test_noalloc_matches_solve(gpu):
    """Two calls in a row, the second smaller (the static array keeps the
    first call's contents): each gives the bits of ssnal_en_solve on the same
    problem, and sizes past the limits are refused."""
    import datagen
    import torch
    from paper_2006_03970_amd.device import design_to_device, vec_to_device
    ctx = gpu.Context(0)
    cases = [("c2", "f32", 500, 100_000), ("c1", "f64", 100, 2000)]
    for name, store, m, n in cases:
        p = datagen.make_problem(name, seed=3, store=store)
        assert (p.m, p.n) == (m, n)
        A, b = design_to_device(p.AT, p.store), vec_to_device(p.b)
        _say("noalloc", name, store)
        xr, ir = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol)
        x = torch.full((p.n,), float("nan"), dtype=torch.float64, device=A.device)
        info = gpu.ssnal_en_solve_noalloc(ctx, A, b, p.lam1, p.lam2, x, tol=p.tol)
        torch.cuda.synchronize()
        assert info["status"] == 0 and ir["status"] == 0
        assert info["kkt_rel"] <= p.tol
        # same kernels with the same split plans: the same bits
        assert bool((x == xr).all())
        assert info["newton_iters"] == ir["newton_iters"]
        rel = abs(info["primal_obj"] - ir["primal_obj"]) / abs(ir["primal_obj"])
        assert rel <= 1e-12
    # past the limits
    p = datagen.make_problem(dict(m=600, n=3000, design="gauss", k=5, snr=5.0, alpha=0.5, c_lam=0.5,
                                  tol=1e-6), seed=4)
    A, b = design_to_device(p.AT, "f64"), vec_to_device(p.b)
    x = torch.empty(p.n, dtype=torch.float64, device=A.device)
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_en_solve_noalloc(ctx, A, b, p.lam1, p.lam2, x, tol=1e-6)
    assert e.value.code == -1
    with pytest.raises(gpu.SsnalError):
        gpu.ssnal_en_solve_noalloc(ctx, A[:, :100].contiguous(), b[:100], p.lam1, p.lam2, x, tol=1e-6,
                                   opts=gpu.make_opts(timing=1))
