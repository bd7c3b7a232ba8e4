"""Parity of the one-workgroup solve (FP64, m <= 120, small m n: the whole of
Algorithm 1 in one workgroup) against the FP64 oracle, through the C ABI, and
its agreement with the multi-kernel path on the same problems."""
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
    diff = (x != 0) ^ (xr != 0)
    return np.all(np.abs(x[diff]) <= thr) and np.all(np.abs(xr[diff]) <= thr)


def _rel_obj(F, Fr):
    return abs(F - Fr) / abs(Fr)


def _check_vs_oracle(orc, p, x, info, tol):
    """eta <= tol on both sides' evaluation, relative objective 1e-10 to the
    oracle's minimiser, the same support apart from coefficients within 1e-8
    of zero."""
    assert info["status"] == 0, info
    check_eta(orc, p.AT, p.b, x, p.lam1, p.lam2, tol, eta_gpu=info["kkt_rel"])
    xr, ir, _ = orc.en_solve(p.AT, p.b, p.lam1, p.lam2, tol=min(tol, 1e-10))
    F = orc.primal_obj(p.AT, p.b, x, p.lam1, p.lam2)
    assert _rel_obj(F, ir["primal_obj"]) <= 1e-10, (F, ir["primal_obj"])
    assert _support_ok(x, xr)
    return xr, ir


def _single_one_wg(m, n):
    """The documented single-solve rule of the one-workgroup path (FP64,
    m <= 120): m n <= 2^17, or the n-vectors (36 bytes a feature) fit in
    LDS beside the Newton matrix."""
    return m <= 120 and (m * n <= 1 << 17 or n <= (150112 - 16 * (-(-m * (m + 1) // 4))) // 36)


def _solve1(gpu, ctx, A, b, p, tol, x0=None, x_out=None, opts=None, m=None):
    """A single solve that runs in one workgroup: ssnal_en_solve when
    m n <= 2^17 (always within the single-solve rule), else a batch of one
    (m n <= 2^21)."""
    import torch
    if p.m * p.n <= 1 << 17:
        return gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, x0=x0, x_out=x_out, tol=tol, opts=opts, m=m)
    if x_out is None:
        x_out = torch.empty(p.n, dtype=torch.float64, device=A.device)
    pr = dict(A=A, b=b, lambda1=p.lam1, lambda2=p.lam2, tol=tol, x_out=x_out, x0=x0, m=m,
              sigma0=opts.sigma0 if opts is not None else 0.0)
    infos, _ = gpu.ssnal_en_solve_batch(ctx, [pr], opts=opts)
    return x_out, infos[0]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_c1_one_workgroup_vs_oracle(gpu, ctx, orc, seed):
    """m=100, n=2000 Gaussian design, tol 1e-10, in one workgroup (a batch of
    one); a single solve also runs in one workgroup (its n-vectors fit in
    LDS) and gives the same bits; the multi-kernel path agrees to 1e-9."""
    import datagen
    p = datagen.make_problem("c1", seed=seed)
    _say("c1 one workgroup seed", seed)
    A, b = _upload(p)
    x, info = _solve1(gpu, ctx, A, b, p, p.tol)
    assert info["one_workgroup"] == 1
    assert info["syncs"] == 1
    _check_vs_oracle(orc, p, x.cpu().numpy(), info, p.tol)
    xs, si = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol)
    assert si["one_workgroup"] == 1
    assert np.array_equal(xs.cpu().numpy(), x.cpu().numpy())
    xm, mi = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, opts=gpu.make_opts(no_small=1))
    assert mi["one_workgroup"] == 0
    assert np.max(np.abs(xm.cpu().numpy() - x.cpu().numpy())) <= 1e-9


def test_agrees_with_multi_kernel_path(gpu, ctx, orc):
    """The same problem through both paths: both meet the oracle bar, and
    their minimisers agree to 1e-9 (they differ only in summation order)."""
    import datagen
    p = datagen.make_problem("c1", seed=11)
    A, b = _upload(p)
    _say("one workgroup vs multi-kernel")
    x1, i1 = _solve1(gpu, ctx, A, b, p, p.tol)
    x2, i2 = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=p.tol, opts=gpu.make_opts(no_small=1))
    assert i1["one_workgroup"] == 1 and i2["one_workgroup"] == 0
    x1, x2 = x1.cpu().numpy(), x2.cpu().numpy()
    _check_vs_oracle(orc, p, x1, i1, p.tol)
    _check_vs_oracle(orc, p, x2, i2, p.tol)
    assert np.max(np.abs(x1 - x2)) <= 1e-9
    # the same sigma schedule: sigma0 from the column norms, x5 per outer iteration
    assert i1["sigma0"] == pytest.approx(i2["sigma0"], rel=1e-14)
    print(f"[report] outer {i1['outer_iters']}/{i2['outer_iters']} newton "
          f"{i1['newton_iters']}/{i2['newton_iters']} passes {i1['gemv_calls']}/{i2['gemv_calls']}")


@pytest.mark.parametrize("m,n,k,c_lam", [(37, 2001, 5, 0.5), (120, 1092, 12, 0.5), (64, 513, 40, 0.05),
                                         (100, 40, 8, 0.5), (120, 17000, 12, 0.5), (120, 2000, 90, 0.5),
                                         (120, 2000, 60, 0.45)])
def test_ragged_and_maximum_shapes(gpu, ctx, orc, m, n, k, c_lam):
    """m off the 16-row MFMA blocks and the 8-column Cholesky panels, n off the
    feature slabs, the largest m (120) at the single-solve limit m n <= 2^17
    and near the batch limit 2^21 (a batch of one), m > n, an active set
    larger than m (160 of 513 at m = 64: the m x m system), and many active
    features at m = 120 (r x r systems of 86 to 151 rows: past 64, two rows
    a lane in the one-wave triangular solves)."""
    import datagen
    p = datagen.make_problem("c1", seed=m + n, m=m, n=n, k=k, c_lam=c_lam)
    A, b = _upload(p)
    _say("one workgroup shape", m, n, k)
    x, info = _solve1(gpu, ctx, A, b, p, p.tol)
    assert info["one_workgroup"] == 1
    _check_vs_oracle(orc, p, x.cpu().numpy(), info, p.tol)


def test_beyond_limits_takes_multi_kernel_path(gpu, ctx):
    """m = 121, or a single solve with m n above 2^17 whose n-vectors do not
    fit in LDS (n > 3047 at m = 100, 2556 at m = 120), or FP32 storage: the
    multi-kernel path.  Just inside the LDS rule above 2^17: one workgroup."""
    import datagen
    for m, n, store in [(121, 1000, "f64"), (100, 3048, "f64"), (120, 2557, "f64"), (100, 1000, "f32")]:
        p = datagen.make_problem("c1", seed=3, m=m, n=n, store=store)
        A, b = _upload(p)
        _say("multi-kernel", m, n, store)
        x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-8)
        assert info["status"] == 0 and info["one_workgroup"] == 0
        assert not _single_one_wg(m, n) or store != "f64"
    for m, n in [(100, 3047), (120, 2556)]:
        p = datagen.make_problem("c1", seed=3, m=m, n=n)
        A, b = _upload(p)
        _say("one workgroup at the LDS limit", m, n)
        x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-8)
        assert info["status"] == 0 and info["one_workgroup"] == 1 and _single_one_wg(m, n)


def test_lasso_limit(gpu, ctx, orc):
    """lambda2 = 0: the Lasso, whose dual objective takes the scaled dual point."""
    import datagen
    p = datagen.make_problem("c1", seed=12)
    p.lam2 = 0.0
    A, b = _upload(p)
    _say("lasso one workgroup")
    x, info = _solve1(gpu, ctx, A, b, p, 1e-9)
    assert info["one_workgroup"] == 1
    x = x.cpu().numpy()
    assert info["status"] == 0, info
    check_eta(orc, p.AT, p.b, x, p.lam1, 0.0, 1e-9, eta_gpu=info["kkt_rel"])
    xr, ir, _ = orc.en_solve(p.AT, p.b, p.lam1, 0.0, tol=1e-11)
    F = orc.primal_obj(p.AT, p.b, x, p.lam1, 0.0)
    assert _rel_obj(F, ir["primal_obj"]) <= 1e-9
    # the reported duality gap is the oracle's objectives' gap at this x
    assert info["rel_gap"] >= -1e-12 and info["rel_gap"] <= 1e-5


def test_woodbury_and_full_system_agree(gpu, ctx, orc):
    """r < m takes the r x r system (eq. smw_formula); no_smw forces the m x m
    one (eq. AJ_system): the same minimiser."""
    import datagen
    p = datagen.make_problem("c1", seed=13, k=4, c_lam=0.8)
    A, b = _upload(p)
    _say("woodbury vs m x m")
    x1, i1 = _solve1(gpu, ctx, A, b, p, p.tol)
    x2, i2 = _solve1(gpu, ctx, A, b, p, p.tol, opts=gpu.make_opts(no_smw=1))
    assert i1["one_workgroup"] == 1 and i2["one_workgroup"] == 1
    assert 0 < i1["nnz"] < p.m
    x1, x2 = x1.cpu().numpy(), x2.cpu().numpy()
    _check_vs_oracle(orc, p, x1, i1, p.tol)
    _check_vs_oracle(orc, p, x2, i2, p.tol)
    assert np.max(np.abs(x1 - x2)) <= 1e-9


def test_ridge_and_zero_solutions(gpu, ctx, orc):
    """lambda1 = 0 (every feature active: the m x m system each step) against
    the closed form; lambda1 above ||A^T b||_inf: x = 0 with r = 0."""
    import torch
    A_, b_, _, _ = pinlib.gaussian_problem(60, 900, 9)
    l2 = 0.7
    A = torch.from_numpy(np.ascontiguousarray(A_.T)).cuda()
    b = torch.from_numpy(b_).cuda()
    _say("ridge one workgroup")
    x, info = gpu.ssnal_en_solve(ctx, A, b, 0.0, l2, tol=1e-11)
    assert info["one_workgroup"] == 1 and info["status"] == 0
    ref = A_.T @ np.linalg.solve(A_ @ A_.T + l2 * np.eye(60), b_)
    assert np.max(np.abs(x.cpu().numpy() - ref)) <= 1e-9
    lmax = np.max(np.abs(A_.T @ b_))
    x, info = gpu.ssnal_en_solve(ctx, A, b, lmax * 1.01, 0.3, tol=1e-10)
    assert info["one_workgroup"] == 1 and info["status"] == 0 and info["nnz"] == 0
    assert np.count_nonzero(x.cpu().numpy()) == 0


@pytest.mark.parametrize("m,n", [(1, 50), (7, 1), (1, 1)])
def test_degenerate_shapes(gpu, ctx, orc, m, n):
    """One row, one column, one entry."""
    import torch
    g = np.random.default_rng(m * 100 + n + 7)
    A_ = g.standard_normal((m, n))
    b_ = g.standard_normal(m)
    l1 = 0.3 * np.max(np.abs(A_.T @ b_))
    l2 = 0.2
    A = torch.from_numpy(np.ascontiguousarray(A_.T)).cuda()
    b = torch.from_numpy(b_).cuda()
    _say("degenerate", m, n)
    x, info = gpu.ssnal_en_solve(ctx, A, b, l1, l2, tol=1e-11)
    assert info["one_workgroup"] == 1
    xr, ir, _ = orc.en_solve(np.ascontiguousarray(A_.T), b_, l1, l2, tol=1e-12)
    assert info["status"] == 0, info
    assert np.max(np.abs(x.cpu().numpy() - xr)) <= 1e-8


def test_warm_start_padded_lda_aliased(gpu, ctx, orc):
    """lda > m with NaN padding rows (never read); a warm start from another
    point, with x0 the output buffer itself, reaches the same minimiser."""
    import datagen
    p = datagen.make_problem("c1", seed=14, n=1000)
    A, b = _upload(p, lda=p.m + 4)
    _say("warm start, padded lda, x0 == x_out")
    x_cold, ic = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10, m=p.m)
    x1, _ = gpu.ssnal_en_solve(ctx, A, b, p.lam1 * 1.2, p.lam2 * 1.2, tol=1e-10, m=p.m)
    x_warm, iw = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, x0=x1, x_out=x1, tol=1e-10, m=p.m)
    assert ic["one_workgroup"] == 1 and iw["one_workgroup"] == 1
    assert ic["status"] == 0 and iw["status"] == 0
    xr, _, _ = orc.en_solve(p.AT, p.b, p.lam1, p.lam2, tol=1e-11)
    assert np.max(np.abs(x_cold.cpu().numpy() - xr)) <= 1e-8
    assert np.max(np.abs(x_warm.cpu().numpy() - xr)) <= 1e-8


@pytest.mark.parametrize("m,n", [(37, 1100), (99, 1300), (119, 2000), (17, 3001)])
def test_odd_m_even_lda_nan_padding(gpu, ctx, orc, m, n):
    """Odd m with an even padded lda (NaN padding rows): the 16-byte passes
    read row m of each column with the last row pair and must mask it (119 x
    2000 runs as a batch of one).  The solve meets the oracle bar and agrees
    with the same problem at lda = m (odd: the 8-byte passes) to 1e-9."""
    import datagen
    p = datagen.make_problem("c1", seed=500 + m, m=m, n=n)
    _say("odd m, even lda", m, n)
    A_pad, b = _upload(p, lda=m + 1)
    A_odd, _ = _upload(p)
    x_pad, ip = _solve1(gpu, ctx, A_pad, b, p, 1e-10, m=m)
    x_odd, io = _solve1(gpu, ctx, A_odd, b, p, 1e-10, m=m)
    assert ip["one_workgroup"] == 1 and io["one_workgroup"] == 1
    _check_vs_oracle(orc, p, x_pad.cpu().numpy(), ip, 1e-10)
    assert np.max(np.abs(x_pad.cpu().numpy() - x_odd.cpu().numpy())) <= 1e-9


def test_unaligned_design(gpu, ctx, orc):
    """A design that starts 8 bytes past a 16-byte boundary (even lda) takes
    the 8-byte passes and reaches the oracle's minimiser."""
    import datagen
    import torch
    p = datagen.make_problem("c1", seed=510, m=64, n=1500)
    A, b = _upload(p)
    buf = torch.full((A.numel() + 1,), float("nan"), dtype=torch.float64, device=A.device)
    buf[1:] = A.reshape(-1)
    Au = buf[1:].view(p.n, p.m)
    assert Au.data_ptr() % 16 == 8
    _say("unaligned design")
    x, info = _solve1(gpu, ctx, Au, b, p, 1e-10, m=p.m)
    assert info["one_workgroup"] == 1
    _check_vs_oracle(orc, p, x.cpu().numpy(), info, 1e-10)


def test_errors_and_status(gpu, ctx):
    """Non-finite b or x0: SSNAL_ENONFINITE; max_outer = 1 at a tight tol:
    SSNAL_NOT_CONVERGED with the certificates of the returned point."""
    import datagen
    p = datagen.make_problem("c1", seed=15, n=1000)
    A, b = _upload(p)
    _say("errors one workgroup")
    bn = b.clone()
    bn[5] = float("inf")
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_en_solve(ctx, A, bn, p.lam1, p.lam2)
    assert e.value.code == -2
    import torch
    x0 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    x0[17] = float("nan")
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, x0=x0)
    assert e.value.code == -2
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-14, opts=gpu.make_opts(max_outer=1))
    assert info["one_workgroup"] == 1 and info["status"] == 1 and info["outer_iters"] == 1
    assert np.isfinite(info["kkt_rel"]) and info["kkt_rel"] > 1e-14
    # the same solve still works after the errors
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10)
    assert info["status"] == 0


def test_repeat_bitwise(gpu, ctx):
    """Fixed-order sums: two one-workgroup solves agree bit for bit."""
    import datagen
    p = datagen.make_problem("c1", seed=16, n=1000)
    A, b = _upload(p)
    _say("repeat one workgroup")
    x1, i1 = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10)
    x2, _ = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10)
    assert i1["one_workgroup"] == 1
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())


def test_batch_one_launch_matches_single(gpu, ctx, orc):
    """A batch of 40 problems: 32 small FP64 ones (m from 20 to 120, m n up to
    4.2e5, some above the single-solve limits; per-problem sigma0 on some)
    run as one launch, one workgroup each, beside 8 others (m = 160, FP32
    storage) on the workers.  A small problem whose single solve also runs in
    one workgroup gives the same bits (same kernel, same summation order);
    one past the single-solve limit agrees with the multi-kernel solve to
    1e-9; every problem meets the oracle bar."""
    import datagen
    import torch
    probs, keep, ref = [], [], []
    for i in range(40):
        if i < 32:
            m, n, store = 20 + (i * 13) % 101, 500 + 97 * i, "f64"
        else:
            m, n, store = 160, 1500, ("f32" if i % 2 else "f64")
        p = datagen.make_problem("c1", seed=100 + i, m=m, n=n, store=store)
        A, b = _upload(p)
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        probs.append(dict(A=A, b=b, lambda1=p.lam1, lambda2=p.lam2, tol=1e-10, x_out=x,
                          sigma0=(0.01 * (i % 3) if i % 3 else 0.0), m=m))
        keep.append(p)
    _say("batch of 40 (32 one-workgroup)")
    infos, rc = gpu.ssnal_en_solve_batch(ctx, probs)
    assert rc == 0, infos
    for i, (pr, p, info) in enumerate(zip(probs, keep, infos)):
        assert info["status"] == 0, (i, info)
        assert info["one_workgroup"] == (1 if i < 32 else 0), (i, info)
        x = pr["x_out"].cpu().numpy()
        AT64 = p.AT64 if p.store != "f64" else p.AT
        check_eta(orc, AT64, p.b, x, p.lam1, p.lam2, 1e-10, eta_gpu=info["kkt_rel"])
        if i < 32:
            opts = gpu.make_opts(sigma0=pr["sigma0"]) if pr["sigma0"] > 0 else None
            A, b = _upload(p)
            xs, si = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10, opts=opts)
            assert si["one_workgroup"] == (1 if _single_one_wg(p.m, p.n) else 0), (i, si)
            if si["one_workgroup"]:
                assert np.array_equal(xs.cpu().numpy(), x), i
            else:
                assert np.max(np.abs(xs.cpu().numpy() - x)) <= 1e-9, i


def test_batch_padded_lda_warm_start(gpu, ctx, orc):
    """Batched one-workgroup solves of a C1 problem (above the single-solve
    limit) with lda > m and NaN padding rows, cold and warm-started from
    another point with x0 the output buffer itself: both reach the oracle's
    minimiser."""
    import datagen
    p = datagen.make_problem("c1", seed=17)
    A, b = _upload(p, lda=p.m + 4)
    _say("batch: padded lda + warm start")
    x_cold, ic = _solve1(gpu, ctx, A, b, p, 1e-10, m=p.m)
    assert ic["one_workgroup"] == 1 and ic["status"] == 0
    q = datagen.make_problem("c1", seed=17)
    q.lam1, q.lam2 = p.lam1 * 1.2, p.lam2 * 1.2
    x1, _ = _solve1(gpu, ctx, A, b, q, 1e-10, m=p.m)
    x_warm, iw = _solve1(gpu, ctx, A, b, p, 1e-10, x0=x1, x_out=x1, m=p.m)
    assert iw["one_workgroup"] == 1 and iw["status"] == 0
    xr, _, _ = orc.en_solve(p.AT, p.b, p.lam1, p.lam2, tol=1e-11)
    assert np.max(np.abs(x_cold.cpu().numpy() - xr)) <= 1e-8
    assert np.max(np.abs(x_warm.cpu().numpy() - xr)) <= 1e-8


def test_served_small_requests(gpu, ctx, orc):
    """Small FP64 requests through the serving loop run in one workgroup:
    each result is its single solve's bits, alone or in a mix with a larger
    FP32 request, and meets the oracle bar."""
    import datagen
    import torch
    reqs = []
    for i, (m, n, store) in enumerate([(40, 900, "f64"), (100, 1200, "f64"), (300, 20000, "f32"),
                                       (64, 2000, "f64")]):
        p = datagen.make_problem("c1", seed=300 + i, m=m, n=n, store=store)
        A, b = _upload(p)
        xa, ia = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-9)
        assert ia["status"] == 0 and ia["one_workgroup"] == (1 if store == "f64" else 0)
        reqs.append((p, A, b, xa.clone(), torch.full((n,), float("nan"), dtype=torch.float64,
                                                   device=A.device)))
    torch.cuda.synchronize()
    _say("served small requests")
    srv = gpu.Server(0, hbm_budget=2 << 30, max_slots=3)
    try:
        tickets = [srv.submit(A, b, p.lam1, p.lam2, 1e-9, x) for p, A, b, _, x in reqs]
        infos = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    torch.cuda.synchronize()
    for (p, A, b, xa, x), info in zip(reqs, infos):
        assert info["status"] == 0, info
        assert bool((x == xa).all())
        if p.store == "f64":
            assert info["one_workgroup"] == 1
            check_eta(orc, p.AT, p.b, x.cpu().numpy(), p.lam1, p.lam2, 1e-9, eta_gpu=info["kkt_rel"])


def test_batch_lasso_and_not_converged(gpu, ctx, orc):
    """A batch of one-workgroup problems mixing the Lasso (lambda2 = 0) with
    elastic nets meets the oracle bar per problem and gives each problem's
    single-solve bits; the same batch capped at one outer iteration at a
    tight tol returns SSNAL_NOT_CONVERGED for every problem, with finite
    certificates of the returned points."""
    import datagen
    import torch
    probs, keep = [], []
    for i in range(6):
        p = datagen.make_problem("c1", seed=600 + i, m=40 + 13 * i, n=700 + 50 * i)
        if i % 2 == 0:
            p.lam2 = 0.0
        A, b = _upload(p)
        probs.append(dict(A=A, b=b, lambda1=p.lam1, lambda2=p.lam2, tol=1e-10,
                          x_out=torch.full((p.n,), float("nan"), dtype=torch.float64, device=A.device)))
        keep.append(p)
    _say("batch: lasso mix")
    infos, rc = gpu.ssnal_en_solve_batch(ctx, probs)
    assert rc == 0, infos
    for pr, p, info in zip(probs, keep, infos):
        assert info["one_workgroup"] == 1 and info["status"] == 0, info
        x = pr["x_out"].cpu().numpy()
        check_eta(orc, p.AT, p.b, x, p.lam1, p.lam2, 1e-10, eta_gpu=info["kkt_rel"])
        xr, ir, _ = orc.en_solve(p.AT, p.b, p.lam1, p.lam2, tol=1e-11)
        F = orc.primal_obj(p.AT, p.b, x, p.lam1, p.lam2)
        assert _rel_obj(F, ir["primal_obj"]) <= 1e-10, (F, ir["primal_obj"])
        assert _support_ok(x, xr)
        xs, si = gpu.ssnal_en_solve(ctx, pr["A"], pr["b"], p.lam1, p.lam2, tol=1e-10)
        assert si["one_workgroup"] == 1
        assert np.array_equal(xs.cpu().numpy(), x)
    _say("batch: max_outer = 1")
    for pr in probs:
        pr["tol"] = 1e-14
        pr["x_out"].fill_(float("nan"))
    infos, rc = gpu.ssnal_en_solve_batch(ctx, probs, opts=gpu.make_opts(max_outer=1))
    assert rc == 1
    for pr, info in zip(probs, infos):
        assert info["one_workgroup"] == 1 and info["status"] == 1 and info["outer_iters"] == 1, info
        assert np.isfinite(info["kkt_rel"]) and info["kkt_rel"] > 1e-14
        assert bool(torch.isfinite(pr["x_out"]).all())


@pytest.mark.parametrize("bad", [float("inf"), float("nan")])
def test_nonfinite_design(gpu, ctx, bad):
    """An Inf or NaN entry of A is refused with SSNAL_ENONFINITE by the single
    solve in one workgroup, by a batch of one, and by the multi-kernel path;
    the context keeps working afterwards."""
    import datagen
    import torch
    p = datagen.make_problem("c1", seed=700, n=1000)
    A, b = _upload(p)
    A[7, 5] = bad  # row 7 of the (n, lda) array: column 7 of A, row 5
    _say("non-finite design", bad)
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10)
    assert e.value.code == -2
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10, opts=gpu.make_opts(no_small=1))
    assert e.value.code == -2
    x = torch.empty(p.n, dtype=torch.float64, device=A.device)
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_en_solve_batch(ctx, [dict(A=A, b=b, lambda1=p.lam1, lambda2=p.lam2, tol=1e-10, x_out=x)])
    assert e.value.code == -2
    A[7, 5] = float(p.AT[7, 5])
    x, info = gpu.ssnal_en_solve(ctx, A, b, p.lam1, p.lam2, tol=1e-10)
    assert info["status"] == 0 and info["one_workgroup"] == 1
