"""Kernel-level parity of the HIP path against the FP64 oracle (through the C ABI).

Inputs are seeded and synthetic; each case prints what it runs before it runs
it.  Sizes span several tiles and a ragged tail.
"""
import numpy as np
import pytest

from tests import pinlib

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx(gpu):
    return gpu.Context(0)


def _design(m, n, seed, store="f64"):
    import datagen
    AT, AT64 = datagen.make_design("gauss", m, n, seed, store)
    return AT, AT64


def _dev(AT, store, lda=None):
    from paper_2006_03970_amd.device import design_to_device
    return design_to_device(AT, store, lda=lda)


def _vec(v):
    from paper_2006_03970_amd.device import vec_to_device
    return vec_to_device(v)


# ----------------------------------------------------------------- A^T v
GEMV_CASES = [
    (100, 2000, "f64", None), (500, 3001, "f64", None), (1000, 777, "f64", None),
    (2000, 513, "f64", None), (37, 1000, "f64", None), (500, 3001, "f64", 504),
    (500, 3001, "f32", None), (1000, 1000, "f32", None), (37, 999, "f32", 40),
    (500, 3001, "bf16", None), (1000, 1000, "bf16", None), (100, 513, "bf16", 104),
    (3000, 257, "f64", None),
    # 8-byte loads (column stride a multiple of 8 but not of 16 bytes) and the
    # element-wise kernel (stride not a multiple of 8 bytes)
    (502, 1001, "f32", None), (252, 700, "bf16", None), (4000, 300, "bf16", 4004),
    (250, 1500, "bf16", None),
    # column stride 8 mod 16 bytes with odd column counts, m at the 8-byte
    # kernel's register caps, and columns shorter than one load
    (101, 777, "f64", None), (2046, 301, "f32", None), (1020, 1001, "bf16", None),
    (4, 101, "bf16", None), (2, 3, "f64", 3),
]


@pytest.mark.parametrize("m,n,store,lda", GEMV_CASES)
@pytest.mark.parametrize("acc64", [False, True])
def test_gemv_t(gpu, ctx, orc, m, n, store, lda, acc64):
    _say("gemv_t", m, n, store, lda, acc64)
    AT, AT64 = _design(m, n, 1000 + m + n, store)
    v = np.random.default_rng(m * n).standard_normal(m)
    w_ref = orc.gemv_t(AT64, v)
    A = _dev(AT, store, lda)
    w = gpu.ssnal_gemv_t(ctx, A, _vec(v), acc64=acc64, m=m).cpu().numpy()
    # |w - w_ref| <= gamma * |a_j|^T |v| with the unit roundoff of the accumulation
    u = 2.0 ** -53 if (store == "f64" or acc64) else 2.0 ** -24
    bound = (2 * m * u + (0 if (store == "f64" or acc64) else 2.0 ** -24)) * (np.abs(AT64) @ np.abs(v))
    assert np.all(np.abs(w - w_ref) <= bound + 1e-300), np.max(np.abs(w - w_ref) / (bound + 1e-300))


# ----------------------------------------------------------------- active set + prox
@pytest.mark.parametrize("n", [1, 2047, 2048, 2049, 100_000, 300_001])
def test_active_prox_bit_exact(gpu, ctx, orc, n):
    _say("active_prox", n)
    g = np.random.default_rng(n)
    x = np.zeros(n)
    nz = g.choice(n, size=max(1, n // 50), replace=False)
    x[nz] = g.standard_normal(nz.size)
    w = g.standard_normal(n)
    sigma, l1, l2 = 0.731, 1.3, 0.45
    # plant exact ties |t| = sigma*lambda1 (w = 0 makes t = x exactly)
    thr = sigma * l1
    k = min(n, 7)
    w[:k] = 0.0
    x[:k] = [thr, -thr, thr, 0.0, -thr, thr, 2 * thr][:k]
    Jr, ur = orc.active_prox(x, w, sigma, l1, l2)
    J, uJ = gpu.ssnal_active_prox(ctx, _vec(x), _vec(w), sigma, l1, l2)
    assert np.array_equal(J.cpu().numpy(), Jr)
    assert np.array_equal(uJ.cpu().numpy(), ur)  # bit for bit


def test_active_prox_empty(gpu, ctx, orc):
    _say("active_prox empty")
    n = 5000
    x = np.zeros(n)
    w = np.full(n, 1e-3)
    J, uJ = gpu.ssnal_active_prox(ctx, _vec(x), _vec(w), 1.0, 10.0, 1.0)
    assert J.numel() == 0


# ----------------------------------------------------------------- Newton matrix
def _active(m, n, r, seed):
    g = np.random.default_rng(seed)
    return np.sort(g.choice(n, size=r, replace=False)).astype(np.int32)


NM_CASES = [(100, 500, 60), (100, 2000, 400), (130, 700, 250), (500, 4000, 900), (500, 4000, 37),
            (257, 3000, 200), (64, 100, 64),
            # the m x m system at the serving workload's largest m, and past it
            (1000, 6000, 1500), (2000, 8000, 2600), (2000, 8000, 700),
            # 128-tile kernel (N >= 256 outputs over K >= 4096 terms): ragged N
            # and K, with the column pitch a whole number of 16-byte chunks
            (296, 9000, 5000), (520, 12000, 4100)]


@pytest.mark.parametrize("m,n,r", NM_CASES)
@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
def test_newton_matrix(gpu, ctx, orc, m, n, r, store):
    import torch
    _say("newton_matrix", m, n, r, store)
    AT, AT64 = _design(m, n, 7 + m + r, store)
    J = _active(m, n, r, m + r)
    kappa = 0.83
    A = _dev(AT, store)
    Jd = torch.from_numpy(J).cuda()
    tol = 1e-12 if store == "f64" else 3e-6  # FP32 accumulation inside a split
    V = gpu.ssnal_newton_matrix(ctx, A, Jd, kappa, 0).cpu().numpy()
    Vr = orc.newton_matrix(AT64, J, kappa)
    assert np.array_equal(V, V.T)
    assert np.max(np.abs(V - Vr)) <= tol * max(1.0, np.max(np.abs(Vr)))
    if r <= 1024:
        W = gpu.ssnal_newton_matrix(ctx, A, Jd, kappa, 1).cpu().numpy()
        Wr = orc.smw_matrix(AT64, J, kappa)
        assert np.array_equal(W, W.T)
        assert np.max(np.abs(W - Wr)) <= tol * max(1.0, np.max(np.abs(Wr)))


# r x r system of the Woodbury form over long columns (K = m >= 4096): the
# 128-tile kernel where the column pitch is a whole number of 16-byte chunks
# (m = 4104 for every storage; m = 4100 is one for FP32 and FP64 but not for
# BF16, which takes the 64-tile kernel), and a padded pitch
SMW_LONG_CASES = [(4104, 5000, 300, None), (4100, 5000, 257, None), (4100, 3000, 390, 4112)]


@pytest.mark.parametrize("m,n,r,lda", SMW_LONG_CASES)
@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
def test_smw_matrix_long_columns(gpu, ctx, orc, m, n, r, lda, store):
    import torch
    _say("smw_matrix long", m, n, r, lda, store)
    AT, AT64 = _design(m, n, 11 + m + r, store)
    J = _active(m, n, r, m + 3 * r)
    kappa = 1.7
    A = _dev(AT, store, lda=lda)
    Jd = torch.from_numpy(J).cuda()
    tol = 1e-12 if store == "f64" else 3e-6
    W = gpu.ssnal_newton_matrix(ctx, A, Jd, kappa, 1, m=m).cpu().numpy()
    Wr = orc.smw_matrix(AT64, J, kappa)
    assert np.array_equal(W, W.T)
    assert np.max(np.abs(W - Wr)) <= tol * max(1.0, np.max(np.abs(Wr)))


# ----------------------------------------------------------------- Cholesky
@pytest.mark.parametrize("N", [1, 5, 64, 100, 128, 129, 200, 500, 1000, 2000, 4095, 4096])
def test_cholesky(gpu, ctx, orc, N):
    import torch
    _say("cholesky", N)
    g = np.random.default_rng(N)
    M = g.standard_normal((N, N + 20)) / np.sqrt(N)
    V = np.eye(N) + 2.0 * M @ M.T
    Lr = orc.cholesky(V)
    Vd = torch.from_numpy(V.copy()).cuda()
    L = gpu.ssnal_cholesky(ctx, Vd).cpu().numpy()
    assert np.all(np.triu(L, 1) == 0.0)
    assert np.max(np.abs(L - Lr)) <= 1e-12 * np.max(np.abs(Lr)) * max(1.0, np.sqrt(N))


@pytest.mark.parametrize("N,row", [(10, 0), (200, 150), (200, 180), (1000, 999), (300, 64)])
def test_cholesky_not_pd(gpu, ctx, N, row):
    """A non-positive pivot in the first or a later block step, in either
    half of a block, is reported with its row (the first one met)."""
    import torch
    _say("cholesky not PD", N, row)
    g = np.random.default_rng(N + row)
    M = g.standard_normal((N, N)) * 0.01
    V = np.eye(N) + M @ M.T
    V[row, :] = 0.0
    V[:, row] = 0.0
    V[row, row] = -1.0
    V[min(row + 3, N - 1), min(row + 3, N - 1)] = -1.0  # a later bad pivot does not replace it
    with pytest.raises(gpu.SsnalError) as e:
        gpu.ssnal_cholesky(ctx, torch.from_numpy(V).cuda())
    assert e.value.code == -5
    assert f"row {row}" in str(e.value), str(e.value)


# ----------------------------------------------------------------- Newton direction
DIR_CASES = [(100, 2000, 76, "f64"), (100, 2000, 150, "f64"), (500, 5000, 208, "f64"),
             (500, 5000, 700, "f64"), (500, 5000, 60, "f64"), (300, 3000, 299, "f64"),
             (500, 5000, 208, "f32"), (500, 5000, 700, "bf16"), (40, 300, 0, "f64"),
             # systems past 544 rows (backward substitution streams rows it cannot
             # hold), even and odd orders
             (1000, 4000, 900, "f64"), (999, 4000, 901, "f64"),
             # m = 2000 (the serving workload's largest m) in both forms, and the
             # Woodbury form at r = 4000 (m = 4500: no m x m system exists)
             (2000, 8000, 2600, "f64"), (2000, 8000, 1300, "f64"), (2000, 8000, 1300, "f32"),
             (4500, 9000, 4000, "f64")]


@pytest.mark.parametrize("m,n,r,store", DIR_CASES)
def test_newton_direction(gpu, ctx, orc, m, n, r, store):
    import torch
    _say("newton_direction", m, n, r, store)
    AT, AT64 = _design(m, n, 31 + m + r, store)
    J = _active(m, n, r, 5 * m + r)
    kappa = 1.7
    gvec = np.random.default_rng(r + 1).standard_normal(m)
    dr = orc.newton_direction(AT64, J, kappa, gvec)
    A = _dev(AT, store)
    Jd = torch.from_numpy(J).cuda()
    tol = 1e-10 if store == "f64" else 1e-4
    forms = ([0] if m <= 4096 else []) + [-1] + ([1] if 0 < r < m else [])
    for form in forms:
        d = gpu.ssnal_newton_direction(ctx, A, Jd, kappa, _vec(gvec), form=form).cpu().numpy()
        assert np.linalg.norm(d - dr) <= tol * np.linalg.norm(dr), form


# ----------------------------------------------------------------- line search
@pytest.mark.parametrize("n", [3000, 100_000])
def test_ls_delta(gpu, ctx, orc, n):
    _say("ls_delta", n)
    g = np.random.default_rng(n + 3)
    sigma, l1, l2 = 0.9, 0.8, 0.3
    t = g.standard_normal(n) * 1.5
    wd = g.standard_normal(n) * 0.7
    gd, dd = -3.2, 5.1
    steps = [0.5 ** k for k in range(31)]
    ref = [orc.ls_delta(t, wd, s, sigma, l1, l2, gd, dd) for s in steps]
    # x = t and w = 0 make the kernel's t = fma(-sigma, 0, t) = t exactly
    got = gpu.ssnal_ls_delta(ctx, _vec(t), _vec(np.zeros(n)), _vec(wd), sigma, l1, l2, gd, dd, steps)
    for a, b_ in zip(got, ref):
        assert a == pytest.approx(b_, rel=1e-11, abs=1e-12 * (abs(gd) + dd))


# ----------------------------------------------------------------- certificates
@pytest.mark.parametrize("store", ["f64", "f32", "bf16"])
def test_kkt_certificates(gpu, ctx, orc, store):
    _say("kkt", store)
    m, n = 200, 5000
    AT, AT64 = _design(m, n, 77, store)
    g = np.random.default_rng(78)
    b = g.standard_normal(m)
    x = np.zeros(n)
    idx = g.choice(n, 40, replace=False)
    x[idx] = g.standard_normal(40)
    l1, l2 = 0.4, 0.2
    out = gpu.ssnal_kkt(ctx, _dev(AT, store), _vec(b), _vec(x), l1, l2)
    assert out["eta"] == pytest.approx(orc.eta(AT64, b, x, l1, l2), rel=1e-11)
    assert out["primal_obj"] == pytest.approx(orc.primal_obj(AT64, b, x, l1, l2), rel=1e-12)
    assert out["dual_obj"] == pytest.approx(orc.dual_obj(AT64, b, AT64.T @ x - b, l1, l2), rel=1e-11)
