"""Pins of the FP64 oracle against facts that do not come from the oracle.

Primitives (prox pair, conjugate, psi, grad psi, Newton matrix, Cholesky,
line-search increment) are checked against numeric 1-D optimisation, finite
differences, the Moreau identity and library routines; the whole solve is
checked against closed forms, brute-force enumeration, KKT certificates,
duality gaps, a coordinate-descent solver and invariances.
"""
import os

import numpy as np
import pytest

from tests import pinlib

HERE = os.path.dirname(os.path.abspath(__file__))
RNG = np.random.default_rng(20200606)


# ---------------------------------------------------------------- primitives

def test_fig1_values(orc):
    """Prox pair and conjugate at the Fig. 1 setting (lambda1=lambda2=sigma=1)."""
    tab = np.loadtxt(os.path.join(HERE, "golden", "fig1_prox_en.txt"))
    for v, psp, pps, pv, psv in tab:
        assert orc.prox_sp(v, 1.0, 1.0, 1.0) == pytest.approx(psp, abs=1e-15)
        assert orc.prox_pstar(v, 1.0, 1.0, 1.0) == pytest.approx(pps, abs=1e-15)
        assert orc.pstar(np.array([v]), 1.0, 1.0) == pytest.approx(psv, abs=1e-15)
        assert pinlib.en_penalty(np.array([v]), 1.0, 1.0) == pytest.approx(pv, abs=1e-15)


@pytest.mark.parametrize("case", range(12))
def test_prox_sp_is_argmin(orc, case):
    """eq. prox_elastic (left) against the definition eq. prox_op, minimised numerically."""
    g = np.random.default_rng(100 + case)
    sigma, l1, l2 = g.uniform(0.05, 5), g.uniform(0.0, 2), g.uniform(0.01, 3)
    t = g.uniform(-4, 4) * max(1.0, sigma * l1)
    f = lambda u: l1 * abs(u) + 0.5 * l2 * u * u + (u - t) ** 2 / (2 * sigma)
    u_num = pinlib.argmin_1d(f, -abs(t) - 1, abs(t) + 1)
    # a numeric argmin is accurate to ~sqrt(eps) relative (the objective is flat there)
    assert orc.prox_sp(t, sigma, l1, l2) == pytest.approx(u_num, abs=1e-6 * (1 + abs(u_num)))


@pytest.mark.parametrize("case", range(12))
def test_pstar_is_sup(orc, case):
    """Prop. 1 against sup_x (z x - p(x)) computed numerically."""
    g = np.random.default_rng(200 + case)
    l1, l2 = g.uniform(0.01, 2), g.uniform(0.05, 3)
    z = g.uniform(-5, 5)
    f = lambda x: -(z * x - l1 * abs(x) - 0.5 * l2 * x * x)
    xs = pinlib.argmin_1d(f, -50, 50)
    assert orc.pstar(np.array([z]), l1, l2) == pytest.approx(-f(xs), abs=1e-9)


@pytest.mark.parametrize("case", range(12))
def test_prox_pstar_moreau_and_argmin(orc, case):
    """eq. prox_elastic (right): Moreau decomposition and the prox definition of p*/sigma."""
    g = np.random.default_rng(300 + case)
    sigma, l1, l2 = g.uniform(0.05, 5), g.uniform(0.01, 2), g.uniform(0.05, 3)
    v = g.uniform(-4, 4) * max(1.0, sigma * l1)
    a = orc.prox_sp(v, sigma, l1, l2)
    c = orc.prox_pstar(v, sigma, l1, l2)
    assert a + sigma * c == pytest.approx(v, rel=1e-14, abs=1e-14)
    # prox_{p*/sigma}(v/sigma) = argmin_z p*(z)/sigma + |z - v/sigma|^2 / 2
    f = lambda z: orc.pstar(np.array([z]), l1, l2) / sigma + 0.5 * (z - v / sigma) ** 2
    z_num = pinlib.argmin_1d(f, -abs(v / sigma) - 5, abs(v / sigma) + 5)
    assert c == pytest.approx(z_num, abs=1e-6 * (1 + abs(z_num)))


def _small_problem(seed, m=12, n=40):
    g = np.random.default_rng(seed)
    A, b, l1, l2 = pinlib.gaussian_problem(m, n, seed, k=4, c_lam=0.4)
    x = np.zeros(n)
    idx = g.choice(n, 6, replace=False)
    x[idx] = g.standard_normal(6)
    y = g.standard_normal(m)
    sigma = g.uniform(0.3, 3.0)
    return A, b, l1, l2, x, y, sigma


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_psi_is_min_over_z(orc, seed):
    """Prop. 2 (1): psi(y) = min_z L_sigma(y, z | x), minimised coordinate-wise."""
    A, b, l1, l2, x, y, sigma = _small_problem(seed)
    w = A.T @ y
    total = 0.5 * y @ y + b @ y
    for i in range(A.shape[1]):
        f = lambda z: (orc.pstar(np.array([z]), l1, l2) - x[i] * (w[i] + z)
                       + 0.5 * sigma * (w[i] + z) ** 2)
        c = -w[i] + x[i] / sigma
        zi = pinlib.argmin_1d(f, c - 20, c + 20)
        total += f(zi)
    assert orc.psi(A.T, b, x, y, sigma, l1, l2) == pytest.approx(total, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_grad_psi_finite_differences(orc, seed):
    """eq. grad_phy against central differences of psi (psi is C^1)."""
    A, b, l1, l2, x, y, sigma = _small_problem(seed)
    g = orc.grad_psi(A.T, b, x, y, sigma, l1, l2)
    h = 1e-6
    fd = np.array([(orc.psi(A.T, b, x, y + h * e, sigma, l1, l2)
                    - orc.psi(A.T, b, x, y - h * e, sigma, l1, l2)) / (2 * h)
                   for e in np.eye(A.shape[0])])
    assert np.max(np.abs(fd - g)) <= 1e-6 * (1 + np.max(np.abs(g)))


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_newton_matrix_is_generalized_hessian(orc, seed):
    """eq. Q_def / eq. AJ_system: V e_k equals the derivative of grad psi along
    e_k wherever the active set is locally constant."""
    A, b, l1, l2, x, y, sigma = _small_problem(seed)
    m = A.shape[0]
    w = A.T @ y
    J, _ = orc.active_prox(x, w, sigma, l1, l2)
    kappa = sigma / (1 + sigma * l2)
    V = orc.newton_matrix(A.T, J, kappa)
    h = 1e-7
    for k in range(m):
        e = np.zeros(m)
        e[k] = h
        Jp, _ = orc.active_prox(x, A.T @ (y + e), sigma, l1, l2)
        Jm, _ = orc.active_prox(x, A.T @ (y - e), sigma, l1, l2)
        if not (np.array_equal(Jp, J) and np.array_equal(Jm, J)):
            continue
        col = (orc.grad_psi(A.T, b, x, y + e, sigma, l1, l2)
               - orc.grad_psi(A.T, b, x, y - e, sigma, l1, l2)) / (2 * h)
        assert np.max(np.abs(col - V[:, k])) <= 1e-6 * (1 + np.max(np.abs(V)))
    assert np.allclose(V, V.T)


def test_active_set_rule_and_tie(orc):
    """eq. Q_def: strict inequality; a tie |t| = sigma*lambda1 is inactive."""
    sigma, l1, l2 = 0.5, 2.0, 0.3
    thr = sigma * l1
    x = np.array([thr, -thr, thr + 1e-9, 0.0, 3.0, -3.0])
    w = np.zeros_like(x)
    J, uJ = orc.active_prox(x, w, sigma, l1, l2)
    assert J.tolist() == [2, 4, 5]
    for j, u in zip(J, uJ):
        assert u == orc.prox_sp(x[j], sigma, l1, l2)


def test_smw_matrix_woodbury_identity(orc):
    """eq. smw_formula: (I + kappa A_J A_J^T)^{-1} = I - A_J W^{-1} A_J^T with W the r x r matrix."""
    A, b, l1, l2 = pinlib.gaussian_problem(25, 60, 21)
    J = np.array([2, 5, 11, 17, 30, 41, 59], dtype=np.int32)
    kappa = 0.37
    W = orc.smw_matrix(A.T, J, kappa)
    V = orc.newton_matrix(A.T, J, kappa)
    AJ = A[:, J]
    lhs = np.linalg.inv(V)
    rhs = np.eye(25) - AJ @ np.linalg.inv(W) @ AJ.T
    assert np.allclose(lhs, rhs, atol=1e-12)
    assert np.allclose(W, W.T)


def test_cholesky_against_library(orc):
    g = np.random.default_rng(11)
    M = g.standard_normal((30, 50))
    V = np.eye(30) + 0.7 * M @ M.T
    L = orc.cholesky(V)
    assert np.allclose(np.triu(L, 1), 0.0)
    assert np.allclose(L, np.linalg.cholesky(V), rtol=1e-12, atol=1e-12)
    with pytest.raises(np.linalg.LinAlgError):
        orc.cholesky(-np.eye(4))


@pytest.mark.parametrize("seed", [12, 13])
def test_newton_direction_solves_system(orc, seed):
    A, b, l1, l2, x, y, sigma = _small_problem(seed)
    J, _ = orc.active_prox(x, A.T @ y, sigma, l1, l2)
    kappa = sigma / (1 + sigma * l2)
    g = orc.grad_psi(A.T, b, x, y, sigma, l1, l2)
    d = orc.newton_direction(A.T, J, kappa, g)
    V = orc.newton_matrix(A.T, J, kappa)
    assert np.linalg.norm(V @ d + g) <= 1e-12 * (1 + np.linalg.norm(g))
    assert g @ d < 0  # descent direction


@pytest.mark.parametrize("seed", [14, 15, 16])
def test_ls_delta_equals_psi_difference(orc, seed):
    """The line-search increment equals psi(y + s d) - psi(y) (Prop. 2 (1))."""
    A, b, l1, l2, x, y, sigma = _small_problem(seed)
    g = orc.grad_psi(A.T, b, x, y, sigma, l1, l2)
    d = np.random.default_rng(seed).standard_normal(A.shape[0])
    t = x - sigma * (A.T @ y)
    wd = A.T @ d
    for s in (1.0, 0.5, 0.125, 2.0 ** -10):
        got = orc.ls_delta(t, wd, s, sigma, l1, l2, g @ d, d @ d)
        ref = orc.psi(A.T, b, x, y + s * d, sigma, l1, l2) - orc.psi(A.T, b, x, y, sigma, l1, l2)
        assert got == pytest.approx(ref, rel=1e-8, abs=1e-11)


def test_objectives_weak_duality_and_zero_gap(orc):
    """F and D: D(y) <= F(x) for arbitrary x, y; equality at the orthonormal closed form."""
    A = pinlib.orthonormal_design(40, 15, 3)
    g = np.random.default_rng(4)
    b = g.standard_normal(40)
    l1, l2 = 0.3, 0.4
    for _ in range(5):
        x, y = g.standard_normal(15), g.standard_normal(40)
        assert orc.dual_obj(A.T, b, y, l1, l2) <= orc.primal_obj(A.T, b, x, l1, l2) + 1e-12
    xs = pinlib.soft(A.T @ b, l1) / (1 + l2)
    F = orc.primal_obj(A.T, b, xs, l1, l2)
    D = orc.dual_obj(A.T, b, A @ xs - b, l1, l2)
    assert F == pytest.approx(pinlib.primal_objective(A, b, xs, l1, l2), rel=1e-14)
    assert abs(F - D) <= 1e-13 * (1 + F)
    assert orc.eta(A.T, b, xs, l1, l2) <= 1e-15
    assert orc.eta(A.T, b, xs + 1e-3 * g.standard_normal(15), l1, l2) > 1e-5


def test_gemv_against_numpy(orc):
    g = np.random.default_rng(5)
    AT = g.standard_normal((301, 77))
    v = g.standard_normal(77)
    assert np.allclose(orc.gemv_t(AT, v), AT @ v, rtol=1e-13, atol=1e-13)
    x = g.standard_normal(301)
    x[::3] = 0
    assert np.allclose(orc.gemv_n(AT, x), AT.T @ x, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- the solve

def _solve(orc, A, b, l1, l2, tol=1e-12, **kw):
    x, info, _ = orc.en_solve(np.ascontiguousarray(A.T), b, l1, l2, tol=tol, **kw)
    return x, info


@pytest.mark.parametrize("m,n", [(40, 10), (30, 30), (50, 12)])
def test_orthonormal_closed_form(orc, m, n):
    """m >= n and A^T A = I: x_i = soft(a_i^T b, lambda1)/(1 + lambda2)."""
    A = pinlib.orthonormal_design(m, n, m + n)
    b = np.random.default_rng(m * n).standard_normal(m) * 2
    for l1, l2 in [(0.5, 0.25), (0.05, 1.5), (1.2, 0.01)]:
        x, info = _solve(orc, A, b, l1, l2)
        ref = pinlib.soft(A.T @ b, l1) / (1 + l2)
        assert info["status"] == 0
        assert np.max(np.abs(x - ref)) <= 1e-10
        assert np.array_equal(x != 0, ref != 0)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_small(orc, seed):
    """Support/sign enumeration at n <= 12 (both m < n and m > n)."""
    g = np.random.default_rng(500 + seed)
    m, n = (8, 12) if seed % 2 == 0 else (20, 9)
    A, b, l1, l2 = pinlib.gaussian_problem(m, n, 500 + seed, k=3, c_lam=g.uniform(0.15, 0.7),
                                           alpha=g.uniform(0.3, 0.9))
    xb, Fb = pinlib.brute_force_en(A, b, l1, l2)
    x, info = _solve(orc, A, b, l1, l2)
    assert info["status"] == 0
    assert np.max(np.abs(x - xb)) <= 1e-9 * (1 + np.max(np.abs(xb)))
    assert np.array_equal(x != 0, xb != 0)
    assert info["primal_obj"] == pytest.approx(Fb, rel=1e-12)


def test_zero_solution_threshold(orc):
    """x* = 0 iff lambda1 >= ||A^T b||_inf (c_lambda >= 1 in the lambda recipe of Sec. 4.1)."""
    A, b, _, _ = pinlib.gaussian_problem(30, 200, 8)
    lmax = np.max(np.abs(A.T @ b))
    for c, zero in [(1.0, True), (1.01, True), (0.99, False)]:
        x, info = _solve(orc, A, b, c * lmax, 0.3)
        assert info["status"] == 0
        assert (np.count_nonzero(x) == 0) == zero


def test_ridge_limit(orc):
    """lambda1 = 0: x = A^T (A A^T + lambda2 I)^{-1} b (J = all columns)."""
    A, b, _, _ = pinlib.gaussian_problem(20, 60, 9)
    l2 = 0.7
    x, info = _solve(orc, A, b, 0.0, l2)
    ref = A.T @ np.linalg.solve(A @ A.T + l2 * np.eye(20), b)
    assert info["status"] == 0
    assert np.max(np.abs(x - ref)) <= 1e-10


def test_single_feature(orc):
    """n = 1: x = soft(a^T b, lambda1)/(|a|^2 + lambda2)."""
    g = np.random.default_rng(10)
    a = g.standard_normal(15) * 0.8
    b = g.standard_normal(15)
    for l1 in (0.0, 0.3, abs(a @ b) * 0.9, abs(a @ b) * 1.1):
        x, info = _solve(orc, a[:, None], b, l1, 0.45)
        ref = pinlib.soft(a @ b, l1) / (a @ a + 0.45)
        assert info["status"] == 0
        assert x[0] == pytest.approx(ref, abs=1e-11)


def test_kkt_certificate_and_gap(orc):
    """KKT of the primal (0 in A^T(Ax-b) + lambda2 x + lambda1 d|x|_1) and the
    duality gap of the returned point, at the small benchmark workload."""
    import datagen
    p = datagen.make_problem("c1", seed=3)
    A = p.AT.T
    x, info = _solve(orc, A, p.b, p.lam1, p.lam2, tol=1e-10)
    assert info["status"] == 0 and info["eta"] <= 1e-10
    assert pinlib.kkt_violation(A, p.b, x, p.lam1, p.lam2) <= 1e-9
    F = pinlib.primal_objective(A, p.b, x, p.lam1, p.lam2)
    assert info["primal_obj"] == pytest.approx(F, rel=1e-13)
    assert (info["primal_obj"] - info["dual_obj"]) / (1 + F) <= 1e-11


def test_coordinate_descent_cross_check(orc):
    """Independent cyclic coordinate descent reaches the same minimiser."""
    A, b, l1, l2 = pinlib.gaussian_problem(60, 400, 12, k=8, c_lam=0.3)
    x, info = _solve(orc, A, b, l1, l2)
    xc = pinlib.coordinate_descent_en(A, b, l1, l2)
    Fo, Fc = pinlib.primal_objective(A, b, x, l1, l2), pinlib.primal_objective(A, b, xc, l1, l2)
    assert abs(Fo - Fc) <= 1e-12 * Fc
    assert np.max(np.abs(x - xc)) <= 1e-7
    assert np.array_equal(np.abs(x) > 1e-8, np.abs(xc) > 1e-8)


@pytest.mark.parametrize("sigma0,factor", [(5e-3, 5), (0.1, 5), (1.0, 10), (2.5, 5), (10.0, 10)])
def test_sigma_independence(orc, sigma0, factor):
    """The minimiser does not depend on the penalty schedule (Sec. 4.1 and the
    screening runs of the supplement use 5e-3 x5 and 1 x10)."""
    A, b, l1, l2 = pinlib.gaussian_problem(40, 300, 13, k=5, c_lam=0.35)
    x0, _ = _solve(orc, A, b, l1, l2)
    x, info = _solve(orc, A, b, l1, l2, sigma0=sigma0, sigma_factor=factor)
    assert info["status"] == 0
    F0, F = pinlib.primal_objective(A, b, x0, l1, l2), pinlib.primal_objective(A, b, x, l1, l2)
    assert abs(F - F0) <= 1e-12 * F0
    assert np.max(np.abs(x - x0)) <= 1e-8


def test_invariances(orc):
    """Column permutation permutes x; flipping a column flips its coefficient;
    (b, lambda1, lambda2) -> (c b, c lambda1, lambda2) scales x by c."""
    A, b, l1, l2 = pinlib.gaussian_problem(30, 120, 14, k=4, c_lam=0.4)
    x, _ = _solve(orc, A, b, l1, l2)
    perm = np.random.default_rng(1).permutation(120)
    xp, _ = _solve(orc, A[:, perm], b, l1, l2)
    assert np.max(np.abs(xp - x[perm])) <= 1e-10
    A2 = A.copy()
    A2[:, 5] *= -1
    A2[:, 17] *= -1
    x2, _ = _solve(orc, A2, b, l1, l2)
    x_ref = x.copy()
    x_ref[[5, 17]] *= -1
    assert np.max(np.abs(x2 - x_ref)) <= 1e-10
    x3, _ = _solve(orc, A, 3.0 * b, 3.0 * l1, l2)
    assert np.max(np.abs(x3 - 3.0 * x)) <= 1e-9


def test_warm_start_same_point(orc):
    """A warm start from a nearby solution reaches the same minimiser (Sec. 3.4)."""
    A, b, l1, l2 = pinlib.gaussian_problem(40, 500, 15, k=6, c_lam=0.3)
    x1, _ = _solve(orc, A, b, l1 * 1.1, l2 * 1.1)
    x_cold, ic = _solve(orc, A, b, l1, l2)
    x_warm, iw = _solve(orc, A, b, l1, l2, x0=x1)
    assert iw["status"] == 0
    assert np.max(np.abs(x_warm - x_cold)) <= 1e-9


def test_status_not_converged(orc):
    A, b, l1, l2 = pinlib.gaussian_problem(30, 200, 16)
    x, info = _solve(orc, A, b, l1, l2, tol=1e-14, max_outer=1)
    assert info["status"] == 1


# ---------------------------------------------------------------- model selection
# gcv / e-bic (Sec. "Parameter tuning", eq. gcv_bic): nu against the singular
# values of A_J, closed forms and special cases; the de-biased fit against a
# library least-squares solver.

def _ms_problem(seed, m=40, n=120, r=6):
    g = np.random.default_rng(seed)
    AT = g.standard_normal((n, m))
    x = np.zeros(n)
    J = np.sort(g.choice(n, size=r, replace=False))
    x[J] = g.standard_normal(r)
    b = g.standard_normal(m)
    return AT, b, x, J


@pytest.mark.parametrize("seed,l2", [(1, 0.3), (2, 2.0), (3, 1e-3)])
def test_model_select_nu_from_singular_values(orc, seed, l2):
    """nu = tr(A_J (A_J^T A_J + l2 I)^{-1} A_J^T) = sum s_i^2 / (s_i^2 + l2)."""
    AT, b, x, J = _ms_problem(seed)
    s = np.linalg.svd(AT[J].T, compute_uv=False)
    res = orc.model_select(AT, b, x, l2)
    assert res["r"] == J.size
    assert res["nu"] == pytest.approx(np.sum(s * s / (s * s + l2)), rel=1e-12)


def test_model_select_orthonormal_columns(orc):
    """Orthonormal selected columns: nu = r / (1 + l2) exactly."""
    g = np.random.default_rng(4)
    m, n, r = 30, 50, 5
    Q, _ = np.linalg.qr(g.standard_normal((m, r)))
    AT = g.standard_normal((n, m))
    J = np.array([2, 7, 11, 30, 44])
    AT[J] = Q.T
    x = np.zeros(n)
    x[J] = 1.0
    res = orc.model_select(AT, g.standard_normal(m), x, 0.25)
    assert res["nu"] == pytest.approx(r / 1.25, rel=1e-13)


def test_model_select_least_squares(orc):
    """The de-biased fit is least squares on J: b in span(A_J) gives rss = 0
    and beta = the generating coefficients; otherwise rss and beta match a
    library solver."""
    AT, b, x, J = _ms_problem(5)
    c = np.random.default_rng(6).standard_normal(J.size)
    b_in = AT[J].T @ c
    res = orc.model_select(AT, b_in, x, 0.5, want_beta=True)
    assert res["status"] == 0
    assert res["rss"] <= 1e-24 * np.sum(b_in ** 2)
    assert np.allclose(res["beta"][J], c, rtol=1e-10, atol=1e-12)
    res = orc.model_select(AT, b, x, 0.5, want_beta=True)
    beta, *_ = np.linalg.lstsq(AT[J].T, b, rcond=None)
    assert res["rss"] == pytest.approx(np.sum((AT[J].T @ beta - b) ** 2), rel=1e-12)
    assert np.allclose(res["beta"][J], beta, rtol=1e-10, atol=1e-13)
    assert np.all(np.delete(res["beta"], J) == 0.0)
    assert res["rss_en"] == pytest.approx(np.sum((AT.T @ x - b) ** 2), rel=1e-13)


def test_model_select_criteria_definitions(orc):
    """x = 0: r = nu = 0, rss = |b|^2, gcv = |b|^2/m, e-bic = log(|b|^2/m);
    and the criteria follow the (rss, nu) they are computed from."""
    AT, b, x, J = _ms_problem(7)
    m, n = AT.shape[1], AT.shape[0]
    res = orc.model_select(AT, b, np.zeros(n), 0.5)
    bb = float(np.sum(b * b))
    assert (res["r"], res["nu"], res["status"]) == (0, 0.0, 0)
    assert res["rss"] == pytest.approx(bb, rel=1e-14)
    assert res["gcv"] == pytest.approx(bb / m, rel=1e-14)
    assert res["ebic"] == pytest.approx(np.log(bb / m), rel=1e-13)
    res = orc.model_select(AT, b, x, 0.5)
    rss, nu = res["rss"], res["nu"]
    assert 0 < nu < J.size
    assert res["gcv"] == pytest.approx(rss / m / (1 - nu / m) ** 2, rel=1e-13)
    assert res["ebic"] == pytest.approx(np.log(rss / m) + nu / m * (np.log(m) + np.log(n)), rel=1e-13)


def test_model_select_degenerate(orc):
    """r >= m leaves the least-squares fit undetermined; a repeated column
    makes A_J^T A_J singular.  Both are reported, with NaN criteria."""
    g = np.random.default_rng(8)
    m, n = 10, 30
    AT = g.standard_normal((n, m))
    b = g.standard_normal(m)
    x = np.zeros(n)
    x[:12] = 1.0
    res = orc.model_select(AT, b, x, 0.5)
    assert res["status"] == 1 and np.isnan(res["rss"]) and np.isnan(res["gcv"])
    s = np.linalg.svd(AT[:12].T, compute_uv=False)
    assert res["nu"] == pytest.approx(np.sum(s * s / (s * s + 0.5)), rel=1e-12)
    AT[3] = 0.0
    AT[3, :4] = 1.0  # |a|^2 = 4: the second pivot of the repeated column is exactly 0
    AT[5] = AT[3]
    x = np.zeros(n)
    x[[3, 5, 9]] = 1.0
    res = orc.model_select(AT, b, x, 0.5)
    assert res["status"] == 2 and np.isnan(res["ebic"])


# ---------------------------------------------------------------- Lasso limit
# lambda2 = 0 (alpha -> 1): p* is the indicator of |z|_inf <= lambda1 (the
# conjugate of a norm), so the dual objective is taken at the scaled feasible
# point theta*rho, theta = min(1, lambda1/|A^T rho|_inf).

def test_lasso_coordinate_descent_cross_check(orc):
    """lambda2 = 0: the solve reaches the minimiser an independent cyclic
    coordinate descent finds (unique for a Gaussian design in general position)."""
    A, b, l1, _ = pinlib.gaussian_problem(60, 400, 12, k=8, c_lam=0.3)
    x, info = _solve(orc, A, b, l1, 0.0, tol=1e-10)
    assert info["status"] == 0
    xc = pinlib.coordinate_descent_en(A, b, l1, 0.0)
    Fo, Fc = pinlib.primal_objective(A, b, x, l1, 0.0), pinlib.primal_objective(A, b, xc, l1, 0.0)
    assert abs(Fo - Fc) <= 1e-12 * Fc
    assert np.max(np.abs(x - xc)) <= 1e-7
    assert pinlib.kkt_violation(A, b, x, l1, 0.0) <= 1e-9
    assert abs(info["rel_gap"]) <= 1e-9


def test_lasso_conjugate_and_dual_bound(orc):
    """p* with lambda2 = 0 is an indicator; the dual objective of any point is
    a finite lower bound of F (weak duality through the feasible scaling),
    attained at the minimiser."""
    lam = 0.7
    assert orc.pstar(np.array([0.3, -0.7, 0.0]), lam, 0.0) == 0.0
    assert orc.pstar(np.array([0.3, -0.71]), lam, 0.0) == np.inf
    A, b, l1, _ = pinlib.gaussian_problem(50, 200, 3, k=5, c_lam=0.2)
    AT = np.ascontiguousarray(A.T)
    g = np.random.default_rng(9)
    for _ in range(5):
        x = np.where(g.random(200) < 0.05, g.standard_normal(200), 0.0)
        rho = A @ x - b
        assert np.max(np.abs(A.T @ rho)) > l1  # an infeasible dual point
        D = orc.dual_obj(AT, b, rho, l1, 0.0)
        assert np.isfinite(D)
        assert D <= pinlib.primal_objective(A, b, x, l1, 0.0)
        # the bound is the dual objective at the scaled point, by hand
        th = l1 / np.max(np.abs(A.T @ rho))
        assert D == pytest.approx(-(0.5 * th * th * rho @ rho + th * b @ rho), rel=1e-12)
    xs, info = _solve(orc, A, b, l1, 0.0, tol=1e-10)
    assert info["status"] == 0
    rho = A @ xs - b
    assert orc.dual_obj(AT, b, rho, l1, 0.0) == pytest.approx(
        pinlib.primal_objective(A, b, xs, l1, 0.0), rel=1e-10)


# ---------------------------------------------------------------- k-fold CV
# k-fold cross validation (Sec. "Parameter tuning") on the full data's grid.

def test_cv_zero_solution_and_composition(orc):
    """Far above lambda_max every fold's solution is 0 and its error is the
    mean of b^2 over its rows; at an interior point a fold's error equals the
    validation error of a cold solve on that fold's training rows."""
    A, b, _, _ = pinlib.gaussian_problem(60, 300, 3, k=5, c_lam=0.3)
    AT = np.ascontiguousarray(A.T)
    k, alpha = 4, 0.6
    fold = (np.arange(60) * 7) % k
    grid = [20.0, 0.4, 0.15]
    err, rc = orc.cv(AT, b, fold, k, alpha, grid, tol=1e-11)
    assert rc == 0
    for f in range(k):
        assert err[f, 0] == pytest.approx(np.mean(b[fold == f] ** 2), rel=1e-14)
    lam_max = np.max(np.abs(A.T @ b)) / alpha
    for f in (0, 3):
        tr = fold != f
        lam = grid[2] * lam_max
        x, info = _solve(orc, A[tr], b[tr], alpha * lam, (1 - alpha) * lam, tol=1e-11)
        assert info["status"] == 0
        e = np.mean((A[~tr] @ x - b[~tr]) ** 2)
        assert err[f, 2] == pytest.approx(e, rel=1e-8)


# ------------------------------------------- conjugate-gradient Newton direction

def _cg_setup(seed, m=30, n=80, nJ=40):
    g = np.random.default_rng(seed)
    A, _, _, _ = pinlib.gaussian_problem(m, n, seed, k=4, c_lam=0.4)
    J = np.sort(g.choice(n, nJ, replace=False)).astype(np.int32)
    kappa = g.uniform(0.2, 2.0)
    grad = g.standard_normal(m)
    return A, J, kappa, grad


def test_newton_matvec_is_matrix_product(orc):
    """The matrix-free product equals the (pinned) Newton matrix times p."""
    A, J, kappa, _ = _cg_setup(31, nJ=17)
    V = orc.newton_matrix(A.T, J, kappa)
    p = np.random.default_rng(32).standard_normal(A.shape[0])
    np.testing.assert_allclose(orc.newton_matvec(A.T, J, kappa, p), V @ p, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("nJ", [1, 3, 6])
def test_newton_cg_finite_termination(orc, nJ):
    """V = I + kappa A_J A_J^T has at most |J| + 1 distinct eigenvalues, so
    conjugate gradients solve V d = -g in at most |J| + 1 steps."""
    A, J, kappa, g = _cg_setup(40 + nJ, nJ=nJ)
    d, it = orc.newton_cg(A.T, J, kappa, g, 1e-12, maxit=200)
    assert 1 <= it <= nJ + 1
    V = orc.newton_matrix(A.T, J, kappa)
    assert np.linalg.norm(V @ d + g) <= 1e-11 * np.linalg.norm(g)


@pytest.mark.parametrize("seed", [21, 22])
def test_newton_cg_matches_cholesky_direction(orc, seed):
    """Run to a tiny residual, CG gives the direction of the dense solve."""
    A, J, kappa, g = _cg_setup(seed)
    d_ch = orc.newton_direction(A.T, J, kappa, g)
    d_cg, it = orc.newton_cg(A.T, J, kappa, g, 1e-14, maxit=1000)
    assert it <= 200
    assert np.linalg.norm(d_cg - d_ch) <= 1e-10 * np.linalg.norm(d_ch)
    assert g @ d_cg < 0


def test_newton_cg_error_decay_and_first_stop(orc):
    """The V-norm error never grows and obeys the Chebyshev bound
    2((sqrt(c)-1)/(sqrt(c)+1))^k of conjugate gradients (c = cond V); the
    returned iterate is the first whose residual meets the test."""
    A, J, kappa, g = _cg_setup(23)
    V = orc.newton_matrix(A.T, J, kappa)
    dstar = np.linalg.solve(V, -g)
    c = np.linalg.cond(V)
    rho = (np.sqrt(c) - 1) / (np.sqrt(c) + 1)
    errs = []
    for k in range(0, 20):
        d, it = orc.newton_cg(A.T, J, kappa, g, 0.0, maxit=k)
        assert it == k
        e = d - dstar
        errs.append(np.sqrt(e @ V @ e))
    for k in range(1, len(errs)):
        assert errs[k] <= errs[k - 1] * (1 + 1e-10) + 1e-14
        assert errs[k] <= 2 * rho ** k * errs[0] * (1 + 1e-9) + 1e-14
    assert errs[-1] < 1e-3 * errs[0]
    eps = 1e-3
    d, it = orc.newton_cg(A.T, J, kappa, g, eps)
    assert np.linalg.norm(V @ d + g) <= eps * np.linalg.norm(g) * (1 + 1e-9)
    d1, it1 = orc.newton_cg(A.T, J, kappa, g, eps, maxit=it - 1)
    assert it1 == it - 1
    assert np.linalg.norm(V @ d1 + g) > eps * np.linalg.norm(g)


def test_newton_cg_solve_reaches_cd_minimiser(orc):
    """The whole solve with CG directions reaches the coordinate-descent
    minimiser, in at most three times the Newton iterations of the exact-direction
    solve (early directions are inexact by design)."""
    A, b, l1, l2 = pinlib.gaussian_problem(60, 400, 12, k=8, c_lam=0.3)
    x, info = _solve(orc, A, b, l1, l2, newton_cg=1)
    assert info["status"] == 0 and info["cg_iters"] > 0
    xc = pinlib.coordinate_descent_en(A, b, l1, l2)
    Fo, Fc = pinlib.primal_objective(A, b, x, l1, l2), pinlib.primal_objective(A, b, xc, l1, l2)
    assert abs(Fo - Fc) <= 1e-12 * Fc
    assert np.max(np.abs(x - xc)) <= 1e-7
    _, info_ch = _solve(orc, A, b, l1, l2)
    assert info_ch["cg_iters"] == 0
    assert info["newton_iters"] <= 3 * info_ch["newton_iters"]


# ---------------------------------------------------------------- host threads

def test_thread_count_does_not_change_results(orc):
    """The oracle's threaded loops (A^T v, A x, both Newton matrices, the
    Cholesky columns) and a whole solve give the same bits with 1 and 4
    threads; the Cholesky also matches LAPACK past the threading cut-off."""
    g = np.random.default_rng(4242)
    m, n = 300, 700
    AT = g.standard_normal((n, m)) / np.sqrt(m)
    v = g.standard_normal(m)
    x = np.where(g.random(n) < 0.1, g.standard_normal(n), 0.0)
    J = np.sort(g.choice(n, 350, replace=False)).astype(np.int32)
    b = AT.T @ x + 0.1 * g.standard_normal(m)
    l1 = 0.3 * np.max(np.abs(AT @ b))
    saved = orc.get_threads()
    out = []
    try:
        for k in (1, 4):
            orc.set_threads(k)
            V = orc.newton_matrix(AT, J, 0.7)
            xs, info, _ = orc.en_solve(AT, b, l1, 0.2, tol=1e-10)
            out.append((orc.gemv_t(AT, v), orc.gemv_n(AT, x), V, orc.smw_matrix(AT, J[:200], 0.7),
                        orc.cholesky(V), xs, info["primal_obj"]))
    finally:
        orc.set_threads(saved)
    for a, c in zip(*out):
        assert np.array_equal(np.asarray(a), np.asarray(c))
    assert np.allclose(out[0][4], np.linalg.cholesky(out[0][2]), rtol=1e-12, atol=1e-12)
