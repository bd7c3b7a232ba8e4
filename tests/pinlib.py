"""Independent reference computations used to pin the oracle.

Nothing here calls the oracle: these are brute-force, closed-form and
textbook-algorithm routes to the same mathematical objects (numpy / scipy
only), so that a mistake in the oracle shows up as a disagreement.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import minimize_scalar


def soft(v, thr):
    return np.sign(v) * np.maximum(np.abs(v) - thr, 0.0)


def argmin_1d(f, lo, hi, tol=1e-13):
    """Minimise a convex 1-D function on [lo, hi] (bounded Brent, then a
    golden-section polish)."""
    r = minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": tol, "maxiter": 2000})
    a, c = r.x - 1e-6 * (hi - lo), r.x + 1e-6 * (hi - lo)
    a, c = max(a, lo), min(c, hi)
    gr = (np.sqrt(5.0) - 1.0) / 2.0
    for _ in range(200):
        x1 = c - gr * (c - a)
        x2 = a + gr * (c - a)
        if f(x1) <= f(x2):
            c = x2
        else:
            a = x1
        if c - a < tol:
            break
    xm = 0.5 * (a + c)
    return xm if f(xm) <= f(r.x) else r.x


def en_penalty(x, l1, l2):
    return l1 * np.sum(np.abs(x)) + 0.5 * l2 * np.sum(np.asarray(x) ** 2)


def brute_force_en(A, b, l1, l2):
    """Exact elastic-net minimiser for n <= 12 by enumerating supports and
    sign patterns: on support S with signs s the stationarity condition is
    (A_S^T A_S + l2 I) x_S = A_S^T b - l1 s; a candidate is valid when
    sign(x_S) = s and |a_i^T (b - A_S x_S)| <= l1 off the support.  The valid
    candidate of least objective is returned (unique: l2 > 0 makes the
    objective strongly convex)."""
    m, n = A.shape
    assert n <= 12
    best, bestF = np.zeros(n), 0.5 * float(b @ b)
    c0 = A.T @ b
    for size in range(1, n + 1):
        for S in itertools.combinations(range(n), size):
            S = list(S)
            AS = A[:, S]
            G = AS.T @ AS + l2 * np.eye(size)
            signs = np.array(list(itertools.product((-1.0, 1.0), repeat=size))).T  # size x 2^size
            X = np.linalg.solve(G, c0[S][:, None] - l1 * signs)
            ok = np.all(X * signs > 0, axis=0)
            if not ok.any():
                continue
            for k in np.nonzero(ok)[0]:
                xS = X[:, k]
                res = b - AS @ xS
                off = [i for i in range(n) if i not in S]
                if off and np.max(np.abs(A[:, off].T @ res)) > l1 * (1 + 1e-10) + 1e-14:
                    continue
                x = np.zeros(n)
                x[S] = xS
                F = 0.5 * float(res @ res) + en_penalty(x, l1, l2)
                if F < bestF:
                    best, bestF = x, F
    return best, bestF


def coordinate_descent_en(A, b, l1, l2, max_sweeps=100000, tol=1e-15):
    """Cyclic coordinate descent with exact coordinate minimisation
    x_j <- soft(a_j^T r + |a_j|^2 x_j, l1) / (|a_j|^2 + l2)."""
    m, n = A.shape
    x = np.zeros(n)
    r = b.copy()
    nrm = np.einsum("ij,ij->j", A, A)
    active = np.arange(n)
    for sweep in range(max_sweeps):
        full = (sweep % 10 == 0)
        idx = np.arange(n) if full else active
        maxd = 0.0
        for j in idx:
            aj = A[:, j]
            old = x[j]
            z = aj @ r + nrm[j] * old
            new = soft(z, l1) / (nrm[j] + l2)
            if new != old:
                r -= aj * (new - old)
                x[j] = new
                maxd = max(maxd, abs(new - old))
        if full:
            active = np.nonzero(x)[0]
            if maxd <= tol * max(1.0, np.max(np.abs(x))):
                break
    return x


def primal_objective(A, b, x, l1, l2):
    r = A @ x - b
    return 0.5 * float(r @ r) + en_penalty(x, l1, l2)


def kkt_violation(A, b, x, l1, l2):
    """max violation of 0 in A^T(Ax-b) + l2 x + l1 d|x|_1, scaled by (1 + max|A^T b|)."""
    g = A.T @ (A @ x - b) + l2 * x
    nz = x != 0
    v1 = np.abs(g[nz] + l1 * np.sign(x[nz]))
    v0 = np.maximum(np.abs(g[~nz]) - l1, 0.0)
    v = max(v1.max(initial=0.0), v0.max(initial=0.0))
    return v / (1.0 + np.max(np.abs(A.T @ b)))


def orthonormal_design(m, n, seed):
    g = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(g.standard_normal((m, n)))
    return Q  # m x n with Q^T Q = I_n (m >= n)


def gaussian_problem(m, n, seed, k=3, c_lam=0.5, alpha=0.5, noise=0.3):
    g = np.random.default_rng(seed)
    A = g.standard_normal((m, n))
    A -= A.mean(axis=0)
    A /= np.linalg.norm(A, axis=0)
    x = np.zeros(n)
    idx = g.choice(n, size=min(k, n), replace=False)
    x[idx] = g.uniform(1, 3, size=idx.size) * np.where(g.random(idx.size) < 0.5, -1, 1)
    b = A @ x + noise * g.standard_normal(m)
    lmax = np.max(np.abs(A.T @ b)) / alpha
    return A, b, alpha * c_lam * lmax, (1 - alpha) * c_lam * lmax
