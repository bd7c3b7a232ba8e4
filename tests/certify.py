"""Certificate checks shared by the GPU parity tests.

A GPU solve stops once its KKT residual eta (the primal natural residual,
FP64 accumulation over the stored design) is at most tol.  The oracle
evaluates the same quantity in FP64 on the same stored values, so the two
must agree to rounding, and the oracle's value must itself meet tol.
"""
from __future__ import annotations

import numpy as np

# both sides compute eta in FP64 over the same stored design; they differ only
# in summation order, which moves eta by far less than this relative amount
ETA_REL = 1e-9


def eta_bound(AT64, b, x, l1, l2, eta):
    """Largest |eta_gpu - eta_oracle| that rounding can explain: both sides
    form rho = A x - b (at most nnz(x) + 1 terms per row) and g = A^T rho (m
    terms per column) in FP64 with their own summation order, then
    e_j = x_j - prox(x_j - g_j) (prox is 1-Lipschitz).  Per feature, twice the
    standard forward-error bound of each sum plus a few ulps of the prox
    arithmetic; eta moves by at most the norm of that over its denominator."""
    u = 2.0 ** -53
    AT64 = np.asarray(AT64)
    m = AT64.shape[1]
    nz = np.flatnonzero(x)
    rho = AT64[nz].T @ x[nz] - b
    absA = np.abs(AT64)
    mag_rho = absA[nz].T @ np.abs(x[nz]) + np.abs(b)
    g = AT64 @ rho
    err_g = 2 * (m + 2) * u * (absA @ np.abs(rho)) + 2 * (nz.size + 2) * u * (absA @ mag_rho)
    err_e = err_g + 8 * u * (np.abs(x) + np.abs(g))
    # a feature with x_j = 0 and |g_j| <= lambda1 on both sides has e_j = 0
    # exactly (the prox returns an exact zero), whatever the rounding of g_j
    live = (x != 0) | (np.abs(g) + err_g > l1)
    den = 1.0 + np.linalg.norm(x) + np.linalg.norm(rho)
    return np.linalg.norm(err_e[live]) / den + 1e-15 * eta


def check_eta(orc, AT64, b, x, l1, l2, tol, eta_gpu=None):
    """The oracle's eta on the stored design meets tol (no slack beyond a
    relative 1e-9 for the last digits), and the GPU's own reported eta is the
    same number to rounding.  Returns the oracle's eta."""
    eta = orc.eta(AT64, b, x, l1, l2)
    assert eta <= tol * (1 + ETA_REL), (eta, tol)
    if eta_gpu is not None:
        diff = abs(eta_gpu - eta)
        print(f"[report] eta oracle {eta:.6e} gpu {eta_gpu:.6e} rel diff {diff / max(eta, 1e-300):.2e}",
              flush=True)
        if diff > ETA_REL * eta:
            assert diff <= eta_bound(AT64, b, x, l1, l2, eta), (eta_gpu, eta, diff)
    return eta
