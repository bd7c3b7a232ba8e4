"""ctypes wrapper of the FP64 CPU oracle (oracle_en.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU solver never does, and
shares no code with it.  Arrays are numpy float64; the design is passed as
AT, an (n, m) C-contiguous array (= A column-major with lda = m).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SSNAL_ORACLE_LIB") or os.path.join(_HERE, "liboracle_en.so")
SRC = os.path.join(_HERE, "oracle_en.c")

# No contraction, no fast-math: IEEE binary64 with one rounding per operation.
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Opts(C.Structure):
    _fields_ = [("sigma0", C.c_double), ("sigma_factor", C.c_double), ("sigma_max", C.c_double),
                ("mu", C.c_double), ("delta", C.c_double), ("max_outer", C.c_int32),
                ("max_inner", C.c_int32), ("max_backtrack", C.c_int32), ("newton_cg", C.c_int32),
                ("cg_maxit", C.c_int32), ("cg_eta", C.c_double), ("cg_tau", C.c_double)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_iters", C.c_int32), ("newton_iters", C.c_int32),
                ("r_final", C.c_int32), ("nnz", C.c_int64), ("eta", C.c_double),
                ("kkt1", C.c_double), ("kkt3", C.c_double), ("primal_obj", C.c_double),
                ("dual_obj", C.c_double), ("rel_gap", C.c_double), ("sigma_final", C.c_double),
                ("cg_iters", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_i64 = C.c_int64
_d = C.c_double


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_prox_sp.restype = _d
        L.orc_prox_sp.argtypes = [_d, _d, _d, _d]
        L.orc_prox_pstar.restype = _d
        L.orc_prox_pstar.argtypes = [_d, _d, _d, _d]
        L.orc_pstar.restype = _d
        L.orc_pstar.argtypes = [_D, _i64, _d, _d]
        L.orc_gemv_t.argtypes = [_D, _i64, _i64, _i64, _D, _D]
        L.orc_gemv_n.argtypes = [_D, _i64, _i64, _i64, _D, _D]
        for f in (L.orc_primal_obj, L.orc_eta):
            f.restype = _d
            f.argtypes = [_D, _i64, _D, _i64, _i64, _D, _d, _d]
        L.orc_dual_obj.restype = _d
        L.orc_dual_obj.argtypes = [_D, _i64, _D, _i64, _i64, _D, _d, _d]
        L.orc_psi.restype = _d
        L.orc_psi.argtypes = [_D, _i64, _D, _i64, _i64, _D, _D, _d, _d, _d]
        L.orc_grad_psi.argtypes = [_D, _i64, _D, _i64, _i64, _D, _D, _d, _d, _d, _D]
        L.orc_active_prox.restype = _i64
        L.orc_active_prox.argtypes = [_D, _D, _i64, _d, _d, _d, _I32, _D]
        L.orc_newton_matrix.argtypes = [_D, _i64, _i64, _I32, _i64, _d, _D]
        L.orc_smw_matrix.argtypes = [_D, _i64, _i64, _I32, _i64, _d, _D]
        L.orc_cholesky.restype = C.c_int
        L.orc_cholesky.argtypes = [_D, _i64]
        L.orc_newton_direction.restype = C.c_int
        L.orc_newton_direction.argtypes = [_D, _i64, _i64, _I32, _i64, _d, _D, _D]
        L.orc_newton_matvec.argtypes = [_D, _i64, _i64, _I32, _i64, _d, _D, _D]
        L.orc_newton_cg.restype = C.c_int
        L.orc_newton_cg.argtypes = [_D, _i64, _i64, _I32, _i64, _d, _D, _d, C.c_int32, _D]
        L.orc_ls_delta.restype = _d
        L.orc_ls_delta.argtypes = [_D, _D, _i64, _d, _d, _d, _d, _d, _d]
        L.orc_model_select.argtypes = [_D, _i64, _D, _i64, _i64, _d, _D, _D, _D]
        L.orc_cv.restype = C.c_int
        L.orc_cv.argtypes = [_D, _i64, _D, _i64, _i64, _I32, C.c_int, _d, _D, C.c_int, _d, _D]
        L.orc_en_solve.restype = C.c_int
        L.orc_en_solve.argtypes = [_D, _i64, _D, _i64, _i64, _d, _d, _D, _d, C.POINTER(Opts),
                                   _D, C.POINTER(Info), _D, C.c_int32, _I32]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _design(AT):
    AT = _f64(AT)
    n, m = AT.shape
    return AT, m, n


def set_threads(k: int) -> None:
    """Host threads for the oracle's independent-sum loops (results do not
    depend on the count)."""
    lib().orc_set_threads(int(k))


def get_threads() -> int:
    return int(lib().orc_get_threads())


# ---- primitives -----------------------------------------------------------

def prox_sp(t, sigma, l1, l2):
    return lib().orc_prox_sp(float(t), sigma, l1, l2)


def prox_pstar(v, sigma, l1, l2):
    return lib().orc_prox_pstar(float(v), sigma, l1, l2)


def pstar(z, l1, l2):
    z = _f64(z)
    return lib().orc_pstar(_dp(z), z.size, l1, l2)


def gemv_t(AT, v):
    AT, m, n = _design(AT)
    v = _f64(v)
    w = np.empty(n)
    lib().orc_gemv_t(_dp(AT), m, m, n, _dp(v), _dp(w))
    return w


def gemv_n(AT, x):
    AT, m, n = _design(AT)
    x = _f64(x)
    out = np.empty(m)
    lib().orc_gemv_n(_dp(AT), m, m, n, _dp(x), _dp(out))
    return out


def primal_obj(AT, b, x, l1, l2):
    AT, m, n = _design(AT)
    b, x = _f64(b), _f64(x)
    return lib().orc_primal_obj(_dp(AT), m, _dp(b), m, n, _dp(x), l1, l2)


def dual_obj(AT, b, y, l1, l2):
    AT, m, n = _design(AT)
    b, y = _f64(b), _f64(y)
    return lib().orc_dual_obj(_dp(AT), m, _dp(b), m, n, _dp(y), l1, l2)


def eta(AT, b, x, l1, l2):
    AT, m, n = _design(AT)
    b, x = _f64(b), _f64(x)
    return lib().orc_eta(_dp(AT), m, _dp(b), m, n, _dp(x), l1, l2)


def psi(AT, b, x, y, sigma, l1, l2):
    AT, m, n = _design(AT)
    b, x, y = _f64(b), _f64(x), _f64(y)
    return lib().orc_psi(_dp(AT), m, _dp(b), m, n, _dp(x), _dp(y), sigma, l1, l2)


def grad_psi(AT, b, x, y, sigma, l1, l2):
    AT, m, n = _design(AT)
    b, x, y = _f64(b), _f64(x), _f64(y)
    g = np.empty(m)
    lib().orc_grad_psi(_dp(AT), m, _dp(b), m, n, _dp(x), _dp(y), sigma, l1, l2, _dp(g))
    return g


def active_prox(x, w, sigma, l1, l2):
    """Returns (J int32, uJ float64) at t = fma(-sigma, w, x)."""
    x, w = _f64(x), _f64(w)
    n = x.size
    J = np.empty(n, dtype=np.int32)
    uJ = np.empty(n)
    r = lib().orc_active_prox(_dp(x), _dp(w), n, sigma, l1, l2, J.ctypes.data_as(_I32), _dp(uJ))
    return J[:r].copy(), uJ[:r].copy()


def newton_matrix(AT, J, kappa):
    AT, m, n = _design(AT)
    J = np.ascontiguousarray(J, dtype=np.int32)
    V = np.empty((m, m))
    lib().orc_newton_matrix(_dp(AT), m, m, J.ctypes.data_as(_I32), J.size, kappa, _dp(V))
    return V


def smw_matrix(AT, J, kappa):
    AT, m, n = _design(AT)
    J = np.ascontiguousarray(J, dtype=np.int32)
    W = np.empty((J.size, J.size))
    lib().orc_smw_matrix(_dp(AT), m, m, J.ctypes.data_as(_I32), J.size, kappa, _dp(W))
    return W


def cholesky(V):
    L = np.array(V, dtype=np.float64, order="C", copy=True)
    rc = lib().orc_cholesky(_dp(L), L.shape[0])
    if rc != 0:
        raise np.linalg.LinAlgError(f"not positive definite at pivot {-rc - 1}")
    return L


def newton_direction(AT, J, kappa, g):
    AT, m, n = _design(AT)
    J = np.ascontiguousarray(J, dtype=np.int32)
    g = _f64(g)
    d = np.empty(m)
    rc = lib().orc_newton_direction(_dp(AT), m, m, J.ctypes.data_as(_I32), J.size, kappa, _dp(g),
                                    _dp(d))
    if rc != 0:
        raise np.linalg.LinAlgError("Newton matrix not positive definite")
    return d


def newton_matvec(AT, J, kappa, p):
    """V p with V = I + kappa A_J A_J^T, never formed (eq. AJ_system)."""
    AT, m, n = _design(AT)
    J = np.ascontiguousarray(J, dtype=np.int32)
    p = _f64(p)
    q = np.empty(m)
    lib().orc_newton_matvec(_dp(AT), m, m, J.ctypes.data_as(_I32), J.size, kappa, _dp(p), _dp(q))
    return q


def newton_cg(AT, J, kappa, g, eps, maxit=500):
    """Conjugate gradients on V d = -g from d = 0 (the approximate solve of
    eq. newton_direction).  Returns (d, iterations)."""
    AT, m, n = _design(AT)
    J = np.ascontiguousarray(J, dtype=np.int32)
    g = _f64(g)
    d = np.empty(m)
    it = lib().orc_newton_cg(_dp(AT), m, m, J.ctypes.data_as(_I32), J.size, kappa, _dp(g), eps,
                             int(maxit), _dp(d))
    return d, it


def ls_delta(t, wd, s, sigma, l1, l2, gd, dd):
    t, wd = _f64(t), _f64(wd)
    return lib().orc_ls_delta(_dp(t), _dp(wd), t.size, s, sigma, l1, l2, gd, dd)


def en_solve(AT, b, l1, l2, tol=1e-10, x0=None, trace_cap=4096, **opts):
    """Whole SsNAL-EN solve.  Returns (x, info dict, trace array)."""
    AT, m, n = _design(AT)
    b = _f64(b)
    o = Opts(**{k: v for k, v in opts.items()})
    x = np.empty(n)
    info = Info()
    trace = np.zeros((trace_cap, 6))
    rows = C.c_int32(0)
    x0p = None
    if x0 is not None:
        x0a = _f64(x0)
        x0p = _dp(x0a)
    rc = lib().orc_en_solve(_dp(AT), m, _dp(b), m, n, float(l1), float(l2), x0p, float(tol),
                            C.byref(o), _dp(x), C.byref(info), _dp(trace), trace_cap,
                            C.byref(rows))
    if rc < 0:
        raise ValueError("invalid arguments to the oracle solve")
    return x, info.as_dict(), trace[: rows.value].copy()


def model_select(AT, b, x, l2, want_beta=False):
    """gcv / e-bic at a solution x (Sec. "Parameter tuning", eq. gcv_bic): a
    dict with r, nu (EN degrees of freedom), rss_en, rss (after least squares
    on the selected features), gcv, ebic, status (0 ok, 1 r >= m, 2 A_J^T A_J
    singular) and, on request, the de-biased coefficients."""
    AT, m, n = _design(AT)
    b, x = _f64(b), _f64(x)
    out = np.empty(7)
    beta = np.empty(n) if want_beta else None
    lib().orc_model_select(_dp(AT), m, _dp(b), m, n, l2, _dp(x), _dp(out),
                           _dp(beta) if want_beta else C.cast(None, _D))
    res = dict(r=int(out[0]), nu=out[1], rss_en=out[2], rss=out[3], gcv=out[4], ebic=out[5],
               status=int(out[6]))
    if want_beta:
        res["beta"] = beta
    return res


def cv(AT, b, fold, k, alpha, c_lambda, tol=1e-10):
    """k-fold cross validation on the full data's grid lam_q = c_lambda[q] *
    ||A^T b||_inf / alpha: (err (k, nlam) mean squared validation errors, status)."""
    AT, m, n = _design(AT)
    b = _f64(b)
    fold = np.ascontiguousarray(fold, dtype=np.int32)
    c = _f64(c_lambda)
    err = np.empty((k, c.size))
    rc = lib().orc_cv(_dp(AT), m, _dp(b), m, n, fold.ctypes.data_as(_I32), int(k), float(alpha),
                      _dp(c), int(c.size), float(tol), _dp(err))
    return err, rc
