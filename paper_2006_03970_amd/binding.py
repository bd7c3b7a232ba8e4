"""ctypes binding of libssnal_en.so (declared in include/ssnal_en.h).

Argument marshalling only: every step of a solve runs in the HIP library.
Device arrays are torch tensors on a ROCm device; the design A is a tensor of
shape (n, lda) (row j = column j of the column-major m x n design, entries
lda > m ignored), dtype float64, float32 or bfloat16.  The library is loaded
from this package directory and its absence is an error: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libssnal_en.so")

SSNAL_F64, SSNAL_F32, SSNAL_BF16 = 0, 1, 2
STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "LINESEARCH_STALL", 3: "PATH_TRUNCATED", -1: "EINVAL",
          -2: "ENONFINITE", -3: "ENOMEM", -4: "EHIP", -5: "ENUMERIC"}


class SsnalError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)} ({code}): {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("sigma0", C.c_double), ("sigma_factor", C.c_double), ("sigma_max", C.c_double),
                ("mu", C.c_double), ("delta", C.c_double), ("max_outer", C.c_int32),
                ("max_inner", C.c_int32), ("max_backtrack", C.c_int32), ("no_refine", C.c_int32),
                ("no_smw", C.c_int32), ("timing", C.c_int32), ("trace_cap", C.c_int32),
                ("trace", C.POINTER(C.c_double)), ("newton_cg", C.c_int32), ("cg_maxit", C.c_int32),
                ("cg_eta", C.c_double), ("cg_tau", C.c_double), ("workers", C.c_int32),
                ("no_small", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_iters", C.c_int32), ("newton_iters", C.c_int32),
                ("r_final", C.c_int32), ("nnz", C.c_int64), ("kkt_rel", C.c_double),
                ("kkt1", C.c_double), ("kkt3", C.c_double), ("primal_obj", C.c_double),
                ("dual_obj", C.c_double), ("rel_gap", C.c_double), ("sigma_final", C.c_double),
                ("gemv_calls", C.c_int32), ("syncs", C.c_int32), ("gemv_ms", C.c_double),
                ("solve_ms", C.c_double), ("atd_launches", C.c_int32), ("atd_ms", C.c_double),
                ("cg_iters", C.c_int32), ("sigma0", C.c_double), ("queue_ms", C.c_double),
                ("upload_ms", C.c_double), ("chol_calls", C.c_int32), ("chol_ms", C.c_double),
                ("chol_gflop", C.c_double), ("one_workgroup", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Problem(C.Structure):
    _fields_ = [("A", C.c_void_p), ("a_dtype", C.c_int), ("lda", C.c_int64), ("m", C.c_int64),
                ("n", C.c_int64), ("b", C.c_void_p), ("lambda1", C.c_double), ("lambda2", C.c_double),
                ("x0", C.c_void_p), ("tol", C.c_double), ("x_out", C.c_void_p),
                ("sigma0", C.c_double), ("location", C.c_int32), ("ready", C.c_void_p)]


SSNAL_ON_DEVICE, SSNAL_ON_HOST = 0, 1


_lib = None
_vp = C.c_void_p
_i64 = C.c_int64
_d = C.c_double
_i = C.c_int


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m "
                               "paper_2006_03970_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        L.ssnal_last_error.restype = C.c_char_p
        L.ssnal_en_opts_init.argtypes = [C.POINTER(Opts)]
        L.ssnal_ctx_create.argtypes = [_i, C.POINTER(_vp)]
        L.ssnal_ctx_destroy.argtypes = [_vp]
        L.ssnal_en_solve.argtypes = [_vp, _vp, _i, _i64, _vp, _i64, _i64, _d, _d, _vp, _d, _vp, _vp,
                                     C.POINTER(Opts), C.POINTER(Info)]
        L.ssnal_en_solve_noalloc.argtypes = L.ssnal_en_solve.argtypes
        L.ssnal_gemv_t.argtypes = [_vp, _vp, _i, _i64, _i64, _i64, _vp, _vp, _i, _vp]
        L.ssnal_active_prox.argtypes = [_vp, _vp, _vp, _i64, _d, _d, _d, _vp, _vp,
                                        C.POINTER(_i64), _vp]
        L.ssnal_newton_matrix.argtypes = [_vp, _vp, _i, _i64, _i64, _vp, _i64, _d, _i, _vp, _vp]
        L.ssnal_cholesky.argtypes = [_vp, _vp, _i64, _vp]
        L.ssnal_newton_direction.argtypes = [_vp, _vp, _i, _i64, _i64, _vp, _i64, _d, _vp, _vp, _i,
                                             _vp]
        L.ssnal_newton_cg.argtypes = [_vp, _vp, _i, _i64, _i64, _vp, _i64, _d, _vp, _d, C.c_int32, _vp,
                                      _vp, C.POINTER(C.c_int32)]
        L.ssnal_ls_delta.argtypes = [_vp, _vp, _vp, _vp, _i64, _d, _d, _d, _d, _d, _i,
                                     C.POINTER(_d), C.POINTER(_d), _vp]
        L.ssnal_kkt.argtypes = [_vp, _vp, _i, _i64, _vp, _i64, _i64, _vp, _d, _d, C.POINTER(_d), _vp]
        L.ssnal_en_model_select.argtypes = [_vp, _vp, _i, _i64, _vp, _i64, _i64, _d, _vp, _vp, _vp,
                                            C.POINTER(Select)]
        L.ssnal_en_cv.argtypes = [_vp, _vp, _i, _i64, _vp, _i64, _i64, _vp, _i, _d, C.POINTER(_d), _i,
                                  _d, _i, _vp, C.POINTER(Opts), C.POINTER(_d), C.POINTER(Info)]
        L.ssnal_en_path.argtypes = [_vp, _vp, _i, _i64, _vp, _i64, _i64, _d, C.POINTER(_d), _i, _i64,
                                    _d, _vp, _vp, C.POINTER(Opts), C.POINTER(Info)]
        L.ssnal_en_solve_batch.argtypes = [_vp, C.POINTER(Problem), _i, C.POINTER(Opts), _vp,
                                           C.POINTER(Info)]
        L.ssnal_srv_create.argtypes = [_i, C.c_size_t, _i, C.POINTER(Opts), C.POINTER(_vp)]
        L.ssnal_srv_submit.argtypes = [_vp, C.POINTER(Problem), C.POINTER(C.c_uint64)]
        L.ssnal_srv_poll.argtypes = [_vp, C.c_uint64, C.POINTER(Info)]
        L.ssnal_srv_wait.argtypes = [_vp, C.c_uint64, C.POINTER(Info)]
        L.ssnal_srv_destroy.argtypes = [_vp]
        L.ssnal_workspace_bytes.argtypes = [_i64, _i64]
        L.ssnal_workspace_bytes.restype = C.c_size_t
        L.ssnal_srv_footprint.argtypes = [C.POINTER(Problem)]
        L.ssnal_srv_footprint.restype = C.c_size_t
        for name in ("ssnal_en_path", "ssnal_en_solve_batch", "ssnal_srv_create", "ssnal_srv_submit",
                     "ssnal_srv_poll", "ssnal_srv_wait"):
            getattr(L, name).restype = _i
        for name in ("ssnal_ctx_create", "ssnal_en_solve", "ssnal_en_solve_noalloc", "ssnal_gemv_t", "ssnal_active_prox",
                     "ssnal_newton_matrix", "ssnal_cholesky", "ssnal_newton_direction",
                     "ssnal_newton_cg", "ssnal_ls_delta", "ssnal_kkt"):
            getattr(L, name).restype = _i
        _lib = L
    return _lib


def last_error() -> str:
    return lib().ssnal_last_error().decode()


def _check(rc, allow_warn=False):
    if rc < 0 or (rc > 0 and not allow_warn):
        raise SsnalError(rc, last_error())
    return rc


def _ptr(t):
    return None if t is None else _vp(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


_DTYPES = {}


def _dtype_code(A):
    if not _DTYPES:
        import torch
        _DTYPES.update({torch.float64: SSNAL_F64, torch.float32: SSNAL_F32, torch.bfloat16: SSNAL_BF16})
    return _DTYPES[A.dtype]


def _design(A, m):
    """(pointer, dtype code, lda, m, n) of a (n, lda) design tensor."""
    assert A.dim() == 2 and (A.stride(1) == 1 or A.shape[1] == 1), \
        "A must be (n, lda) with unit inner stride"
    n = A.shape[0]
    lda = A.stride(0) if n > 1 else A.shape[1]
    if A.shape[1] == 1:
        lda = 1
        assert n == 1 or A.stride(0) == 1, "A must be (n, lda) with lda = 1 here"
    m = lda if m is None else m
    return _ptr(A), _dtype_code(A), lda, m, n


class Context:
    """Owns one ssnal_ctx (device workspace) on a device."""

    def __init__(self, device: int = 0):
        p = _vp()
        _check(lib().ssnal_ctx_create(device, C.byref(p)))
        self.ptr = p
        self.device = device

    def close(self):
        if getattr(self, "ptr", None):
            lib().ssnal_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def make_opts(**kw) -> Opts:
    o = Opts()
    lib().ssnal_en_opts_init(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# ---------------------------------------------------------------- entry points

def ssnal_en_solve(ctx, A, b, lambda1, lambda2, x0=None, tol=1e-6, x_out=None, m=None, opts=None,
                   stream=None, trace_cap=0):
    """One solve.  Returns (x_out, info dict[, trace rows]).  Warnings
    (NOT_CONVERGED, LINESEARCH_STALL) are reported in info['status']."""
    import torch
    pA, dt, lda, m, n = _design(A, m)
    if x_out is None:
        x_out = torch.empty(n, dtype=torch.float64, device=A.device)
    o = opts if opts is not None else make_opts()
    trace = None
    if trace_cap:
        trace = (C.c_double * (6 * trace_cap))()
        o.trace = C.cast(trace, C.POINTER(C.c_double))
        o.trace_cap = trace_cap
    info = Info()
    rc = lib().ssnal_en_solve(ctx.ptr, pA, dt, lda, _ptr(b), m, n, float(lambda1), float(lambda2),
                              _ptr(x0), float(tol), _stream(stream), _ptr(x_out), C.byref(o),
                              C.byref(info))
    _check(rc, allow_warn=True)
    d = info.as_dict()
    if trace_cap:
        import numpy as np
        rows = d["newton_iters"] + (0 if d["status"] == 0 else 1)
        tr = np.ctypeslib.as_array(trace)[: 6 * trace_cap].reshape(trace_cap, 6)
        nz = int(np.count_nonzero(tr[:, 3]))
        return x_out, d, tr[:nz].copy()
    return x_out, d


def ssnal_en_solve_noalloc(ctx, A, b, lambda1, lambda2, x_out, x0=None, tol=1e-6, m=None, opts=None,
                           stream=None):
    """ssnal_en_solve with the workspace in the library's static device array
    (no allocation in the call; m <= 512, n <= 131072).  x_out is required.
    Returns the info dict."""
    pA, dt, lda, m, n = _design(A, m)
    o = opts if opts is not None else make_opts()
    info = Info()
    rc = lib().ssnal_en_solve_noalloc(ctx.ptr, pA, dt, lda, _ptr(b), m, n, float(lambda1), float(lambda2),
                                      _ptr(x0), float(tol), _stream(stream), _ptr(x_out), C.byref(o),
                                      C.byref(info))
    _check(rc, allow_warn=True)
    return info.as_dict()


def ssnal_gemv_t(ctx, A, v, w=None, acc64=False, m=None, stream=None):
    import torch
    pA, dt, lda, m, n = _design(A, m)
    if w is None:
        w = torch.empty(n, dtype=torch.float64, device=A.device)
    _check(lib().ssnal_gemv_t(ctx.ptr, pA, dt, lda, m, n, _ptr(v), _ptr(w), int(bool(acc64)),
                              _stream(stream)))
    return w


def ssnal_active_prox(ctx, x, w, sigma, lambda1, lambda2, stream=None):
    import torch
    n = x.numel()
    J = torch.empty(n, dtype=torch.int32, device=x.device)
    uJ = torch.empty(n, dtype=torch.float64, device=x.device)
    r = _i64(0)
    _check(lib().ssnal_active_prox(ctx.ptr, _ptr(x), _ptr(w), n, float(sigma), float(lambda1),
                                   float(lambda2), _ptr(J), _ptr(uJ), C.byref(r), _stream(stream)))
    return J[: r.value], uJ[: r.value]


def ssnal_newton_matrix(ctx, A, J, kappa, form, m=None, stream=None):
    import torch
    pA, dt, lda, m, n = _design(A, m)
    r = J.numel()
    N = m if form == 0 else r
    out = torch.empty((N, N), dtype=torch.float64, device=A.device)
    _check(lib().ssnal_newton_matrix(ctx.ptr, pA, dt, lda, m, _ptr(J), r, float(kappa), int(form),
                                     _ptr(out), _stream(stream)))
    return out


def ssnal_cholesky(ctx, V, stream=None):
    """In place: V (N x N, FP64, contiguous) becomes L (lower, upper zeroed)."""
    _check(lib().ssnal_cholesky(ctx.ptr, _ptr(V), V.shape[0], _stream(stream)))
    return V


def ssnal_newton_direction(ctx, A, J, kappa, g, form=-1, m=None, stream=None):
    import torch
    pA, dt, lda, m, n = _design(A, m)
    d = torch.empty(m, dtype=torch.float64, device=A.device)
    _check(lib().ssnal_newton_direction(ctx.ptr, pA, dt, lda, m, _ptr(J), J.numel(), float(kappa),
                                        _ptr(g), _ptr(d), int(form), _stream(stream)))
    return d


def ssnal_newton_cg(ctx, A, J, kappa, g, eps, maxit=500, m=None, stream=None):
    """Conjugate-gradient Newton direction.  Returns (d, iterations)."""
    import torch
    pA, dt, lda, m, n = _design(A, m)
    d = torch.empty(m, dtype=torch.float64, device=A.device)
    it = C.c_int32(0)
    _check(lib().ssnal_newton_cg(ctx.ptr, pA, dt, lda, m, _ptr(J), J.numel(), float(kappa), _ptr(g),
                                 float(eps), int(maxit), _stream(stream), _ptr(d), C.byref(it)))
    return d, it.value


def ssnal_ls_delta(ctx, x, w, wd, sigma, lambda1, lambda2, gd, dd, steps, stream=None):
    K = len(steps)
    s = (C.c_double * K)(*[float(v) for v in steps])
    out = (C.c_double * K)()
    _check(lib().ssnal_ls_delta(ctx.ptr, _ptr(x), _ptr(w), _ptr(wd), x.numel(), float(sigma),
                                float(lambda1), float(lambda2), float(gd), float(dd), K, s, out,
                                _stream(stream)))
    return [out[k] for k in range(K)]


def ssnal_kkt(ctx, A, b, x, lambda1, lambda2, m=None, stream=None):
    pA, dt, lda, m, n = _design(A, m)
    out = (C.c_double * 4)()
    _check(lib().ssnal_kkt(ctx.ptr, pA, dt, lda, _ptr(b), m, n, _ptr(x), float(lambda1),
                           float(lambda2), out, _stream(stream)))
    return {"eta": out[0], "primal_obj": out[1], "dual_obj": out[2], "rel_gap": out[3]}


class Select(C.Structure):
    _fields_ = [("status", C.c_int32), ("r", C.c_int32), ("nu", C.c_double), ("rss_en", C.c_double),
                ("rss", C.c_double), ("gcv", C.c_double), ("ebic", C.c_double)]


def ssnal_en_model_select(ctx, A, b, x, lambda2, m=None, want_beta=False, stream=None):
    """gcv / e-bic at a solution x: a dict with status, r, nu, rss_en, rss, gcv,
    ebic and, on request, the de-biased coefficients (device tensor)."""
    import torch
    pA, dt, lda, m, n = _design(A, m)
    beta = torch.empty(n, dtype=torch.float64, device=x.device) if want_beta else None
    s = Select()
    _check(lib().ssnal_en_model_select(ctx.ptr, pA, dt, lda, _ptr(b), m, n, float(lambda2), _ptr(x),
                                       _stream(stream), _ptr(beta) if want_beta else None,
                                       C.byref(s)))
    out = {k: getattr(s, k) for k, _ in Select._fields_}
    if want_beta:
        out["beta"] = beta
    return out


def ssnal_en_cv(ctx, A, b, fold, k, alpha, c_lambda, tol=1e-6, slots=8, m=None, opts=None, stream=None):
    """k-fold cross validation over the full data's grid: (err (k, nlam) mean
    squared validation errors, infos (k, nlam) dicts, status).  fold: device
    int32 tensor of m labels in [0, k); folds run on min(slots, k) concurrent
    workers."""
    import numpy as np
    pA, dt, lda, m, n = _design(A, m)
    nlam = len(c_lambda)
    cl = (C.c_double * nlam)(*[float(v) for v in c_lambda])
    err = (C.c_double * (k * nlam))()
    infos = (Info * (k * nlam))()
    o = opts if opts is not None else make_opts()
    rc = lib().ssnal_en_cv(ctx.ptr, pA, dt, lda, _ptr(b), m, n, _ptr(fold), int(k), float(alpha), cl,
                           nlam, float(tol), int(slots), _stream(stream), C.byref(o), err, infos)
    if rc < 0:
        _check(rc)
    E = np.array(err[:], dtype=np.float64).reshape(k, nlam)
    I = [[infos[f * nlam + q].as_dict() for q in range(nlam)] for f in range(k)]
    return E, I, rc


def workspace_bytes(m, n) -> int:
    """Device bytes a context holds for an (m, n) problem (serving admission footprint)."""
    return int(lib().ssnal_workspace_bytes(int(m), int(n)))


def ssnal_en_path(ctx, A, b, alpha, c_lambda, tol=1e-6, X_out=None, m=None, max_active=0,
                  opts=None, stream=None):
    """Warm-started path over lam_k = c_lambda[k] * lam_max.  Returns (X (n, nlam) with
    column-major storage viewed as X_out[k] = point k, list of info dicts, status)."""
    import torch
    pA, dt, lda, m, n = _design(A, m)
    nlam = len(c_lambda)
    if X_out is None:
        X_out = torch.empty((nlam, n), dtype=torch.float64, device=A.device)
    assert X_out.is_contiguous() and X_out.numel() == nlam * n
    cl = (C.c_double * nlam)(*[float(v) for v in c_lambda])
    infos = (Info * nlam)()
    o = opts if opts is not None else make_opts()
    rc = lib().ssnal_en_path(ctx.ptr, pA, dt, lda, _ptr(b), m, n, float(alpha), cl, nlam,
                             int(max_active), float(tol), _stream(stream), _ptr(X_out), C.byref(o),
                             infos)
    _check(rc, allow_warn=True)
    return X_out, [infos[k].as_dict() for k in range(nlam)], rc


def _problem(A, b, lambda1, lambda2, tol, x_out, x0=None, m=None, sigma0=0.0, ready=None):
    """ssnal_en_problem of tensors that all live on the device, or all in host
    memory (a served host-resident request)."""
    pA, dt, lda, m, n = _design(A, m)
    on_host = not A.is_cuda
    for t in (b, x_out, x0):
        assert t is None or t.is_cuda != on_host, "A, b, x0, x_out: all host or all device"
    return Problem(pA, dt, lda, m, n, _ptr(b), float(lambda1), float(lambda2), _ptr(x0), float(tol),
                   _ptr(x_out), float(sigma0), SSNAL_ON_HOST if on_host else SSNAL_ON_DEVICE,
                   None if ready is None else _vp(ready.cuda_event))


def srv_footprint(A, m=None):
    """Device bytes a served request with this design occupies (admission footprint)."""
    import torch
    pA, dt, lda, m, n = _design(A, m)
    on_host = A.device.type == "cpu"
    p = Problem(pA, dt, lda, m, n, None, 0.0, 0.0, None, 1.0, None, 0.0,
                SSNAL_ON_HOST if on_host else SSNAL_ON_DEVICE, None)
    return int(lib().ssnal_srv_footprint(C.byref(p)))


def batch_args(problems):
    """The ssnal_en_problem array of a batch (problems: list of dicts with A,
    b, lambda1, lambda2, tol, x_out[, x0, sigma0, m (rows when A's leading
    dimension is padded)]); the caller keeps the tensors alive while it is in
    use."""
    arr = (Problem * len(problems))()
    for i, p in enumerate(problems):
        arr[i] = _problem(p["A"], p["b"], p["lambda1"], p["lambda2"], p["tol"], p["x_out"], p.get("x0"),
                          m=p.get("m"), sigma0=p.get("sigma0", 0.0))
    return arr


def solve_batch_args(ctx, arr, opts=None, stream=None, workers=0):
    """ssnal_en_solve_batch over an array from batch_args.  Returns (the
    ctypes Info array, worst status)."""
    cnt = len(arr)
    infos = (Info * cnt)()
    o = opts if opts is not None else make_opts()
    if workers:
        o.workers = int(workers)
    rc = lib().ssnal_en_solve_batch(ctx.ptr, arr, cnt, C.byref(o), _stream(stream), infos)
    _check(rc, allow_warn=True)
    return infos, rc


def ssnal_en_solve_batch(ctx, problems, opts=None, stream=None, workers=0):
    """problems: list of dicts with A, b, lambda1, lambda2, tol, x_out[, x0,
    sigma0, m].  workers: concurrent workers (0 = the library's default of 8, 1 =
    in turn on `stream`).  Returns (list of info dicts, worst status)."""
    infos, rc = solve_batch_args(ctx, batch_args(problems), opts, stream, workers)
    return [infos[i].as_dict() for i in range(len(infos))], rc


class Server:
    """Serving loop (slot table, admission by workspace footprint)."""

    def __init__(self, device=0, hbm_budget=8 << 30, max_slots=4, opts=None):
        p = _vp()
        o = C.byref(opts) if opts is not None else None
        _check(lib().ssnal_srv_create(device, int(hbm_budget), int(max_slots), o, C.byref(p)))
        self.ptr = p
        self._keep = {}

    def submit(self, A, b, lambda1, lambda2, tol, x_out, x0=None, sigma0=0.0, m=None) -> int:
        """Queue a request.  Device tensors: an event recorded on the current
        stream orders the solve after the work that wrote them.  Host tensors
        (pinned for asynchronous uploads): the server uploads A, b and x0 on
        admission and writes x_out back."""
        import torch
        t = C.c_uint64(0)
        ready = None
        if A.device.type != "cpu":
            ready = torch.cuda.Event()
            ready.record(torch.cuda.current_stream(A.device))
        prob = _problem(A, b, lambda1, lambda2, tol, x_out, x0, m=m, sigma0=sigma0, ready=ready)
        _check(lib().ssnal_srv_submit(self.ptr, C.byref(prob), C.byref(t)))
        self._keep[t.value] = (A, b, x_out, x0, ready)  # alive until collected
        return t.value

    def poll(self, ticket):
        info = Info()
        rc = lib().ssnal_srv_poll(self.ptr, ticket, C.byref(info))
        if rc == 1:
            return None
        self._keep.pop(ticket, None)
        _check(rc, allow_warn=True)
        return info.as_dict()

    def wait(self, ticket):
        info = Info()
        rc = lib().ssnal_srv_wait(self.ptr, ticket, C.byref(info))
        self._keep.pop(ticket, None)
        _check(rc, allow_warn=True)
        return info.as_dict()

    def close(self):
        if getattr(self, "ptr", None):
            lib().ssnal_srv_destroy(self.ptr)
            self.ptr = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
