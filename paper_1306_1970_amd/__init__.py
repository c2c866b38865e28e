"""Python binding of the MI355X fused-lasso MM solver (``libflr.so``).

Argument marshalling only: every step of the solve runs in the HIP kernels
behind the C ABI declared in ``include/flr.h``; the functions here carry
the same names.  Arrays may be numpy arrays (host) or torch tensors (host
or device; a device tensor is passed by its data pointer and used where it
lives).  There is no CPU fallback: if the library is missing or no GPU is
visible, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflr.so")

FLR_OK, FLR_ERR_INVALID_ARG, FLR_ERR_OUT_OF_MEMORY, FLR_ERR_DEVICE = 0, 1, 2, 3
FLR_ERR_NUMERICAL, FLR_ERR_MAX_ITER, FLR_ERR_BUSY, FLR_ERR_NOT_READY = 4, 5, 6, 7
FLR_F64, FLR_F32, FLR_BF16 = 0, 1, 2
FLR_PREC_FP64, FLR_PREC_MIXED_FP32 = 0, 1
FLR_PRECOND_AUTO, FLR_PRECOND_TRIDIAG, FLR_PRECOND_JACOBI, FLR_PRECOND_BAND = 0, 1, 2, 3
FLR_METHOD_PCG, FLR_METHOD_CHOLESKY = 0, 1

# every symbol include/flr.h declares
EXPORTS = [
    "flr_default_opts", "flr_ctx_create", "flr_ctx_destroy", "flr_create", "flr_destroy", "flr_solve",
    "flr_solve_ex", "flr_solve_grid", "flr_problem_footprint", "flr_problem_n", "flr_problem_p", "flr_problem_m",
    "flr_server_create", "flr_server_submit", "flr_server_poll", "flr_server_stats", "flr_server_destroy",
    "flr_profile_kernels", "flr_profile_grid", "flr_profile_dense", "flr_status_string", "flr_last_error", "flr_solve_batch",
    "flr_solve_grid_static", "flr_solve_path", "flr_create_flsa", "flr_problem_is_flsa",
]


class FlrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (status_name(status), msg))
        self.status = status


class flr_solve_opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("inner_tol", C.c_double), ("max_iter", C.c_int32), ("max_cg", C.c_int32),
                ("precision", C.c_int32), ("preconditioner", C.c_int32), ("warm_start", C.c_void_p),
                ("use_last", C.c_int32), ("method", C.c_int32)]


class flr_result(C.Structure):
    _fields_ = [("objective", C.c_double), ("rel_change", C.c_double), ("rel_residual", C.c_double),
                ("seconds", C.c_double), ("cg_iters", C.c_int64), ("mm_iters", C.c_int32), ("status", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libflr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError("libflr.so is not built: run __graft_entry__.build() or "
                                    "python paper_1306_1970_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.flr_default_opts.argtypes = [C.POINTER(flr_solve_opts)]
        L.flr_ctx_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
        L.flr_ctx_destroy.argtypes = [vp]
        L.flr_create.argtypes = [vp, vp, C.c_int, i64, i64, i64, vp, vp, i64, C.POINTER(vp)]
        L.flr_destroy.argtypes = [vp]
        L.flr_create_flsa.argtypes = [vp, vp, i64, vp, i64, C.POINTER(vp)]
        L.flr_problem_is_flsa.argtypes = [vp]
        L.flr_problem_is_flsa.restype = i32
        L.flr_solve.argtypes = [vp, d, d, d, vp, C.POINTER(d), C.POINTER(i32)]
        L.flr_solve_ex.argtypes = [vp, d, d, d, C.POINTER(flr_solve_opts), vp, C.POINTER(flr_result)]
        L.flr_solve_grid.argtypes = [vp, vp, vp, i32, d, C.POINTER(flr_solve_opts), vp, vp]
        L.flr_solve_grid_static.argtypes = [vp, vp, vp, i32, d, C.POINTER(flr_solve_opts), vp, vp]
        L.flr_solve_path.argtypes = [vp, vp, vp, vp, i32, d, C.POINTER(flr_solve_opts), vp, vp]
        L.flr_problem_footprint.argtypes = [vp, C.POINTER(C.c_size_t)]
        for f in ("flr_problem_n", "flr_problem_p", "flr_problem_m"):
            getattr(L, f).argtypes = [vp]
            getattr(L, f).restype = i64
        L.flr_server_create.argtypes = [vp, C.c_size_t, i32, C.POINTER(vp)]
        L.flr_server_submit.argtypes = [vp, vp, d, d, d, C.POINTER(flr_solve_opts), C.POINTER(C.c_uint64)]
        L.flr_server_poll.argtypes = [vp, C.c_uint64, C.c_int, vp, C.POINTER(flr_result)]
        L.flr_server_stats.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_size_t)]
        L.flr_server_destroy.argtypes = [vp]
        L.flr_profile_kernels.argtypes = [vp, i32, vp]
        L.flr_profile_grid.argtypes = [vp, i32, i32, vp]
        L.flr_profile_dense.argtypes = [vp, d, d, i32, vp]
        L.flr_solve_batch.argtypes = [vp, i32, vp, vp, d, C.POINTER(flr_solve_opts), vp, vp]
        L.flr_status_string.argtypes = [C.c_int]
        L.flr_status_string.restype = C.c_char_p
        L.flr_last_error.restype = C.c_char_p
        for name in EXPORTS:
            f = getattr(L, name)
            if f.restype is C.c_int and name not in ("flr_status_string",):
                f.restype = C.c_int
        _lib = L
    return _lib


def status_name(st: int) -> str:
    try:
        return lib().flr_status_string(int(st)).decode()
    except Exception:  # pragma: no cover
        return "status %d" % st


def last_error() -> str:
    return lib().flr_last_error().decode()


def _check(st, ok=(FLR_OK,)):
    if st not in ok:
        raise FlrError(st, last_error())
    return st


def _ptr(a):
    """Data pointer of a numpy array or torch tensor (None passes through)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def default_opts(**kw) -> flr_solve_opts:
    o = flr_solve_opts()
    lib().flr_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "warm_start":
            o.warm_start = _ptr(v)
        else:
            setattr(o, k, v)
    return o


# ---------------------------------------------------------------------------
# C ABI, same names
# ---------------------------------------------------------------------------
def flr_ctx_create(device: int = 0, hip_stream: int | None = None):
    out = C.c_void_p()
    _check(lib().flr_ctx_create(device, hip_stream, C.byref(out)))
    return out


def flr_ctx_destroy(ctx):
    lib().flr_ctx_destroy(ctx)


def flr_create(ctx, X, x_dtype: int, n: int, p: int, ldx: int, y, edges, m: int):
    out = C.c_void_p()
    _check(lib().flr_create(ctx, _ptr(X), x_dtype, n, p, ldx, _ptr(y), _ptr(edges) if m else None, m,
                            C.byref(out)))
    return out


def flr_destroy(h):
    lib().flr_destroy(h)


def flr_create_flsa(ctx, y, p: int, edges, m: int):
    out = C.c_void_p()
    _check(lib().flr_create_flsa(ctx, _ptr(y), p, _ptr(edges) if m else None, m, C.byref(out)))
    return out


def flr_problem_is_flsa(h) -> int:
    return int(lib().flr_problem_is_flsa(h))


def flr_solve(h, lambda1, lambda2, tol, beta_out):
    f = C.c_double()
    it = C.c_int32()
    st = lib().flr_solve(h, lambda1, lambda2, tol, _ptr(beta_out), C.byref(f), C.byref(it))
    _check(st, ok=(FLR_OK, FLR_ERR_MAX_ITER, FLR_ERR_NUMERICAL))
    return st, f.value, it.value


def flr_solve_ex(h, lambda1, lambda2, tol, opts, beta_out):
    res = flr_result()
    st = lib().flr_solve_ex(h, lambda1, lambda2, tol, C.byref(opts) if opts is not None else None, _ptr(beta_out),
                            C.byref(res))
    _check(st, ok=(FLR_OK, FLR_ERR_MAX_ITER, FLR_ERR_NUMERICAL))
    return st, res


def flr_solve_grid(h, lambda1, lambda2, tol, opts, beta_out):
    l1 = np.ascontiguousarray(lambda1, dtype=np.float64)
    l2 = np.ascontiguousarray(lambda2, dtype=np.float64)
    B = int(l1.size)
    res = (flr_result * B)()
    st = lib().flr_solve_grid(h, l1.ctypes.data, l2.ctypes.data, B, tol, C.byref(opts) if opts is not None else None,
                              _ptr(beta_out), C.cast(res, C.c_void_p))
    _check(st, ok=(FLR_OK, FLR_ERR_MAX_ITER, FLR_ERR_NUMERICAL))
    return st, list(res)


def flr_solve_grid_static(h, lambda1, lambda2, tol, opts, beta_out):
    """flr_solve_grid with its workspace in the library's static device array (no allocation)."""
    l1 = np.ascontiguousarray(lambda1, dtype=np.float64)
    l2 = np.ascontiguousarray(lambda2, dtype=np.float64)
    B = int(l1.size)
    res = (flr_result * B)()
    st = lib().flr_solve_grid_static(h, l1.ctypes.data, l2.ctypes.data, B, tol,
                                     C.byref(opts) if opts is not None else None, _ptr(beta_out),
                                     C.cast(res, C.c_void_p))
    _check(st, ok=(FLR_OK, FLR_ERR_MAX_ITER, FLR_ERR_NUMERICAL))
    return st, list(res)


def flr_solve_path(h, lambda1, lambda2, eps, tol, opts, beta_out):
    """Warm-started sequence of solves (regularization path and/or eps-continuation)."""
    l1 = np.ascontiguousarray(lambda1, dtype=np.float64)
    l2 = np.ascontiguousarray(lambda2, dtype=np.float64)
    e = None if eps is None else np.ascontiguousarray(eps, dtype=np.float64)
    k = int(l1.size)
    res = (flr_result * k)()
    st = lib().flr_solve_path(h, l1.ctypes.data, l2.ctypes.data, None if e is None else e.ctypes.data, k, tol,
                              C.byref(opts) if opts is not None else None, _ptr(beta_out), C.cast(res, C.c_void_p))
    _check(st, ok=(FLR_OK, FLR_ERR_MAX_ITER, FLR_ERR_NUMERICAL))
    return st, list(res)


def flr_problem_footprint(h) -> int:
    b = C.c_size_t()
    _check(lib().flr_problem_footprint(h, C.byref(b)))
    return int(b.value)


def flr_server_create(ctx, hbm_budget_bytes: int, max_slots: int):
    out = C.c_void_p()
    _check(lib().flr_server_create(ctx, hbm_budget_bytes, max_slots, C.byref(out)))
    return out


def flr_server_submit(s, h, lambda1, lambda2, tol, opts=None) -> int:
    t = C.c_uint64()
    _check(lib().flr_server_submit(s, h, lambda1, lambda2, tol, C.byref(opts) if opts is not None else None,
                                   C.byref(t)))
    return int(t.value)


def flr_server_poll(s, ticket: int, blocking: bool, beta_out=None):
    res = flr_result()
    st = lib().flr_server_poll(s, ticket, 1 if blocking else 0, _ptr(beta_out), C.byref(res))
    _check(st, ok=(FLR_OK, FLR_ERR_MAX_ITER, FLR_ERR_NUMERICAL, FLR_ERR_NOT_READY))
    return st, res


def flr_server_stats(s):
    q, r, b = C.c_int32(), C.c_int32(), C.c_size_t()
    _check(lib().flr_server_stats(s, C.byref(q), C.byref(r), C.byref(b)))
    return q.value, r.value, int(b.value)


def flr_server_destroy(s):
    lib().flr_server_destroy(s)


def flr_profile_kernels(h, reps: int):
    """Average durations (us) of the X v, X^T u and block kernels (HIP events on the problem's stream)."""
    out = np.zeros(3)
    _check(lib().flr_profile_kernels(h, reps, out.ctypes.data))
    return float(out[0]), float(out[1]), float(out[2])


def flr_solve_batch(problems, lambda1, lambda2, tol, opts=None, betas=None):
    """Ragged batch: one call solves every (problem, lambda1, lambda2); betas: list of arrays (or None)."""
    k = len(problems)
    hs = (C.c_void_p * k)(*[p.h if hasattr(p, "h") else p for p in problems])
    l1 = np.ascontiguousarray(lambda1, dtype=np.float64)
    l2 = np.ascontiguousarray(lambda2, dtype=np.float64)
    res = (flr_result * k)()
    outs = None
    if betas is not None:
        outs = (C.c_void_p * k)(*[_ptr(b) for b in betas])
    o = opts if opts is not None else default_opts()
    st = lib().flr_solve_batch(hs, k, l1.ctypes.data, l2.ctypes.data, tol, C.byref(o),
                               C.cast(outs, C.c_void_p) if outs is not None else None, C.cast(res, C.c_void_p))
    _check(st, ok=(FLR_OK, FLR_ERR_MAX_ITER, FLR_ERR_NUMERICAL))
    return st, list(res)


def flr_profile_dense(h, lam1: float, lam2: float, reps: int):
    """Average durations (us) of one Algorithm 1 step's assembly, Cholesky factor and triangular solves."""
    out = np.zeros(3)
    _check(lib().flr_profile_dense(h, lam1, lam2, reps, out.ctypes.data))
    return float(out[0]), float(out[1]), float(out[2])


def flr_profile_grid(h, B: int, reps: int):
    """Average durations (us) of the two batched GEMMs (X O and X^T U) for B columns."""
    out = np.zeros(2)
    _check(lib().flr_profile_grid(h, B, reps, out.ctypes.data))
    return float(out[0]), float(out[1])


# ---------------------------------------------------------------------------
# small object wrappers
# ---------------------------------------------------------------------------
_DT = {FLR_F64: np.float64, FLR_F32: np.float32, FLR_BF16: np.uint16}


class Context:
    def __init__(self, device: int = 0):
        self.h = flr_ctx_create(device)

    def close(self):
        if self.h:
            flr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Solution:
    beta: np.ndarray
    status: int
    objective: float
    mm_iters: int
    cg_iters: int
    rel_change: float
    rel_residual: float
    seconds: float


class Problem:
    """A resident FLR problem: X (numpy array in its stored dtype, or a
    device tensor), y (float64), edges (int64 pairs)."""

    def __init__(self, ctx: Context, X, x_dtype: int, y, edges, use_tuned: bool = True):
        self.ctx = ctx
        if hasattr(X, "data_ptr"):
            n, p = int(X.shape[0]), int(X.shape[1])
            ldx = int(X.stride(0))
            self._X = X
        else:
            X = np.ascontiguousarray(X, dtype=_DT[x_dtype])
            n, p = X.shape
            ldx = p
            self._X = X
        yv = np.ascontiguousarray(y, dtype=np.float64)
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).reshape(-1, 2))
        self.n, self.p, self.m_in = n, p, e.shape[0]
        from . import autotune

        tuned = autotune.lookup(n, p, x_dtype) if use_tuned else None
        with autotune.launch_shape(tuned["target_wg_a"] if tuned else None, tuned["target_wg_b"] if tuned else None):
            self.h = flr_create(ctx.h, self._X, x_dtype, n, p, ldx, yv, e, e.shape[0])
        self._X = None  # the library holds its own copy

    @classmethod
    def from_instance(cls, ctx, inst):
        return cls(ctx, inst.X, inst.dtype, inst.y, inst.edges)

    @classmethod
    def flsa(cls, ctx, y, edges):
        """A fused lasso signal approximation problem (X = I): flr_create_flsa."""
        self = cls.__new__(cls)
        self.ctx = ctx
        yv = np.ascontiguousarray(y, dtype=np.float64)
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).reshape(-1, 2))
        self.n = self.p = int(yv.size)
        self.m_in = e.shape[0]
        self._X = None
        self.h = flr_create_flsa(ctx.h, yv, self.p, e, e.shape[0])
        return self

    @property
    def footprint(self) -> int:
        return flr_problem_footprint(self.h)

    def solve(self, lam1, lam2, tol=1e-8, out=None, **opts) -> Solution:
        o = default_opts(**opts)
        beta = np.zeros(self.p) if out is None else out
        st, r = flr_solve_ex(self.h, lam1, lam2, tol, o, beta)
        b = beta if isinstance(beta, np.ndarray) else beta
        return Solution(b, st, r.objective, r.mm_iters, r.cg_iters, r.rel_change, r.rel_residual, r.seconds)

    def solve_grid(self, lam1, lam2, tol=1e-8, static=False, **opts):
        """Batched grid solve; static=True uses flr_solve_grid_static (no allocation)."""
        o = default_opts(**opts)
        B = len(lam1)
        beta = np.zeros((B, self.p))
        fn = flr_solve_grid_static if static else flr_solve_grid
        st, res = fn(self.h, lam1, lam2, tol, o, beta)
        return st, beta, [r.as_dict() for r in res]

    def solve_path(self, lam1, lam2, tol=1e-8, eps=None, **opts):
        """Solves along (lam1[k], lam2[k], eps[k]), each warm-started at the previous solution."""
        o = default_opts(**opts)
        beta = np.zeros((len(lam1), self.p))
        st, res = flr_solve_path(self.h, lam1, lam2, eps, tol, o, beta)
        return st, beta, [r.as_dict() for r in res]

    def close(self):
        if self.h:
            flr_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
