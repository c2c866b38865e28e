"""Python access to the FP64 CPU oracle (``liboracle_flr.so``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product path never imports it.
The oracle is plain C (see ``flr_oracle.c``); this file only marshals
numpy arrays into it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle_flr.so")
_SRC = os.path.join(_HERE, "flr_oracle.c")

F64, F32, BF16 = 0, 1, 2
ALG_AUTO, ALG1, ALG2 = 0, 1, 2
OK, MAX_ITER, NUMERICAL, BAD_ARG = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("p", C.c_int64), ("ldx", C.c_int64), ("xdtype", C.c_int),
                ("X", C.c_void_p), ("y", C.c_void_p), ("m", C.c_int64), ("edges", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("tol", C.c_double), ("inner_tol", C.c_double), ("max_iter", C.c_int32),
                ("max_cg", C.c_int64), ("method", C.c_int32), ("beta0", C.c_void_p)]


class _Result(C.Structure):
    _fields_ = [("objective", C.c_double), ("rel_change", C.c_double), ("rel_residual", C.c_double),
                ("mm_iters", C.c_int32), ("status", C.c_int32), ("cg_iters", C.c_int64),
                ("method_used", C.c_int32), ("threads", C.c_int32)]


class _Traj(C.Structure):
    _fields_ = [("f", C.c_double), ("f_eps", C.c_double), ("rel_change", C.c_double),
                ("rel_residual", C.c_double), ("cg", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        P, D = C.POINTER(_Problem), C.c_double
        L.ofl_solve.argtypes = [P, D, D, C.POINTER(_Opts), C.c_void_p, C.POINTER(_Result), C.c_void_p]
        L.ofl_solve.restype = C.c_int
        L.ofl_objective.argtypes = [P, D, D, C.c_void_p]
        L.ofl_objective.restype = D
        L.ofl_objective_eps.argtypes = [P, D, D, D, C.c_void_p]
        L.ofl_objective_eps.restype = D
        L.ofl_surrogate.argtypes = [P, D, D, D, C.c_void_p, C.c_void_p]
        L.ofl_surrogate.restype = D
        L.ofl_init_beta.argtypes = [P, C.c_void_p]
        L.ofl_gradient_eps.argtypes = [P, D, D, D, C.c_void_p, C.c_void_p]
        L.ofl_system.argtypes = [P, D, D, D, C.c_void_p, C.c_void_p, C.c_void_p]
        L.ofl_num_threads.restype = C.c_int
        _lib = L
    return _lib


class Problem:
    """Holds the stored X (float64 / float32 / uint16 bf16 bits), y and E."""

    def __init__(self, X, dtype, y, edges):
        dt = {F64: np.float64, F32: np.float32, BF16: np.uint16}[dtype]
        self.X = np.ascontiguousarray(X, dtype=dt)
        self.dtype = dtype
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        self.edges = np.ascontiguousarray(np.asarray(edges, dtype=np.int64).reshape(-1, 2))
        n, p = self.X.shape
        self._s = _Problem(n, p, p, dtype, self.X.ctypes.data, self.y.ctypes.data, self.edges.shape[0],
                           self.edges.ctypes.data if self.edges.size else None)

    @classmethod
    def from_instance(cls, inst):
        return cls(inst.X, inst.dtype, inst.y, inst.edges)

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def p(self):
        return self.X.shape[1]


@dataclass
class Result:
    beta: np.ndarray
    objective: float
    rel_change: float
    rel_residual: float
    mm_iters: int
    cg_iters: int
    status: int
    method: int
    threads: int
    traj: np.ndarray | None = None


def solve(P: Problem, lam1, lam2, eps=1e-8, tol=1e-8, inner_tol=0.0, max_iter=0, max_cg=0,
          method=ALG_AUTO, beta0=None, trajectory=False) -> Result:
    L = lib()
    b0 = None if beta0 is None else np.ascontiguousarray(beta0, dtype=np.float64)
    o = _Opts(eps, tol, inner_tol, max_iter, max_cg, method, None if b0 is None else b0.ctypes.data)
    out = np.zeros(P.p)
    res = _Result()
    cap = max_iter if max_iter > 0 else 10000
    tr = (_Traj * cap)() if trajectory else None
    L.ofl_solve(C.byref(P._s), lam1, lam2, C.byref(o), out.ctypes.data, C.byref(res),
                C.cast(tr, C.c_void_p) if tr is not None else None)
    traj = None
    if trajectory:
        k = res.mm_iters
        traj = np.array([(tr[i].f, tr[i].f_eps, tr[i].rel_change, tr[i].rel_residual, tr[i].cg) for i in range(k)],
                        dtype=[("f", "f8"), ("f_eps", "f8"), ("rel_change", "f8"), ("rel_residual", "f8"),
                               ("cg", "i8")])
    return Result(out, res.objective, res.rel_change, res.rel_residual, res.mm_iters, res.cg_iters, res.status,
                  res.method_used, res.threads, traj)


def objective(P: Problem, lam1, lam2, beta) -> float:
    b = np.ascontiguousarray(beta, dtype=np.float64)
    return lib().ofl_objective(C.byref(P._s), lam1, lam2, b.ctypes.data)


def objective_eps(P: Problem, lam1, lam2, eps, beta) -> float:
    b = np.ascontiguousarray(beta, dtype=np.float64)
    return lib().ofl_objective_eps(C.byref(P._s), lam1, lam2, eps, b.ctypes.data)


def surrogate(P: Problem, lam1, lam2, eps, beta, beta_ref) -> float:
    b = np.ascontiguousarray(beta, dtype=np.float64)
    r = np.ascontiguousarray(beta_ref, dtype=np.float64)
    return lib().ofl_surrogate(C.byref(P._s), lam1, lam2, eps, b.ctypes.data, r.ctypes.data)


def init_beta(P: Problem) -> np.ndarray:
    out = np.zeros(P.p)
    lib().ofl_init_beta(C.byref(P._s), out.ctypes.data)
    return out


def gradient_eps(P: Problem, lam1, lam2, eps, beta) -> np.ndarray:
    b = np.ascontiguousarray(beta, dtype=np.float64)
    g = np.zeros(P.p)
    lib().ofl_gradient_eps(C.byref(P._s), lam1, lam2, eps, b.ctypes.data, g.ctypes.data)
    return g


def system(P: Problem, lam1, lam2, eps, beta_ref):
    """Dense Q(beta_ref) = X^T X + lam1 A + lam2 B and c = X^T y (small p)."""
    b = np.ascontiguousarray(beta_ref, dtype=np.float64)
    Q = np.zeros((P.p, P.p))
    c = np.zeros(P.p)
    lib().ofl_system(C.byref(P._s), lam1, lam2, eps, b.ctypes.data, Q.ctypes.data, c.ctypes.data)
    return Q, c


def num_threads() -> int:
    return int(lib().ofl_num_threads())
