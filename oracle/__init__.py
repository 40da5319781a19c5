"""CPU oracle for the SPD solve -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1405_4644_amd``) and never imports it.

``liboracle.so`` is built from ``oracle.c`` with plain ``gcc -O2`` (no fast-math,
no FMA contraction).  Matrices are passed column-major; for the symmetric A the
row-/column-major distinction does not matter.  Right-hand sides are handled
as ``(m, n)`` row-major arrays whose row c is column c of the n x m matrix,
i.e. exactly the column-major memory layout.

Functions mirror the paper's steps (Section 3.1, Eq. (3), Algorithm 1); see
``oracle.c`` for the definitions.  ``exact`` holds exact rational references
for tiny systems.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

PREC = {"bf16": 0, "fp16": 1, "fp32": 2, "fp64": 3}
STATUS_OK, STATUS_NOT_SPD, STATUS_NO_CONVERGENCE = 0, 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("prec_used", C.c_int32), ("iters_low", C.c_int32),
                ("iters_high", C.c_int32), ("fallbacks", C.c_int32), ("info", C.c_int64),
                ("eta", C.c_double)]


@dataclass
class IRReport:
    status: int
    prec_used: int
    iters_low: int
    iters_high: int
    fallbacks: int
    info: int
    eta: float


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        i64, f64, i32, vp = C.c_int64, C.c_double, C.c_int32, C.c_void_p
        L.oracle_potrf.argtypes = [i64, vp, i64, vp, i64]
        L.oracle_potrf.restype = i64
        for f in (L.oracle_fsub, L.oracle_bsub):
            f.argtypes = [i64, i64, vp, i64, vp, i64]
            f.restype = None
        L.oracle_potrs.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64]
        L.oracle_residual.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, vp, i64]
        L.oracle_residual_rows.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, i64, vp, vp]
        L.oracle_residual_given_rows.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, i64, vp, vp]
        L.oracle_norminf_sym.argtypes = [i64, vp, i64]
        L.oracle_norminf_sym.restype = f64
        L.oracle_backward_error.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, vp]
        L.oracle_rne_f16.argtypes = [C.c_float]
        L.oracle_rne_f16.restype = C.c_float
        L.oracle_rne_bf16.argtypes = [C.c_float]
        L.oracle_rne_bf16.restype = C.c_float
        L.oracle_lowprec_factor.argtypes = [i64, vp, i64, i32, i32, f64, vp, i64, vp, C.POINTER(f64)]
        L.oracle_lowprec_factor.restype = i64
        L.oracle_ir.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, i32, i32, f64, f64, i32,
                                i32, C.POINTER(_Report)]
        L.oracle_ir_factor.argtypes = [i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, i32, f64, i32,
                                       C.POINTER(_Report)]
        L.oracle_ir_factor.restype = i32
        L.oracle_cg_ir.argtypes = [i64, i64, vp, i64, i64, vp, i64, vp, i64, f64, f64, i32, i32,
                                   C.POINTER(_Report)]
        L.oracle_cg_ir.restype = i32
        L.oracle_ir.restype = i32
        L.oracle_threads.restype = i32
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _f64(a):
    a = np.asarray(a, dtype=np.float64)
    return a


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _colmajor(A):
    """Return a Fortran-ordered float64 copy/view of the square matrix A."""
    return np.asfortranarray(_f64(A))


def potrf(A):
    """Cholesky A = L L^T from the lower triangle.  Returns (L, info)."""
    A = _colmajor(A)
    n = A.shape[0]
    L = np.zeros((n, n), dtype=np.float64, order="F")
    info = lib().oracle_potrf(n, _ptr(A), n, _ptr(L), n)
    return L, int(info)


def _rhs(Bt):
    Bt = np.ascontiguousarray(_f64(Bt))
    if Bt.ndim == 1:
        Bt = Bt[None, :]
    return Bt


def fsub(L, Bt):
    L = _colmajor(L)
    Y = _rhs(Bt).copy()
    m, n = Y.shape
    lib().oracle_fsub(n, m, _ptr(L), n, _ptr(Y), n)
    return Y


def bsub(L, Bt):
    L = _colmajor(L)
    Y = _rhs(Bt).copy()
    m, n = Y.shape
    lib().oracle_bsub(n, m, _ptr(L), n, _ptr(Y), n)
    return Y


def potrs(L, Bt):
    """X = L^{-T} L^{-1} B (Eq. (3)); B and X as (m, n)."""
    L = _colmajor(L)
    B = _rhs(Bt)
    m, n = B.shape
    X = np.empty_like(B)
    lib().oracle_potrs(n, m, _ptr(L), n, _ptr(B), n, _ptr(X), n)
    return X


def solve(A, Bt):
    """Plain binary64 Cholesky solve: the result Algorithm 1 converges to.
    Returns (X as (m, n), info)."""
    L, info = potrf(A)
    if info:
        return None, info
    return potrs(L, Bt), 0


def residual(A, Xt, Bt):
    A = _colmajor(A)
    X, B = _rhs(Xt), _rhs(Bt)
    m, n = X.shape
    R = np.empty_like(X)
    lib().oracle_residual(n, m, _ptr(A), n, _ptr(X), n, _ptr(B), n, _ptr(R), n)
    return R


def residual_rows(A, Xt, Bt, rows):
    """Residual entries r_i for the given rows only; returns (m, len(rows))."""
    A = _colmajor(A)
    X, B = _rhs(Xt), _rhs(Bt)
    m, n = X.shape
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    R = np.empty((m, rows.size), dtype=np.float64)
    lib().oracle_residual_rows(n, m, _ptr(A), n, _ptr(X), n, _ptr(B), n, rows.size,
                               _ptr(rows), _ptr(R))
    return R


def residual_given_rows(Arows, Xt, Bt, rows):
    """Residual entries b_i - sum_j a_ij x_j of the listed rows, from those
    rows of the symmetric A only (Arows: len(rows) x n).  Returns (m, len(rows))."""
    X, B = _rhs(Xt), _rhs(Bt)
    m, n = X.shape
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    Ar = np.asfortranarray(np.asarray(Arows, dtype=np.float64))
    assert Ar.shape == (rows.size, n)
    R = np.empty((m, rows.size), dtype=np.float64)
    lib().oracle_residual_given_rows(n, m, _ptr(Ar), rows.size, _ptr(X), n, _ptr(B), n, rows.size,
                                     _ptr(rows), _ptr(R))
    return R


def norminf_sym(A):
    A = _colmajor(A)
    return float(lib().oracle_norminf_sym(A.shape[0], _ptr(A), A.shape[0]))


def backward_error(A, Xt, Bt):
    """eta_c = ||b_c - A x_c||_inf / (||A||_inf ||x_c||_inf + ||b_c||_inf)."""
    A = _colmajor(A)
    X, B = _rhs(Xt), _rhs(Bt)
    m, n = X.shape
    eta = np.empty(m, dtype=np.float64)
    lib().oracle_backward_error(n, m, _ptr(A), n, _ptr(X), n, _ptr(B), n, _ptr(eta))
    return eta


def rne_f16(x: float) -> float:
    return float(lib().oracle_rne_f16(float(np.float32(x))))


def rne_bf16(x: float) -> float:
    return float(lib().oracle_rne_bf16(float(np.float32(x))))


def lowprec_factor(A, prec="fp32", equilibrate=True, theta=0.1):
    """The low-precision factorisation of Algorithm 1 with its scaling, as ``ir`` forms it.  Returns
    (L widened to binary64, d, mu, info): L is the factor of
    H = round32(mu D A D) (binary32 arithmetic; binary16/bfloat16 update
    operands), or of A itself for "fp64" (d = 1, mu = 1)."""
    A = _colmajor(A)
    n = A.shape[0]
    L = np.zeros((n, n), dtype=np.float64, order="F")
    d = np.empty(n, dtype=np.float64)
    mu = C.c_double(0.0)
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    info = lib().oracle_lowprec_factor(n, _ptr(A), n, p, int(bool(equilibrate)), float(theta), _ptr(L), n,
                                       _ptr(d), C.byref(mu))
    return L, d, float(mu.value), int(info)


def ir(A, Bt, prec="fp32", equilibrate=True, theta=0.1, tol=1e-14, max_iter=10, fallback=True):
    """Algorithm 1 emulated on the CPU.  Returns (X as (m, n), IRReport)."""
    A = _colmajor(A)
    B = _rhs(Bt)
    m, n = B.shape
    X = np.zeros_like(B)
    rep = _Report()
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    lib().oracle_ir(n, m, _ptr(A), n, _ptr(B), n, _ptr(X), n, p, int(bool(equilibrate)),
                    float(theta), float(tol), int(max_iter), int(bool(fallback)), C.byref(rep))
    return X, IRReport(rep.status, rep.prec_used, rep.iters_low, rep.iters_high, rep.fallbacks,
                       rep.info, rep.eta)


def ir_factor(A, L, Bt, prec="fp64", tol=1e-14, max_iter=10):
    """Algorithm 1 after its factorisation (first solve and refinement) with a
    given lower-triangular factor L in place of its own (the perturbed-factor
    experiment, Section 3.1, Fig. 3(b)):
    binary64 substitutions (prec "fp64") or L rounded to binary32 ("fp32"),
    no equilibration.  Returns (X as (m, n), IRReport)."""
    A = _colmajor(A)
    L = _colmajor(L)
    B = _rhs(Bt)
    m, n = B.shape
    X = np.zeros_like(B)
    rep = _Report()
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    lib().oracle_ir_factor(n, m, _ptr(A), n, _ptr(L), n, _ptr(B), n, _ptr(X), n, p, float(tol), int(max_iter),
                           C.byref(rep))
    return X, IRReport(rep.status, rep.prec_used, rep.iters_low, rep.iters_high, rep.fallbacks,
                       rep.info, rep.eta)


def cg_ir(A, Bt, X0t=None, half_band=-1, tol=1e-14, inner_tol=1e-6, max_outer=30, max_inner=2000):
    """Algorithm 2 (CG with iterative refinement) emulated on the CPU: the
    product with A~ (binary32, dense or the band |i-j| <= half_band) in
    binary32, everything else in binary64, restarted from binary64 residuals.
    Returns (X as (m, n), IRReport): iters_low = products, iters_high =
    binary64 residuals."""
    A = _colmajor(A)
    B = _rhs(Bt)
    m, n = B.shape
    X = np.zeros_like(B) if X0t is None else np.array(_rhs(X0t), dtype=np.float64, order="C")
    rep = _Report()
    lib().oracle_cg_ir(n, m, _ptr(A), n, int(half_band), _ptr(B), n, _ptr(X), n, float(tol), float(inner_tol),
                       int(max_outer), int(max_inner), C.byref(rep))
    return X, IRReport(rep.status, rep.prec_used, rep.iters_low, rep.iters_high, rep.fallbacks,
                       rep.info, rep.eta)


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(k: int) -> None:
    """Threads of the oracle's parallel loops from now on (OpenMP)."""
    lib().oracle_set_threads(int(k))
