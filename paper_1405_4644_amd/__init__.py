"""Python binding of libspd: mixed-precision Cholesky with iterative
refinement for dense SPD systems on MI355X (gfx950).

This module only marshals arguments to the C ABI declared in include/spd.h;
every step of the computation runs in the library's HIP kernels.  There is no
fallback: if libspd.so is missing or cannot be loaded, every call raises.
PyTorch supplies device memory and the current stream.

Layouts
  A   (n, n) float64 CUDA tensor.  Column-major storage (A.stride(0) == 1) is
      read as is; a row-major contiguous tensor is read as the column-major
      matrix A^T -- identical for the symmetric matrices this library solves.
      Only the lower triangle (of the column-major view) is read.
  B, X  (n,) vectors or (m, n) row-major tensors whose row c is right-hand
      side c -- i.e. the column-major n x m layout of Eq. (2).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspd.so")
_lib = None

# status and precision codes (spd.h)
OK, ERR_INVALID_ARG, ERR_NOT_SPD, ERR_NO_CONVERGENCE, ERR_DEVICE, ERR_OUT_OF_MEMORY, ERR_UNSUPPORTED = range(7)
PREC = {"bf16": 0, "fp16": 1, "fp32": 2, "fp64": 3, "auto": 4}
PREC_NAME = {v: k for k, v in PREC.items()}


class SPDError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_str(status)} ({status})")


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("fallback", C.c_int32),
                ("equilibrate", C.c_int32), ("theta", C.c_double)]


class CGOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("max_inner", C.c_int32)]


class Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("prec_used", C.c_int32), ("iters_low", C.c_int32),
                ("iters_high", C.c_int32), ("fallbacks", C.c_int32), ("info", C.c_int64),
                ("eta", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneResult(C.Structure):
    _fields_ = [("group", C.c_int32), ("upd_slots", C.c_int32), ("ms", C.c_double), ("from_cache", C.c_int32),
                ("n", C.c_int64), ("small_tiles", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# exported entry points: (name, restype, argtypes)
_vp, _i64, _i32, _f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double
_SIGS = [
    ("spd_opts_default", None, [C.POINTER(Opts)]),
    ("spd_factor", C.c_int, [_vp, _i64, _i64, C.c_int, C.POINTER(Opts), _vp, C.POINTER(_vp), C.POINTER(_i64)]),
    ("spd_solve", C.c_int, [_vp, _vp, _i64, _i64, _vp, _i64, _vp]),
    ("spd_refine", C.c_int, [_vp, _vp, _i64, _vp, _i64, _i64, _vp, _i64, C.POINTER(Opts), C.POINTER(Report), _vp]),
    ("spd_posv", C.c_int, [_vp, _i64, _i64, _vp, _i64, _i64, _vp, _i64, C.c_int, C.POINTER(Opts),
                           C.POINTER(Report), _vp, C.POINTER(_vp)]),
    ("spd_residual", C.c_int, [_vp, _i64, _i64, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _vp]),
    ("spd_residual_noalloc", C.c_int, [_vp, _i64, _i64, _vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _vp]),
    ("spd_solve_batched", C.c_int, [_i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(Opts), _vp, _vp]),
    ("spd_batched_config", C.c_int, [_i64, C.POINTER(_i32), C.POINTER(_i32)]),
    ("spd_solve_batched_timed", C.c_int, [_i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(Opts), _vp, _vp,
                                          _vp]),
    ("spd_picker_set", C.c_int, [_vp, _vp]),
    ("spd_picker_features", C.c_int, [_i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("spd_mlp_forward", C.c_int, [_vp, _vp, _i64, _vp, _vp]),
    ("spd_mlp_grad", C.c_int, [_vp, _vp, _vp, _i64, _vp, _vp, _vp]),
    ("spd_mlp_adam", C.c_int, [_vp, _vp, _vp, _vp, _i64, _i32, C.c_float, C.c_float, C.c_float, C.c_float, _vp]),
    ("spd_factor_import", C.c_int, [_vp, _i64, _i64, C.c_int, _vp, C.POINTER(_vp), C.POINTER(_i64)]),
    ("spd_factor_set_wait_limit", C.c_int, [_vp, _f64]),
    ("spd_autotune", C.c_int, [_i64, C.c_int, _vp, C.POINTER(TuneResult)]),
    ("spd_autotune_clear", None, []),
    ("spd_factor_destroy", None, [_vp]),
    ("spd_factor_query", C.c_int, [_vp, C.POINTER(_i64), C.POINTER(_i32), C.POINTER(_i32)]),
    ("spd_factor_export", C.c_int, [_vp, _vp, _i64, _vp, C.POINTER(_f64), _vp]),
    ("spd_cg_opts_default", None, [C.POINTER(CGOpts)]),
    ("spd_cg_prepare", C.c_int, [_vp, _i64, _i64, _i64, _vp, C.POINTER(_vp)]),
    ("spd_cg_refine", C.c_int, [_vp, _vp, _i64, _vp, _i64, _i64, _vp, _i64, C.POINTER(CGOpts), C.POINTER(Report),
                                _vp]),
    ("spd_cg_destroy", None, [_vp]),
    ("spd_profile_enable", None, [C.c_int]),
    ("spd_profile_reset", None, []),
    ("spd_profile_query", C.c_int, [C.c_int, C.POINTER(_i64), C.POINTER(_f64), C.POINTER(_f64), C.POINTER(_f64)]),
    ("spd_status_str", C.c_char_p, [C.c_int]),
    ("spd_version", C.c_char_p, []),
]


def load(path: str | None = None):
    """Load libspd.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libspd.so not built ({p}); run `python -m paper_1405_4644_amd.build`")
    # torch first: it carries its own HIP runtime (same soname), which libspd
    # then binds to.  Loaded the other way round, the process maps two HIP
    # runtimes and torch's streams and allocations are foreign to libspd.
    _torch()
    lib = C.CDLL(p)
    for name, res, args in _SIGS:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_str(s: int) -> str:
    return load().spd_status_str(int(s)).decode()


def default_opts(**kw) -> Opts:
    o = Opts()
    load().spd_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_dev(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")


def _mat(A):
    _check_dev(A, "A")
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    n = A.shape[0]
    if A.stride(0) == 1 and (n <= 1 or A.stride(1) >= n):
        ld = max(A.stride(1), 1)
    elif A.stride(1) == 1:
        ld = max(A.stride(0), 1)
    else:
        raise ValueError("A must have unit stride in one dimension")
    return C.c_void_p(A.data_ptr()), n, max(ld, n, 1)


def _rhs(B, n, name="B"):
    _check_dev(B, name)
    if B.dim() == 1:
        if B.shape[0] != n or (n > 1 and B.stride(0) != 1):
            raise ValueError(f"{name} must have length n and unit stride")
        return C.c_void_p(B.data_ptr()), max(n, 1), 1
    if B.dim() != 2 or B.shape[1] != n or (n > 1 and B.stride(1) != 1):
        raise ValueError(f"{name} must be (m, n) with unit stride along n")
    return C.c_void_p(B.data_ptr()), max(B.stride(0), n, 1), B.shape[0]


class Factor:
    """Owns an spd_factor_t handle (released by close() or garbage collection)."""

    def __init__(self):
        self.h = C.c_void_p()

    def close(self):
        if self.h:
            load().spd_factor_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_wait_limit(self, seconds: float):
        """spd_factor_set_wait_limit: bound of the substitutions' waits."""
        st = load().spd_factor_set_wait_limit(self.h, float(seconds))
        if st:
            raise SPDError(st, "spd_factor_set_wait_limit")

    def query(self):
        n, p, nb = C.c_int64(), C.c_int32(), C.c_int32()
        st = load().spd_factor_query(self.h, C.byref(n), C.byref(p), C.byref(nb))
        if st:
            raise SPDError(st, "spd_factor_query")
        return {"n": n.value, "prec": PREC_NAME[p.value], "nb": nb.value}


class CG:
    """Owns an spd_cg_t handle: the binary32 operator of Algorithm 2."""

    def __init__(self):
        self.h = C.c_void_p()
        self.n = 0

    def close(self):
        if self.h:
            load().spd_cg_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cg_default_opts(**kw) -> CGOpts:
    o = CGOpts()
    load().spd_cg_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def cg_prepare(A, half_band: int = -1, H: CG | None = None) -> CG:
    """spd_cg_prepare: the binary32 operator A~ (dense, or the band
    |i - j| <= half_band) for Algorithm 2."""
    pa, n, lda = _mat(A)
    H = H or CG()
    st = load().spd_cg_prepare(pa, n, lda, int(half_band), _stream(), C.byref(H.h))
    if st:
        raise SPDError(st, "spd_cg_prepare")
    H.n = n
    return H


def cg_refine(H: CG, A, B, X=None, opts: CGOpts | None = None):
    """spd_cg_refine (Algorithm 2 with binary64 restarts).  X (zero if not
    given) is the starting point and is updated in place.  Returns (X, Report)."""
    torch = _torch()
    pa, n, lda = _mat(A)
    pb, ldb, m = _rhs(B, n)
    if X is None:
        X = torch.zeros_like(B)
    px, ldx, _ = _rhs(X, n, "X")
    rep = Report()
    load().spd_cg_refine(H.h, pa, lda, pb, ldb, m, px, ldx, C.byref(opts) if opts else None, C.byref(rep), _stream())
    return X, rep


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)


def factor(A, prec="fp32", opts: Opts | None = None, F: Factor | None = None, check=True):
    """spd_factor: returns (Factor, info).  Raises on errors other than NOT_SPD unless check=False."""
    lib = load()
    pa, n, lda = _mat(A)
    F = F or Factor()
    info = C.c_int64()
    st = lib.spd_factor(pa, n, lda, _prec(prec), C.byref(opts) if opts else None, _stream(),
                        C.byref(F.h), C.byref(info))
    if check and st not in (OK, ERR_NOT_SPD):
        raise SPDError(st, "spd_factor")
    return F, int(info.value), st


def factor_import(L, prec="fp64", F: Factor | None = None, check=True):
    """spd_factor_import: the caller's lower-triangular factor L (an n x n
    float64 device tensor read as the matrix L[i][j], i >= j) becomes the
    handle's factor at `prec` ("fp64" or "fp32"), with no equilibration or
    scaling.  Returns (Factor, info, status)."""
    _check_dev(L, "L")
    if L.dim() != 2 or L.shape[0] != L.shape[1]:
        raise ValueError("L must be square")
    n = L.shape[0]
    if not (L.stride(0) == 1 and (n <= 1 or L.stride(1) >= n)):
        L = L.t().contiguous().t()  # column-major copy (the C ABI reads column-major)
    ld = max(L.stride(1), n, 1)
    lib = load()
    F = F or Factor()
    info = C.c_int64()
    st = lib.spd_factor_import(C.c_void_p(L.data_ptr()), n, ld, _prec(prec), _stream(), C.byref(F.h),
                               C.byref(info))
    if check and st not in (OK, ERR_NOT_SPD):
        raise SPDError(st, "spd_factor_import")
    return F, int(info.value), st


def solve(F: Factor, B, X=None):
    """spd_solve (Algorithm 1's first solve with the low-precision factor).  Returns X."""
    torch = _torch()
    n = F.query()["n"]
    pb, ldb, m = _rhs(B, n)
    if X is None:
        X = torch.empty_like(B)
    px, ldx, _ = _rhs(X, n, "X")
    st = load().spd_solve(F.h, pb, ldb, m, px, ldx, _stream())
    if st:
        raise SPDError(st, "spd_solve")
    return X


def refine(F: Factor, A, B, X, opts: Opts | None = None) -> Report:
    """spd_refine (Algorithm 1's refinement loop), X updated in place; returns the Report."""
    pa, n, lda = _mat(A)
    pb, ldb, m = _rhs(B, n)
    px, ldx, _ = _rhs(X, n, "X")
    rep = Report()
    load().spd_refine(F.h, pa, lda, pb, ldb, m, px, ldx, C.byref(opts) if opts else None, C.byref(rep),
                      _stream())
    return rep


def posv(A, B, prec="fp32", opts: Opts | None = None, F: Factor | None = None, X=None):
    """The whole of Algorithm 1: returns (X, Report, Factor)."""
    torch = _torch()
    pa, n, lda = _mat(A)
    pb, ldb, m = _rhs(B, n)
    if X is None:
        X = torch.empty_like(B)
    px, ldx, _ = _rhs(X, n, "X")
    F = F or Factor()
    rep = Report()
    load().spd_posv(pa, n, lda, pb, ldb, m, px, ldx, _prec(prec), C.byref(opts) if opts else None,
                    C.byref(rep), _stream(), C.byref(F.h))
    return X, rep, F


def residual(A, X, B, want_R=True):
    """spd_residual: returns (R or None, eta as a list) -- binary64 residual and backward errors."""
    import numpy as np
    torch = _torch()
    pa, n, lda = _mat(A)
    pb, ldb, m = _rhs(B, n)
    px, ldx, _ = _rhs(X, n, "X")
    R = torch.empty_like(B) if want_R else None
    pr, ldr = (_rhs(R, n, "R")[:2]) if want_R else (None, max(n, 1))
    eta = np.zeros(m, dtype=np.float64)
    st = load().spd_residual(pa, n, lda, px, ldx, pb, ldb, m, pr, ldr,
                             eta.ctypes.data_as(C.c_void_p), _stream())
    if st:
        raise SPDError(st, "spd_residual")
    return R, eta


def export(F: Factor):
    """Returns (L, d, mu): the factor of H = mu D A D as an (n, n) float64 tensor
    in column-major storage (use L.T for the row-major view), and D's diagonal."""
    torch = _torch()
    n = F.query()["n"]
    # allocate as (n, n) row-major; the library writes column-major, so the
    # tensor holds L^T when read row-major.
    Lt = torch.empty((n, n), dtype=torch.float64, device="cuda")
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    mu = C.c_double()
    st = load().spd_factor_export(F.h, C.c_void_p(Lt.data_ptr()), max(n, 1), C.c_void_p(d.data_ptr()),
                                  C.byref(mu), _stream())
    if st:
        raise SPDError(st, "spd_factor_export")
    return Lt.T, d, mu.value


K_UPDATE, K_RESIDUAL, K_CG_MV, K_CHAIN_UPDATE, K_TRSV, K_CONVERT = 0, 1, 2, 3, 4, 5


def profile_enable(on: bool = True):
    load().spd_profile_enable(int(bool(on)))


def profile_reset():
    load().spd_profile_reset()


def profile_query(kernel: int):
    """(launches, total_ms, total_flops, total_bytes) for a kernel class."""
    n, ms, fl, by = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
    st = load().spd_profile_query(int(kernel), C.byref(n), C.byref(ms), C.byref(fl), C.byref(by))
    if st:
        raise SPDError(st, "spd_profile_query")
    return n.value, ms.value, fl.value, by.value


# spd_report as laid out in device memory (batched reports)
REPORT_DTYPE = None


def _report_dtype():
    import numpy as np
    global REPORT_DTYPE
    if REPORT_DTYPE is None:
        REPORT_DTYPE = np.dtype({"names": [f for f, _ in Report._fields_],
                                 "formats": ["<i4", "<i4", "<i4", "<i4", "<i4", "<i8", "<f8"],
                                 "offsets": [getattr(Report, f).offset for f, _ in Report._fields_],
                                 "itemsize": C.sizeof(Report)})
    return REPORT_DTYPE


class Batch:
    """Device arrays of a packed batch: n, nrhs (int32), a_off, b_off (int64),
    A (float64, system s column-major n x n at a_off[s]), B and X (float64,
    n x m column-major at b_off[s]), prec (int32, in/out), reps (raw reports)."""

    def __init__(self, n, nrhs, a_off, A, b_off, B, X=None, prec="fp32"):
        torch = _torch()
        self.n, self.nrhs, self.a_off, self.b_off, self.A, self.B = n, nrhs, a_off, b_off, A, B
        for t, name, dt in ((n, "n", torch.int32), (nrhs, "nrhs", torch.int32), (a_off, "a_off", torch.int64),
                            (b_off, "b_off", torch.int64), (A, "A", torch.float64), (B, "B", torch.float64)):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise TypeError(f"{name} must be a contiguous {dt} CUDA tensor")
        self.batch = int(n.numel())
        self.X = torch.zeros_like(B) if X is None else X
        if isinstance(prec, torch.Tensor):
            self.prec = prec
        else:
            self.prec = torch.full((self.batch,), _prec(prec), dtype=torch.int32, device=n.device)
        self.reps = torch.zeros((max(self.batch, 1), C.sizeof(Report)), dtype=torch.uint8, device=n.device)

    def reports(self):
        import numpy as np
        raw = self.reps[:self.batch].cpu().numpy()
        return np.frombuffer(raw.tobytes(), dtype=_report_dtype())


def solve_batched(bt: Batch, opts: Opts | None = None, check=True, ticks=None) -> int:
    """Every system of the batch through Algorithm 1 in one persistent launch
    (asynchronous; the first call for a batch size also autotunes and
    synchronises).  Per-system outcomes: bt.reports(), bt.prec; with `ticks`
    (int64 CUDA tensor of batch entries) also each system's wall-clock ticks."""
    args = (bt.batch, C.c_void_p(bt.n.data_ptr()), C.c_void_p(bt.nrhs.data_ptr()),
            C.c_void_p(bt.a_off.data_ptr()), C.c_void_p(bt.A.data_ptr()),
            C.c_void_p(bt.b_off.data_ptr()), C.c_void_p(bt.B.data_ptr()),
            C.c_void_p(bt.X.data_ptr()), C.c_void_p(bt.prec.data_ptr()),
            C.byref(opts) if opts else None, C.c_void_p(bt.reps.data_ptr()))
    if ticks is None:
        st = load().spd_solve_batched(*args, _stream())
    else:
        st = load().spd_solve_batched_timed(*args, C.c_void_p(ticks.data_ptr()), _stream())
    if check and st != OK:
        raise SPDError(st, "spd_solve_batched")
    return st


# ---- learned precision picker --------------------------------------------------
PICKER_NFEAT, PICKER_NPARAM = 16, 5508


def _f32(t, name, numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements")


def picker_set(params=None):
    """Use these perceptron parameters for SPD_AUTO (None: switch the picker off)."""
    if params is None:
        st = load().spd_picker_set(None, _stream())
    else:
        _f32(params, "params", PICKER_NPARAM)
        st = load().spd_picker_set(C.c_void_p(params.data_ptr()), _stream())
    if st != OK:
        raise SPDError(st, "spd_picker_set")


PICKER_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "picker_weights.npz")


def picker_load(path: str | None = None):
    """Load trained perceptron parameters (default: the ones trained by
    paper_1405_4644_amd.picker_train and shipped with the package) and use
    them for SPD_AUTO; returns the parameter tensor."""
    import numpy as np
    torch = _torch()
    with np.load(path or PICKER_WEIGHTS, allow_pickle=False) as z:
        params = torch.from_numpy(np.ascontiguousarray(z["params"], dtype=np.float32)).cuda()
    picker_set(params)
    return params


def picker_features(bt: Batch):
    torch = _torch()
    feat = torch.empty((bt.batch, PICKER_NFEAT), dtype=torch.float32, device=bt.n.device)
    st = load().spd_picker_features(bt.batch, C.c_void_p(bt.n.data_ptr()), C.c_void_p(bt.nrhs.data_ptr()),
                                    C.c_void_p(bt.a_off.data_ptr()), C.c_void_p(bt.A.data_ptr()),
                                    C.c_void_p(feat.data_ptr()), _stream())
    if st != OK:
        raise SPDError(st, "spd_picker_features")
    return feat


def mlp_forward(params, X):
    torch = _torch()
    _f32(params, "params", PICKER_NPARAM)
    _f32(X, "X")
    out = torch.empty((X.shape[0], 4), dtype=torch.float32, device=X.device)
    st = load().spd_mlp_forward(C.c_void_p(params.data_ptr()), C.c_void_p(X.data_ptr()), X.shape[0],
                                C.c_void_p(out.data_ptr()), _stream())
    if st != OK:
        raise SPDError(st, "spd_mlp_forward")
    return out


def mlp_grad(params, X, y):
    """(gradient, loss) of the mean cross-entropy; both CUDA tensors."""
    torch = _torch()
    _f32(params, "params", PICKER_NPARAM)
    _f32(X, "X")
    if y.dtype != torch.int32 or not y.is_cuda:
        raise TypeError("y must be an int32 CUDA tensor")
    g = torch.empty(PICKER_NPARAM, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    st = load().spd_mlp_grad(C.c_void_p(params.data_ptr()), C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr()),
                             X.shape[0], C.c_void_p(g.data_ptr()), C.c_void_p(loss.data_ptr()), _stream())
    if st != OK:
        raise SPDError(st, "spd_mlp_grad")
    return g, loss


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    st = load().spd_mlp_adam(C.c_void_p(params.data_ptr()), C.c_void_p(grad.data_ptr()), C.c_void_p(m.data_ptr()),
                             C.c_void_p(v.data_ptr()), params.numel(), int(step), lr, beta1, beta2, eps, _stream())
    if st != OK:
        raise SPDError(st, "spd_mlp_adam")


def batched_config(batch: int):
    g, w = _i32(), _i32()
    st = load().spd_batched_config(int(batch), C.byref(g), C.byref(w))
    return (g.value, w.value) if st == OK else None


def autotune(n: int, prec="fp32") -> dict:
    """spd_autotune: the factorisation schedule for this order (rounded to a
    power of two) and precision, timed now or taken from the cache."""
    r = TuneResult()
    st = load().spd_autotune(int(n), _prec(prec), _stream(), C.byref(r))
    if st:
        raise SPDError(st, "spd_autotune")
    return r.as_dict()


def autotune_clear():
    load().spd_autotune_clear()


def version() -> str:
    return load().spd_version().decode()
