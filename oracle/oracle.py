"""ctypes wrapper of the C oracle (``mpir_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The library under test never imports
this module, and this module never imports the library: the two share no code.
Every function follows the passages cited in ``mpir_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpir_oracle.so")

F64, F32, F16, BF16 = 0, 1, 2, 3
LU_F64, LU_F32, LU_F16MIXED, LU_F16STRICT, LU_BF16MIXED = 0, 1, 2, 3, 4
TS_F64, TS_F32, TS_F16 = 0, 1, 2
STOP_NAMES = {0: "converged", 1: "stagnated", 2: "dstagnated", 3: "litmax",
              4: "nonfinite"}
OK, SINGULAR, ERR_ARG, ERR_ALLOC, ERR_NONFINITE, ERR_RANGE = 0, 1, -1, -2, -4, -5

_NP = {F64: np.float64, F32: np.float32}
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math, OpenMP)."""
    from oracle.build_oracle import build_oracle
    return build_oracle(force=force)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        p, i64, i32, d, vp = C.POINTER, C.c_int64, C.c_int32, C.c_double, C.c_void_p
        L.orc_fl_h.restype = d
        L.orc_fl_h.argtypes = [d]
        L.orc_fl_h_array.argtypes = [i64, vp, vp]
        L.orc_fl_b.restype = d
        L.orc_fl_b.argtypes = [d]
        L.orc_fl_b_array.argtypes = [i64, vp, vp]
        L.orc_downcast.restype = C.c_int
        L.orc_downcast.argtypes = [i64, vp, i64, C.c_int, C.c_int, vp, p(d)]
        L.orc_lu.restype = C.c_int
        L.orc_lu.argtypes = [i64, vp, C.c_int, vp, p(i64)]
        L.orc_apply_pivots.argtypes = [i64, vp, vp]
        L.orc_trsv_lu.argtypes = [i64, vp, C.c_int, vp]
        L.orc_lu_solve.argtypes = [i64, vp, vp, C.c_int, vp]
        L.orc_residual.argtypes = [i64, vp, i64, C.c_int, C.c_int, vp, vp, vp]
        L.orc_pow2_ceil.restype = d
        L.orc_pow2_ceil.argtypes = [d]
        L.orc_ir_solve.restype = C.c_int
        L.orc_ir_solve.argtypes = [i64, vp, i64, C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int, C.c_int, vp, vp,
                                   d, d, d, C.c_int, C.c_int, d, C.c_int,
                                   p(i32), p(i32), vp, vp, vp, p(i64)]
        L.orc_solve_f64.restype = C.c_int
        L.orc_solve_f64.argtypes = [i64, vp, i64, C.c_int, vp, vp, p(i64)]
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _prec_of(arr: np.ndarray) -> int:
    if arr.dtype == np.float64:
        return F64
    if arr.dtype == np.float32:
        return F32
    raise TypeError(f"unsupported working precision {arr.dtype}")


def fl_h(x):
    """Round binary64 values to binary16 (returned as binary64)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.empty_like(a)
    lib().orc_fl_h_array(a.size, _ptr(a), _ptr(out))
    return out


def fl_b(x):
    """Round binary64 values to bfloat16 (returned as binary64)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.empty_like(a)
    lib().orc_fl_b_array(a.size, _ptr(a), _ptr(out))
    return out


def downcast(at: np.ndarray, tf: int, lda: int | None = None):
    """A_F = I_W^F(A) (row-major, binary64 container) and ||A||_inf.

    ``at`` is column-major storage of A (at[j, i] = A[i, j])."""
    at = np.ascontiguousarray(at)
    n = at.shape[1]
    lda = n if lda is None else lda
    af = np.empty((n, n), dtype=np.float64)
    anorm = C.c_double(0.0)
    st = lib().orc_downcast(n, _ptr(at), lda, _prec_of(at), tf, _ptr(af), C.byref(anorm))
    return af, anorm.value, st


def lu(af: np.ndarray, mode: int):
    """LU with partial pivoting of a row-major matrix (copied)."""
    a = np.array(af, dtype=np.float64, order="C", copy=True)
    n = a.shape[0]
    ipiv = np.zeros(n, dtype=np.int32)
    info = C.c_int64(0)
    st = lib().orc_lu(n, _ptr(a), mode, _ptr(ipiv), C.byref(info))
    return a, ipiv, info.value, st


def lu_solve(lu_rm: np.ndarray, ipiv: np.ndarray, y: np.ndarray, ts: int):
    lu_rm = np.ascontiguousarray(lu_rm, dtype=np.float64)
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    v = np.array(y, dtype=np.float64, copy=True)
    lib().orc_lu_solve(v.size, _ptr(lu_rm), _ptr(ipiv), ts, _ptr(v))
    return v


def trsv_lu(lu_rm: np.ndarray, y: np.ndarray, ts: int):
    """U^{-1} L^{-1} y (no pivoting) with the packed factors."""
    lu_rm = np.ascontiguousarray(lu_rm, dtype=np.float64)
    v = np.array(y, dtype=np.float64, copy=True)
    lib().orc_trsv_lu(v.size, _ptr(lu_rm), ts, _ptr(v))
    return v


def apply_pivots(ipiv: np.ndarray, y: np.ndarray):
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int32)
    v = np.array(y, dtype=np.float64, copy=True)
    lib().orc_apply_pivots(v.size, _ptr(ipiv), _ptr(v))
    return v


def residual(at: np.ndarray, b: np.ndarray, x: np.ndarray, tr: int = F64,
             lda: int | None = None):
    """r = b - A x in precision tr (sum in increasing column order).

    ``at`` holds A column by column: at[j, i] = A[i, j].  With ``lda`` given,
    ``at`` has shape (n, lda), lda >= n, and entries i >= n of each column
    are padding that is never read."""
    at = np.ascontiguousarray(at)
    tw = _prec_of(at)
    b = np.ascontiguousarray(b, dtype=_NP[tw])
    x = np.ascontiguousarray(x, dtype=_NP[tw])
    n = b.size
    lda = n if lda is None else lda
    if lda < max(n, 1) or at.size < (n - 1) * lda + n:
        raise ValueError("A buffer too small for n and lda")
    r = np.empty(n, dtype=np.float64)
    lib().orc_residual(n, _ptr(at), lda, tw, tr, _ptr(b), _ptr(x), _ptr(r))
    return r


def pow2_ceil(m: float) -> float:
    return lib().orc_pow2_ceil(float(m))


@dataclass
class IRResult:
    status: int
    x: np.ndarray
    n_iter: int
    stop: int
    rhist: np.ndarray
    dhist: np.ndarray
    relres: float
    bwd_err: float
    anorm: float
    bnorm: float
    xnorm: float
    info: int
    extra: dict = field(default_factory=dict)

    @property
    def stop_name(self) -> str:
        return STOP_NAMES.get(self.stop, str(self.stop))


def default_lu_mode(tf: int) -> int:
    return {F64: LU_F64, F32: LU_F32, F16: LU_F16MIXED, BF16: LU_BF16MIXED}[tf]


def default_ts(tf: int) -> int:
    return TS_F64 if tf == F64 else TS_F32


def ir_solve(at: np.ndarray, b: np.ndarray, tf: int, tr: int | None = None,
             lu_mode: int | None = None, ts: int | None = None,
             Cr: float = 1.0, Ce: float = 1.0, Rmax: float = 0.5,
             litmax: int = 10, residterm: bool = True, tol_rel: float = 0.0,
             lda: int | None = None, onthefly: bool = False) -> IRResult:
    """Run Algorithm IR on A x = b (A given in column-major storage).

    onthefly: the mixed-precision solve of each correction (the package's
    onthefly option): the scaled residual is not rounded to TF and the
    substitutions run in TW arithmetic on the TF factors."""
    at = np.ascontiguousarray(at)
    tw = _prec_of(at)
    tr = tw if tr is None else tr
    lu_mode = default_lu_mode(tf) if lu_mode is None else lu_mode
    mps = onthefly and tf != tw
    if ts is None:
        ts = (TS_F64 if tw == F64 else TS_F32) if mps else default_ts(tf)
    rhat = tw if mps else tf
    n = at.shape[1]
    lda = n if lda is None else lda
    b = np.ascontiguousarray(b, dtype=_NP[tw])
    x = np.zeros(n, dtype=_NP[tw])
    cap = litmax + 2
    rh = np.zeros(cap, dtype=np.float64)
    dh = np.zeros(cap, dtype=np.float64)
    out = np.zeros(5, dtype=np.float64)
    nit, stop, info = C.c_int32(0), C.c_int32(0), C.c_int64(0)
    st = lib().orc_ir_solve(n, _ptr(at), lda, tw, tf, tr, lu_mode, ts, rhat,
                            _ptr(b), _ptr(x), Cr, Ce, Rmax, litmax,
                            1 if residterm else 0, tol_rel, cap,
                            C.byref(nit), C.byref(stop), _ptr(rh), _ptr(dh),
                            _ptr(out), C.byref(info))
    k = nit.value
    return IRResult(st, x, k, stop.value, rh[:k + 1].copy(), dh[:k].copy(),
                    out[0], out[1], out[2], out[3], out[4], info.value)


def solve_f64(at: np.ndarray, b: np.ndarray):
    """Binary64 LU solve of the promoted problem; returns (x, info, status)."""
    at = np.ascontiguousarray(at)
    tw = _prec_of(at)
    n = at.shape[1]
    b = np.ascontiguousarray(b, dtype=_NP[tw])
    x = np.zeros(n, dtype=np.float64)
    info = C.c_int64(0)
    st = lib().orc_solve_f64(n, _ptr(at), n, tw, _ptr(b), _ptr(x), C.byref(info))
    return x, info.value, st


def num_threads() -> int:
    return lib().orc_num_threads()
