"""The outer loop shared by the Krylov-IR oracles (GMRES-IR, BiCGSTAB-IR;
paper: sections "Krylov-IR", "IR-Krylov").

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The library under test never imports
this module, and this module never imports the library.

* A_F = I_W^F(A), LU with partial pivoting in the TF mode of ``oracle.lu``.
* x = 0 (TW), r = b, rhist = [||b||_inf].
* Each correction: ``inner(op, P r)`` solves P A d = P r, P = U^{-1} L^{-1} Pi
  and A both applied in binary64 (A promoted from TW); it returns (d, k).
* TW = F64: x = x + d.  TW = F32 (TR = F64 > TW): d is rounded to binary32
  and x = fl_s(x + d), as in Algorithm IR with the residual in extended
  precision.
* r = b - A x in binary64 (sum in column order); rhist, dhist (||d||_inf of
  the correction as added), khist.
* Termination as in Algorithm IR: TR = TW: converged (||r|| <= tol ||b||),
  then litmax, then stagnation (||r_k|| >= Rmax ||r_{k-1}||); TR > TW:
  litmax, then eq. wilkterm on the corrections.  A non-finite residual or
  correction stops with code 4.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import oracle as O


@dataclass
class KrylovIRResult:
    x: np.ndarray
    n_iter: int
    stop: int
    rhist: np.ndarray
    dhist: np.ndarray
    khist: np.ndarray
    relres: float
    info: int


def krylov_ir_solve(at: np.ndarray, b: np.ndarray, tf: int, inner, Rmax: float = 0.5,
                    litmax: int = 10, tol_rel: float = 0.0) -> KrylovIRResult:
    """Krylov-IR on A x = b, A in column-major storage (TW = F64 or F32),
    TR = F64."""
    at = np.ascontiguousarray(at)
    if at.dtype not in (np.float64, np.float32):
        raise TypeError("TW must be binary64 or binary32")
    tw32 = at.dtype == np.float32
    n = at.shape[1]
    A = at.T.astype(np.float64)
    b = np.ascontiguousarray(b, dtype=at.dtype)
    af, _, _ = O.downcast(at, tf)
    lu_rm, ipiv, info, _ = O.lu(af, O.default_lu_mode(tf))
    x = np.zeros(n, dtype=at.dtype)
    if info:
        return KrylovIRResult(x, 0, 0, np.array([]), np.array([]), np.array([], dtype=int), np.nan, info)
    tol = tol_rel if tol_rel > 0 else 2.0 ** -52

    def prec(v):
        return O.lu_solve(lu_rm, ipiv, v, O.TS_F64)

    def op(v):
        return prec(A @ v)

    r = b.astype(np.float64)
    bnorm = float(np.abs(r).max())
    rh, dh, kh = [bnorm], [], []
    stop = 0
    if bnorm == 0.0:
        return KrylovIRResult(x, 0, 0, np.array(rh), np.array(dh), np.array(kh, dtype=int), 0.0, 0)
    it = 0
    while True:
        d, k = inner(op, prec(r))
        if tw32:
            dw = d.astype(np.float32)
            x = (x + dw).astype(np.float32)
            dn = float(np.abs(dw).max())
        else:
            x = x + d
            dn = float(np.abs(d).max())
        r = O.residual(at, b, x, O.F64)
        it += 1
        rn = float(np.abs(r).max())
        rh.append(rn)
        dh.append(dn)
        kh.append(k)
        if not (np.isfinite(rn) and np.isfinite(dn)):
            stop = 4
            break
        if not tw32:
            if rn <= tol * bnorm:
                stop = 0
                break
            if it >= litmax:
                stop = 3
                break
            if rh[-1] >= Rmax * rh[-2]:
                stop = 1
                break
        else:
            if it >= litmax:
                stop = 3
                break
            if it >= 2 and dh[-1] >= Rmax * dh[-2]:
                stop = 2
                break
    return KrylovIRResult(x, it, stop, np.array(rh), np.array(dh), np.array(kh, dtype=int),
                          rh[-1] / bnorm, 0)
