"""BiCGSTAB-IR oracle: iterative refinement whose correction equation is
solved by BiCGSTAB (van der Vorst's stabilised bi-conjugate gradients),
preconditioned with the low-precision LU (paper: section "Krylov-IR"; the
package's mpblu, used in section "IR-Krylov").

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The library under test never imports
this module, and this module never imports the library.

What it computes, in binary64 (TW = TR = F64):

* A_F = I_W^F(A), LU with partial pivoting in the TF mode of ``oracle.lu``.
* x = 0, r = b, the termination rules of Algorithm IR.
* Each correction: BiCGSTAB on P A d = P r, P = U^{-1} L^{-1} Pi applied in
  binary64 on the TF factors, from d = 0 with shadow vector r^ = P r, at most
  ``maxit`` iterations; it stops when ||s||_2 (after the half step) or
  ||r||_2 (after the full step) is at most ``eta`` ||P r||_2, or on a
  breakdown (a zero denominator), keeping the last iterate.  The number of
  iterations (a half step counts as one) goes to khist.
* x = x + d, r = b - A x (binary64, sum in column order), histories.

The paper fixes neither the preconditioning side, the inner tolerance nor
the iteration limit; the readings (left preconditioning as in GMRES-IR,
eta = 1e-13, at most 10 iterations) are listed with the project's other
readings.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import oracle as O


def bicgstab(apply_op, rhs: np.ndarray, maxit: int, eta: float):
    """BiCGSTAB from d = 0 for apply_op(d) = rhs.  Returns (d, k, est): the
    iterate after k iterations and the norm of its recurrence residual."""
    n = rhs.size
    d = np.zeros(n)
    r = rhs.copy()
    beta0 = float(np.linalg.norm(r))
    if beta0 == 0.0 or not np.isfinite(beta0):
        return d, 0, beta0
    rs = r.copy()                      # shadow residual
    rho_old = alpha = omega = 1.0
    p = np.zeros(n)
    v = np.zeros(n)
    tol = eta * beta0
    for k in range(1, maxit + 1):
        rho = float(rs @ r)
        if rho == 0.0:
            return d, k - 1, float(np.linalg.norm(r))
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply_op(p)
        den = float(rs @ v)
        if den == 0.0:
            return d, k - 1, float(np.linalg.norm(r))
        alpha = rho / den
        s = r - alpha * v
        sn = float(np.linalg.norm(s))
        if sn <= tol:
            return d + alpha * p, k, sn
        t = apply_op(s)
        tt = float(t @ t)
        if tt == 0.0:
            return d + alpha * p, k, sn
        omega = float(t @ s) / tt
        d = d + alpha * p + omega * s
        r = s - omega * t
        rn = float(np.linalg.norm(r))
        if rn <= tol or omega == 0.0:
            return d, k, rn
        rho_old = rho
    return d, maxit, float(np.linalg.norm(r))


@dataclass
class BicgstabIRResult:
    x: np.ndarray
    n_iter: int
    stop: int
    rhist: np.ndarray
    dhist: np.ndarray
    khist: np.ndarray
    relres: float
    info: int


def bicgstab_ir_solve(at: np.ndarray, b: np.ndarray, tf: int, maxit: int = 10,
                      eta: float = 1e-13, Rmax: float = 0.5, litmax: int = 10,
                      tol_rel: float = 0.0) -> BicgstabIRResult:
    """BiCGSTAB-IR on A x = b, A given in column-major storage (binary64)."""
    at = np.ascontiguousarray(at, dtype=np.float64)
    n = at.shape[1]
    A = at.T
    b = np.ascontiguousarray(b, dtype=np.float64)
    af, _, _ = O.downcast(at, tf)
    lu_rm, ipiv, info, _ = O.lu(af, O.default_lu_mode(tf))
    x = np.zeros(n)
    if info:
        return BicgstabIRResult(x, 0, 0, np.array([]), np.array([]), np.array([], dtype=int),
                                np.nan, info)
    tol = tol_rel if tol_rel > 0 else 2.0 ** -52

    def prec(v):
        return O.lu_solve(lu_rm, ipiv, v, O.TS_F64)

    def op(v):
        return prec(A @ v)

    r = b.copy()
    bnorm = float(np.abs(b).max())
    rh, dh, kh = [bnorm], [], []
    stop = 0
    if bnorm == 0.0:
        return BicgstabIRResult(x, 0, 0, np.array(rh), np.array(dh), np.array(kh, dtype=int), 0.0, 0)
    it = 0
    while True:
        d, k, _ = bicgstab(op, prec(r), maxit, eta)
        x = x + d
        r = O.residual(at, b, x, O.F64)
        it += 1
        rn = float(np.abs(r).max())
        rh.append(rn)
        dh.append(float(np.abs(d).max()))
        kh.append(k)
        if not np.isfinite(rn):
            stop = 4
            break
        if rn <= tol * bnorm:
            stop = 0
            break
        if it >= litmax:
            stop = 3
            break
        if rh[-1] >= Rmax * rh[-2]:
            stop = 1
            break
    return BicgstabIRResult(x, it, stop, np.array(rh), np.array(dh), np.array(kh, dtype=int),
                            rh[-1] / bnorm, 0)
