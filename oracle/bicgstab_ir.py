"""BiCGSTAB-IR oracle: iterative refinement whose correction equation is
solved by BiCGSTAB (van der Vorst's stabilised bi-conjugate gradients),
preconditioned with the low-precision LU (paper: section "Krylov-IR"; the
package's mpblu, used in section "IR-Krylov").

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The library under test never imports
this module, and this module never imports the library.

What it computes (the outer loop, TW = F64 or F32 with TR = F64, is the
one of ``oracle.krylov_ir``):

* Each correction: BiCGSTAB on P A d = P r, P = U^{-1} L^{-1} Pi applied in
  binary64 on the TF factors, from d = 0 with shadow vector r^ = P r, at most
  ``maxit`` iterations; it stops when ||s||_2 (after the half step) or
  ||r||_2 (after the full step) is at most ``eta`` ||P r||_2, or on a
  breakdown (a zero denominator), keeping the last iterate.  The number of
  iterations (a half step counts as one) goes to khist.

The paper fixes neither the preconditioning side, the inner tolerance nor
the iteration limit; the readings (left preconditioning as in GMRES-IR,
eta = 1e-13, at most 10 iterations) are listed with the project's other
readings.
"""
from __future__ import annotations

import numpy as np

from oracle.krylov_ir import KrylovIRResult, krylov_ir_solve


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


BicgstabIRResult = KrylovIRResult


def bicgstab_ir_solve(at: np.ndarray, b: np.ndarray, tf: int, maxit: int = 10,
                      eta: float = 1e-13, Rmax: float = 0.5, litmax: int = 10,
                      tol_rel: float = 0.0) -> KrylovIRResult:
    """BiCGSTAB-IR on A x = b, A given in column-major storage (TW = F64 or
    F32), TR = F64 (the outer loop of ``oracle.krylov_ir``)."""
    def inner(op, rhs):
        d, k, _ = bicgstab(op, rhs, maxit, eta)
        return d, k
    return krylov_ir_solve(at, b, tf, inner, Rmax=Rmax, litmax=litmax, tol_rel=tol_rel)
