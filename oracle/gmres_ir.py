"""GMRES-IR oracle: iterative refinement whose correction equation is solved
by left-preconditioned GMRES, the low-precision LU being the preconditioner
(paper: sections "Krylov-IR" and "GMRES-IR"; statistics in "Harvesting
Iteration Statistics: Part 2").

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  The library under test never imports
this module, and this module never imports the library.

What it computes (the outer loop, TW = F64 or F32 with TR = F64, is the
one of ``oracle.krylov_ir``):

* Each correction: GMRES on P A d = P r with P = U^{-1} L^{-1} Pi (the
  factors promoted to binary64 and the substitutions done in binary64, the
  paper's on-the-fly solve), x0 = 0, at most ``basissize`` iterations (no
  restart), Arnoldi with classical Gram-Schmidt applied twice, Givens
  rotations on the Hessenberg matrix; it stops when the estimated
  preconditioned residual is at most ``eta`` ||P r||_2.  The number of
  iterations goes to khist.

The paper fixes neither the orthogonalisation nor the inner tolerance; the
readings (classical Gram-Schmidt twice; eta = 1e-13 by default, the setting
under which the printed statistics session of "Harvesting Iteration
Statistics: Part 2" reproduces) are listed with the project's other
readings.
"""
from __future__ import annotations

import numpy as np

from oracle.krylov_ir import KrylovIRResult, krylov_ir_solve


def givens(a: float, b: float):
    """(c, s) with [c s; -s c] [a; b] = [r; 0], r = hypot(a, b)."""
    if b == 0.0:
        return 1.0, 0.0
    r = float(np.hypot(a, b))
    return a / r, b / r


def gmres(apply_op, rhs: np.ndarray, m: int, eta: float):
    """Left-preconditioned GMRES from x0 = 0 (``apply_op`` already includes
    the preconditioner, ``rhs`` is the preconditioned right-hand side).

    Returns (d, k, est): the iterate after k iterations and the estimated
    residual norm |g_k|."""
    n = rhs.size
    beta = float(np.linalg.norm(rhs))
    if beta == 0.0 or not np.isfinite(beta):
        return np.zeros(n), 0, beta
    V = np.zeros((m + 1, n))
    V[0] = rhs / beta
    H = np.zeros((m + 1, m))
    g = np.zeros(m + 1)
    g[0] = beta
    cs = np.zeros(m)
    sn = np.zeros(m)
    k_end = m
    for k in range(m):
        w = apply_op(V[k])
        # classical Gram-Schmidt, applied twice
        h = V[:k + 1] @ w
        w = w - V[:k + 1].T @ h
        h2 = V[:k + 1] @ w
        w = w - V[:k + 1].T @ h2
        h = h + h2
        hk1 = float(np.linalg.norm(w))
        H[:k + 1, k] = h
        H[k + 1, k] = hk1
        if hk1 > 0.0:
            V[k + 1] = w / hk1
        # earlier rotations, then the one that zeroes H[k+1, k]
        for i in range(k):
            t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
            H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        cs[k], sn[k] = givens(H[k, k], H[k + 1, k])
        H[k, k] = cs[k] * H[k, k] + sn[k] * H[k + 1, k]
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        if abs(g[k + 1]) <= eta * beta or hk1 == 0.0:
            k_end = k + 1
            break
    # back substitution with the triangular H, then d = V^T y
    y = np.zeros(k_end)
    for i in range(k_end - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:k_end] @ y[i + 1:k_end]) / H[i, i]
    d = V[:k_end].T @ y
    return d, k_end, abs(g[k_end])


GmresIRResult = KrylovIRResult


def gmres_ir_solve(at: np.ndarray, b: np.ndarray, tf: int, basissize: int = 10,
                   eta: float = 1e-13, Rmax: float = 0.5, litmax: int = 10,
                   tol_rel: float = 0.0) -> KrylovIRResult:
    """GMRES-IR on A x = b, A given in column-major storage (TW = F64 or
    F32), TR = F64 (the outer loop of ``oracle.krylov_ir``)."""
    def inner(op, rhs):
        d, k, _ = gmres(op, rhs, basissize, eta)
        return d, k
    return krylov_ir_solve(at, b, tf, inner, Rmax=Rmax, litmax=litmax, tol_rel=tol_rel)
