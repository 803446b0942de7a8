"""Pins of the oracle's residual (eq. xferrule, section "Evaluating the
residual in extended precision"), of its report line (relres and the normwise
backward error of section "Residual or Backward Error") and of its binary16
solve mode, against exact rational arithmetic at N <= 8.

eq. xferrule: A, x and b are promoted exactly from TW to TR and every
operation is then done in TR.  The replay below does each product and each
sum with Fractions and rounds it to TR by the format's definition, summing in
increasing column index and subtracting the sum from b_i, which is the order
the oracle states.  The oracle must agree bit for bit.  A mistake in the C
code that changes any rounding -- accumulating a TR = F32 sum in binary64, a
fused multiply-add, a transposed index, reading the padding rows of lda > n,
a dropped b -- changes at least one of these values.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from test_oracle_exact import rnd, replay_lu, replay_trsv

# (TW, TR) pairs the paper allows: TR is TW or wider (eq. xferrule promotes).
PAIRS = [("f64", "f64"), ("f32", "f64"), ("f32", "f32")]
NP = {"f64": np.float64, "f32": np.float32}


def replay_residual(a, b, x, tr):
    """r_i = fl_R(b_i - acc_i), acc_i = fl_R(acc + fl_R(a_ij x_j)), j = 0.. ."""
    n = len(b)
    r = []
    for i in range(n):
        acc = Fr(0)
        for j in range(n):
            acc = rnd(acc + rnd(a[i][j] * x[j], tr), tr)
        r.append(rnd(b[i] - acc, tr))
    return r


def _cases():
    rng = np.random.default_rng(2024)
    out = []
    for n in (1, 2, 3, 5, 8):
        for s in range(4):
            a = rng.standard_normal((n, n)) * 10.0 ** rng.integers(-4, 4, (n, n))
            x = rng.standard_normal(n) * 10.0 ** rng.integers(-2, 3, n)
            # b close to A x so the subtraction cancels (the refinement's case)
            b = a @ x * (1 + 1e-6 * rng.standard_normal(n))
            out.append((f"n{n}s{s}", a, x, b))
    # cancellation down to zero, exact products, a zero column
    a = np.array([[1.0, 2.0, -3.0], [0.5, 0.0, 4.0], [3.0, -1.0, 0.25]])
    x = np.array([1.0, 1.0, 1.0])
    out.append(("exact", a, x, a @ x))
    a = np.array([[1e8, 1.0, -1e8, 3.0], [2.0, 2.0**-30, 7.0, 0.0],
                  [1.0, 1.0, 1.0, 1.0], [0.0, 0.0, 0.0, 0.0]])
    out.append(("cancel", a, np.array([1.0, 3.0, 1.0, 2.0**-20]), np.array([1.0, 2.0, 3.0, 4.0])))
    return out


@pytest.mark.parametrize("tw,tr", PAIRS)
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_residual_bitwise_vs_rational_replay(orc, case, tw, tr):
    _, a, x, b = case
    n = len(b)
    dt = NP[tw]
    a, x, b = a.astype(dt), x.astype(dt), b.astype(dt)
    lda = n + 3
    buf = np.full((n, lda), np.nan, dtype=dt)   # padding rows are NaN: never read
    buf[:, :n] = a.T                             # column-major: buf[j, i] = A[i, j]
    r = orc.residual(buf, b, x, orc.F64 if tr == "f64" else orc.F32, lda=lda)
    ra = [[Fr(float(a[i, j])) for j in range(n)] for i in range(n)]
    rr = replay_residual(ra, [Fr(float(v)) for v in b], [Fr(float(v)) for v in x], tr)
    assert all(np.isfinite(r))
    for i in range(n):
        assert Fr(float(r[i])) == rr[i], (i, float(r[i]), float(rr[i]))


def test_binary32_residual_is_not_a_binary64_sum(orc):
    """The cases above discriminate: with TR = F32 a binary64 accumulation
    (rounded once at the end) gives a different r for some of them."""
    differs = 0
    for _, a, x, b in _cases():
        n = len(b)
        a, x, b = a.astype(np.float32), x.astype(np.float32), b.astype(np.float32)
        r = orc.residual(np.ascontiguousarray(a.T), b, x, orc.F32)
        ra = [[Fr(float(a[i, j])) for j in range(n)] for i in range(n)]
        wide = replay_residual(ra, [Fr(float(v)) for v in b], [Fr(float(v)) for v in x], "f64")
        wide = [rnd(v, "f32") for v in wide]
        differs += any(Fr(float(r[i])) != wide[i] for i in range(n))
    assert differs >= 3


@pytest.mark.parametrize("tw,tf,tr", [("f64", "f32", "f64"), ("f64", "f16", "f64"),
                                      ("f32", "f16", "f32"), ("f32", "f32", "f64")])
def test_report_line_vs_exact(orc, tw, tf, tr):
    """relres = ||b - A x|| / ||b|| and eta = ||b - A x|| / (||A|| ||x|| + ||b||)
    of the returned x (section "Residual or Backward Error"): the oracle's
    binary64 values against the exact residual of its own x.  Their residual
    is a binary64 dot product, so |r_i - r_i(exact)| <= gamma_{n+1}(u_d)
    (sum_j |a_ij x_j| + |b_i|) bounds the difference; ||A||, ||b|| and ||x||
    are exact maxima of exactly summed rows."""
    n = 8
    rng = np.random.default_rng(7)
    a = (rng.standard_normal((n, n)) + 4 * np.eye(n)).astype(NP[tw])
    b = rng.standard_normal(n).astype(NP[tw])
    T = {"f32": orc.F32, "f16": orc.F16}[tf]
    R = {"f64": orc.F64, "f32": orc.F32}[tr]
    res = orc.ir_solve(np.ascontiguousarray(a.T), b, T, tr=R, litmax=1)
    assert res.n_iter == 1
    A = [[Fr(float(a[i, j])) for j in range(n)] for i in range(n)]
    X = [Fr(float(v)) for v in res.x]
    B = [Fr(float(v)) for v in b]
    r = [B[i] - sum(A[i][j] * X[j] for j in range(n)) for i in range(n)]
    rn = max(abs(v) for v in r)
    anorm = max(sum(abs(v) for v in row) for row in A)
    bnorm = max(abs(v) for v in B)
    xnorm = max(abs(v) for v in X)
    # ||A|| is summed left to right in binary64 (one rounding per addition)
    assert abs(Fr(res.anorm) - anorm) <= anorm * n * Fr(2) ** -53
    assert Fr(res.bnorm) == bnorm and Fr(res.xnorm) == xnorm
    g = (n + 1) * 2.0**-53 / (1 - (n + 1) * 2.0**-53)
    slack = Fr(g) * max(sum(abs(A[i][j] * X[j]) for j in range(n)) + abs(B[i]) for i in range(n))
    relres = rn / bnorm
    eta = rn / (anorm * xnorm + bnorm)
    assert abs(Fr(res.relres) - relres) <= slack / bnorm + relres * Fr(2) ** -52
    assert abs(Fr(res.bwd_err) - eta) <= slack / (anorm * xnorm + bnorm) * (1 + Fr(1, 100)) \
        + eta * Fr(2) ** -50
    # a wrong denominator (||A|| ||x|| alone, or + ||b|| dropped) fails here
    assert res.bwd_err < res.relres


@pytest.mark.parametrize("mode", ["f16mixed", "f16strict"])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [2, 5, 8])
def test_binary16_solve_mode_vs_rational_replay(orc, mode, seed, n):
    """ORC_TS_F16: substitutions with every product, difference and quotient
    rounded to binary16, on binary16 factors and a binary16 right-hand side
    (the all-half low-precision solve of section "Interprecision Transfers:
    Part I" read literally).  Replayed with Fractions rounded to binary16."""
    rng = np.random.default_rng(100 * n + seed)
    a = rng.standard_normal((n, n)) + 2 * np.eye(n)
    af, _, st = orc.downcast(np.ascontiguousarray(a.T), orc.F16)
    assert st == 0
    lu_mode = {"f16mixed": orc.LU_F16MIXED, "f16strict": orc.LU_F16STRICT}[mode]
    lu, ipiv, info, _ = orc.lu(af, lu_mode)
    assert info == 0
    ra = [[Fr(float(af[i, j])) for j in range(n)] for i in range(n)]
    rl, rp, _ = replay_lu(ra, mode)
    assert list(ipiv) == rp
    y0 = orc.fl_h(rng.standard_normal(n))
    y = orc.trsv_lu(lu, y0, orc.TS_F16)
    ry = replay_trsv(rl, [Fr(float(v)) for v in y0], "f16")
    assert all(np.isfinite(y))
    assert all(Fr(float(y[i])) == ry[i] for i in range(n))
    # and it is not the binary32 solve: rounding every operation to binary16
    # moves the result for most of these systems
    y32 = orc.trsv_lu(lu, y0, orc.TS_F32)
    assert np.array_equal(orc.fl_h(y), y)
    if n == 8:
        assert not np.array_equal(y, y32)
