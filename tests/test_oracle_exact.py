"""Brute-force pins of the oracle at N <= 8 with exact rational arithmetic.

1. The exact solution of A x = b (Fractions, Gaussian elimination without
   rounding) bounds the oracle's binary64 solve: forward error <= c*kappa*u.
2. The emulated low-precision LU of every mode is replayed with Fractions,
   applying IEEE round-to-nearest-even to binary32/binary16/bfloat16 after each
   operation, from the format's definition (precision p, minimum exponent,
   overflow).  This pins the C rounding machinery -- contraction, excess
   precision, the binary16 rounding routine -- independently of it: L, U and
   the pivot sequence must agree bit for bit.
"""
from fractions import Fraction as Fr
import math

import numpy as np
import pytest

FMT = {"f64": (53, -1022, 1023), "f32": (24, -126, 127), "f16": (11, -14, 15),
       "bf16": (8, -126, 127)}
INF = float("inf")


def rnd(v, fmt):
    """Round a Fraction to the nearest value of the binary format (ties even)."""
    if v == INF or v == -INF:
        return v
    p, emin, emax = FMT[fmt]
    if v == 0:
        return Fr(0)
    s = -1 if v < 0 else 1
    a = abs(v)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fr(2) ** e > a:
        e -= 1
    while Fr(2) ** (e + 1) <= a:
        e += 1
    e = max(e, emin)
    q = Fr(2) ** (e - (p - 1))
    m = a / q
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fr(1, 2) or (rem == Fr(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * q
    if r > (2 - Fr(2) ** (1 - p)) * Fr(2) ** emax:
        return s * INF
    return s * r


def replay_lu(a, mode):
    """Right-looking LU with partial pivoting, each op rounded per mode."""
    n = len(a)
    a = [row[:] for row in a]
    ipiv = []
    info = 0
    work = {"f64": "f64", "f32": "f32", "f16mixed": "f32", "f16strict": "f16",
            "bf16mixed": "f32"}[mode]
    low = {"f16mixed": "f16", "bf16mixed": "bf16"}.get(mode)
    for k in range(n):
        p = max(range(k, n), key=lambda i: (abs(a[i][k]), -i))
        ipiv.append(p)
        if p != k:
            a[k], a[p] = a[p], a[k]
        if low:
            for j in range(k, n):
                a[k][j] = rnd(a[k][j], low)
        if a[k][k] == 0:
            info = info or k + 1
            continue
        for i in range(k + 1, n):
            l = rnd(a[i][k] / a[k][k], work)
            if low:
                l = rnd(l, low)
            a[i][k] = l
            for j in range(k + 1, n):
                prod = rnd(l * a[k][j], work)
                a[i][j] = rnd(a[i][j] - prod, work)
    return a, ipiv, info


def replay_trsv(lu, y, fmt):
    n = len(y)
    y = [rnd(v, fmt) for v in y]          # the solve works on TS numbers
    for j in range(n):
        for i in range(j + 1, n):
            y[i] = rnd(y[i] - rnd(lu[i][j] * y[j], fmt), fmt)
    for j in range(n - 1, -1, -1):
        y[j] = rnd(y[j] / lu[j][j], fmt)
        for i in range(j):
            y[i] = rnd(y[i] - rnd(lu[i][j] * y[j], fmt), fmt)
    return y


def exact_solve(a, b):
    n = len(b)
    m = [row[:] + [bb] for row, bb in zip(a, b)]
    for k in range(n):
        p = next(i for i in range(k, n) if m[i][k] != 0)
        m[k], m[p] = m[p], m[k]
        for i in range(k + 1, n):
            f = m[i][k] / m[k][k]
            for j in range(k, n + 1):
                m[i][j] -= f * m[k][j]
    x = [Fr(0)] * n
    for i in range(n - 1, -1, -1):
        x[i] = (m[i][n] - sum(m[i][j] * x[j] for j in range(i + 1, n))) / m[i][i]
    return x


def _cases():
    rng = np.random.default_rng(11)
    out = []
    for n in (1, 2, 3, 5, 8):
        for s in range(3):
            a = rng.standard_normal((n, n)) * 10.0 ** rng.integers(-3, 3)
            out.append((n, s, a))
    # ties in the pivot search, a zero pivot, tiny and huge entries
    out.append((4, 90, np.array([[1.0, 2, 3, 4], [-1, 2, 0, 1], [1, -2, 5, 1], [0.5, 1, 1, 2]])))
    out.append((3, 91, np.array([[0.0, 1, 2], [0, 3, 4], [0, 5, 7]])))
    out.append((3, 92, np.array([[1e-6, 3e4, 2], [7e-8, 1, 4e3], [2, 5e-5, 7]])))
    return out


@pytest.mark.parametrize("mode", ["f64", "f32", "f16mixed", "f16strict", "bf16mixed"])
@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"n{c[0]}s{c[1]}")
def test_lu_bitwise_vs_rational_replay(orc, mode, case):
    n, _, a = case
    tf = {"f64": orc.F64, "f32": orc.F32, "f16mixed": orc.F16, "f16strict": orc.F16,
          "bf16mixed": orc.BF16}[mode]
    lu_mode = {"f64": orc.LU_F64, "f32": orc.LU_F32, "f16mixed": orc.LU_F16MIXED,
               "f16strict": orc.LU_F16STRICT, "bf16mixed": orc.LU_BF16MIXED}[mode]
    at = np.ascontiguousarray(a.T)
    af, anorm, st = orc.downcast(at, tf)
    assert st == 0
    init_fmt = {"f64": "f64", "f32": "f32", "f16mixed": "f16", "f16strict": "f16",
                "bf16mixed": "bf16"}[mode]
    ra = [[rnd(Fr(float(a[i, j])), init_fmt) for j in range(n)] for i in range(n)]
    assert all(Fr(float(af[i, j])) == ra[i][j] for i in range(n) for j in range(n))
    lu, ipiv, info, st = orc.lu(af, lu_mode)
    rl, rp, rinfo = replay_lu(ra, mode)
    assert list(ipiv) == rp and info == rinfo
    for i in range(n):
        for j in range(n):
            assert Fr(float(lu[i, j])) == rl[i][j], (i, j)
    if info == 0:
        ts, fmt = ((orc.TS_F64, "f64") if mode == "f64" else (orc.TS_F32, "f32"))
        y0 = np.linspace(-1.0, 2.0, n)
        y = orc.trsv_lu(lu, y0, ts)
        ry = replay_trsv(rl, [Fr(float(v)) for v in y0], fmt)
        assert all(Fr(float(y[i])) == ry[i] for i in range(n))


@pytest.mark.parametrize("case", _cases()[:-2], ids=lambda c: f"n{c[0]}s{c[1]}")
def test_f64_solve_vs_exact_rational(orc, case):
    n, _, a = case
    rng = np.random.default_rng(5)
    b = rng.standard_normal(n)
    x, info, st = orc.solve_f64(np.ascontiguousarray(a.T), b)
    assert st == 0 and info == 0
    xe = exact_solve([[Fr(float(v)) for v in row] for row in a], [Fr(float(v)) for v in b])
    xe = np.array([float(v) for v in xe])
    kappa = np.linalg.cond(a, np.inf)
    err = np.abs(x - xe).max() / np.abs(xe).max()
    assert err <= 8 * n * kappa * 2.0**-53


def test_rnd_helper_agrees_with_numpy_casts():
    rng = np.random.default_rng(3)
    for v in rng.standard_normal(300) * 10.0 ** rng.integers(-8, 5, 300):
        assert float(rnd(Fr(float(v)), "f32")) == float(np.float32(v))
        assert float(rnd(Fr(float(v)), "f16")) == float(np.float16(v))
    assert rnd(Fr(65520), "f16") == INF and rnd(Fr(65519), "f16") == 65504
    assert math.isinf(float(rnd(Fr(2) ** 128, "f32")))
