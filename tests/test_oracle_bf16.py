"""Pins of the oracle's bfloat16 arithmetic (the 16-bit format with the
binary32 exponent range and an 8-bit significand, section "Half Precision"):

* the rounding operator fl_b against torch's independent float32 -> bfloat16
  conversion (round to nearest, ties to even) on every bfloat16 value, every
  midpoint and its neighbours, random and extreme values;
* binary64 inputs against an exact rational rounding from the definition;
* the bfloat16 LU (bf16mixed) against its componentwise backward-error bound
  at any n, its factors being bfloat16 numbers;
* the refinement's contraction: each residual at most
  ||I - A (P^T L U)^{-1}||_inf times the previous one plus rounding, the
  operator norm computed independently in binary64 from the factors.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I

torch = pytest.importorskip("torch")


def _bf16_to_f64(bits_u16):
    b = torch.from_numpy(bits_u16.astype(np.int16)).view(torch.bfloat16)
    return b.to(torch.float64).numpy()


def _all_bf16_values():
    v = _bf16_to_f64(np.arange(0, 1 << 16, dtype=np.uint32).astype(np.uint16))
    return v[np.isfinite(v)]


def _torch_round(x64):
    """float32-exact inputs -> bfloat16 by torch (RNE), back to float64."""
    t = torch.from_numpy(np.asarray(x64, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def test_bf16_values_are_fixed_points(orc):
    v = _all_bf16_values()
    assert np.array_equal(orc.fl_b(v).view(np.uint64), v.view(np.uint64))


def test_midpoints_and_neighbours_match_torch(orc):
    v = np.unique(_all_bf16_values())
    mids = (v[:-1] + v[1:]) / 2                       # exact in binary32 too
    m32 = mids.astype(np.float32).astype(np.float64)
    assert np.array_equal(m32, mids)
    nb = np.concatenate([np.nextafter(mids.astype(np.float32), np.float32(np.inf)),
                         np.nextafter(mids.astype(np.float32), np.float32(-np.inf))]).astype(np.float64)
    cand = np.concatenate([mids, nb])
    cand = cand[np.isfinite(cand)]
    assert np.array_equal(orc.fl_b(cand), _torch_round(cand))


def test_random_and_extreme_float32_values_match_torch(orc):
    rng = np.random.default_rng(1)
    x = (rng.standard_normal(200000) * 10.0 ** rng.integers(-40, 38, 200000)).astype(np.float32)
    x = np.concatenate([x, np.float32([0.0, -0.0, 1e-45, 1.4e-45, 9.2e-41, 3.3895e38, 3.4e38,
                                       -3.4028235e38, 1.17549435e-38])]).astype(np.float64)
    x = x[np.isfinite(x)]
    assert np.array_equal(orc.fl_b(x), _torch_round(x))
    assert np.signbit(orc.fl_b(np.array([-0.0])))[0]
    assert np.isnan(orc.fl_b(np.array([np.nan])))[0]


def _rnd_exact(v):
    """Round a binary64 value to bfloat16 with exact rationals (p = 8,
    emin = -126, largest finite (2 - 2^-7) 2^127)."""
    if v == 0:
        return 0.0
    a = abs(Fr(v))
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fr(2) ** e > a:
        e -= 1
    while Fr(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    q = Fr(2) ** (e - 7)
    m = a / q
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fr(1, 2) or (rem == Fr(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * q
    if r > (2 - Fr(2) ** -7) * Fr(2) ** 127:
        return float("inf") if v > 0 else float("-inf")
    return float(r) if v > 0 else -float(r)


def test_binary64_inputs_round_once(orc):
    # binary64 values between float32 neighbours of a bfloat16 midpoint:
    # rounding through binary32 first would be wrong for some of them
    rng = np.random.default_rng(2)
    v = np.unique(_all_bf16_values())
    v = v[(np.abs(v) > 1e-30) & (np.abs(v) < 1e30)]
    mids = (v[:-1] + v[1:]) / 2
    pick = mids[rng.integers(0, mids.size, 3000)]
    d = np.abs(pick) * 2.0**-40
    cand = np.concatenate([pick + d, pick - d, rng.standard_normal(3000) * 10.0 ** rng.integers(-30, 30, 3000)])
    ref = np.array([_rnd_exact(float(c)) for c in cand])
    assert np.array_equal(orc.fl_b(cand), ref)


def _unpack(lu):
    L = np.tril(lu, -1) + np.eye(lu.shape[0])
    return L, np.triu(lu)


def _perm_from_ipiv(ipiv):
    perm = np.arange(len(ipiv))
    for k, p in enumerate(ipiv):
        perm[[k, p]] = perm[[p, k]]
    return perm


def _gamma(k, u):
    return k * u / (1 - k * u)


@pytest.mark.parametrize("kind,n,alpha", [("gauss", 600, 0.0), ("gmat", 900, 10.0), ("gmat", 700, 1.0)])
def test_bf16mixed_backward_error_bound(orc, kind, n, alpha):
    # bfloat16 factors, binary32 updates: one bfloat16 rounding per L and U
    # entry plus the binary32 update errors, valid at any n:
    #   |L U - P A_F| <= (3 u_b + gamma_3n(u_s)) |L||U|,   u_b = 2^-8
    at = I.random_dense(n, 5) if kind == "gauss" else I.gmat_operator(n, alpha)
    af, _, st = orc.downcast(at, orc.BF16)
    assert st == 0 and np.array_equal(orc.fl_b(af), af)
    lu, ipiv, info, _ = orc.lu(af, orc.LU_BF16MIXED)
    assert info == 0
    assert np.array_equal(orc.fl_b(lu), lu)            # L and U hold bfloat16 numbers
    L, U = _unpack(lu)
    lhs = np.abs(L @ U - af[_perm_from_ipiv(ipiv)])
    rhs = (3 * 2.0**-8 + _gamma(3 * n, 2.0**-24)) * (np.abs(L) @ np.abs(U))
    assert np.all(lhs <= rhs)
    assert np.abs(np.tril(lu, -1)).max() <= 1.0


@pytest.mark.parametrize("n,alpha", [(300, 1.0), (400, 10.0)])
def test_refinement_contracts_at_the_operator_rate(orc, n, alpha):
    # r_{k+1} = (I - A M^{-1}) r_k + rounding, M = P^T L U: with TR = TW = F64
    # the residual falls at least by rho = ||I - A M^{-1}||_inf per step
    # (up to the bfloat16 rounding of the scaled residual, a relative 2^-8
    # of r_k through A M^{-1}), until it reaches the binary64 floor
    at = I.gmat_operator(n, alpha)
    A = at.T
    b = I.rhs_ones(at)
    af, _, _ = orc.downcast(at, orc.BF16)
    lu, ipiv, info, _ = orc.lu(af, orc.LU_BF16MIXED)
    L, U = _unpack(lu)
    perm = _perm_from_ipiv(ipiv)
    M = np.empty_like(A)
    M[perm] = L @ U                                   # P^T L U
    R = np.eye(n) - A @ np.linalg.inv(M)
    rho = np.abs(R).sum(1).max()
    AMi = np.abs(A @ np.linalg.inv(M)).sum(1).max()
    assert rho < 0.5
    r = orc.ir_solve(at, b, orc.BF16, tol_rel=1e-14, litmax=30)
    assert r.stop_name == "converged"
    floor = 64 * n * 2.0**-53 * np.abs(A).sum(1).max() * np.abs(r.x).max()
    for k in range(1, r.n_iter + 1):
        bound = (rho + 2.0**-8 * AMi) * r.rhist[k - 1] + floor
        assert r.rhist[k] <= bound, (k, r.rhist[k], bound)
