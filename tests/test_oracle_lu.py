"""Pins of the oracle's LU against LAPACK and against the paper's
componentwise backward-error bound (section "Estimates for ||M_IR||",
eq. comperr: |L U - A_F| <= gamma_3N(u_F) |L| |U|)."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2311_14616_amd import inputs as I


def _unpack(lu):
    n = lu.shape[0]
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    return L, U


def _perm_from_ipiv(ipiv):
    n = len(ipiv)
    perm = np.arange(n)
    for k, p in enumerate(ipiv):
        perm[[k, p]] = perm[[p, k]]
    return perm


def _gamma(k, u):
    return k * u / (1 - k * u)


@pytest.mark.parametrize("n,seed", [(40, 1), (129, 2), (300, 3)])
def test_f64_lu_matches_lapack_dgetrf(orc, n, seed):
    at = I.random_dense(n, seed)
    a = at.T
    af, _, _ = orc.downcast(at, orc.F64)
    lu, ipiv, info, st = orc.lu(af, orc.LU_F64)
    lu_ref, piv_ref = sla.lu_factor(a)
    assert info == 0 and np.array_equal(ipiv, piv_ref)
    assert np.abs(lu - lu_ref).max() <= 1e3 * n * 2.0**-53 * np.abs(lu_ref).max()


@pytest.mark.parametrize("n,seed", [(40, 4), (200, 5)])
def test_f32_lu_matches_lapack_sgetrf(orc, n, seed):
    at = I.random_dense(n, seed)
    a32 = at.T.astype(np.float32)
    af, _, _ = orc.downcast(at, orc.F32)
    assert np.array_equal(af, a32.astype(np.float64))
    lu, ipiv, info, st = orc.lu(af, orc.LU_F32)
    lu_ref, piv_ref = sla.lu_factor(a32)
    assert lu_ref.dtype == np.float32
    assert info == 0 and np.array_equal(ipiv, piv_ref)
    assert np.abs(lu - lu_ref).max() <= 1e3 * n * 2.0**-24 * np.abs(lu_ref).max()


@pytest.mark.parametrize("mode,u,n", [("f64", 2.0**-53, 300), ("f32", 2.0**-24, 300),
                                      ("f16mixed", 2.0**-11, 200), ("f16strict", 2.0**-11, 100)])
@pytest.mark.parametrize("kind", ["gauss", "gmat10"])
def test_componentwise_backward_error_bound(orc, mode, u, n, kind):
    at = I.random_dense(n, 7) if kind == "gauss" else I.gmat_operator(n, 10.0)
    tf = {"f64": orc.F64, "f32": orc.F32}.get(mode, orc.F16)
    lu_mode = {"f64": orc.LU_F64, "f32": orc.LU_F32, "f16mixed": orc.LU_F16MIXED,
               "f16strict": orc.LU_F16STRICT}[mode]
    af, _, st = orc.downcast(at, tf)
    assert st == 0
    lu, ipiv, info, _ = orc.lu(af, lu_mode)
    assert info == 0
    L, U = _unpack(lu)
    pa = af[_perm_from_ipiv(ipiv)]
    lhs = np.abs(L @ U - pa)
    rhs = _gamma(3 * n, u) * (np.abs(L) @ np.abs(U))
    assert np.all(lhs <= rhs)
    # partial pivoting: every multiplier is at most one in magnitude
    assert np.abs(np.tril(lu, -1)).max() <= 1.0


def test_f16_factors_are_binary16_numbers(orc):
    n = 64
    at = I.gmat_operator(n, 100.0)
    af, _, _ = orc.downcast(at, orc.F16)
    for mode in (orc.LU_F16MIXED, orc.LU_F16STRICT):
        lu, ipiv, info, _ = orc.lu(af, mode)
        assert np.array_equal(lu, lu.astype(np.float16).astype(np.float64))


def test_zero_column_reports_first_zero_pivot(orc):
    n = 6
    a = I.random_dense(n, 3).T.copy()
    a[:, 2] = 0.0
    af, _, _ = orc.downcast(np.ascontiguousarray(a.T), orc.F64)
    _, ipiv, info, st = orc.lu(af, orc.LU_F64)
    assert info == 3 and st == orc.SINGULAR


def test_downcast_errors(orc):
    at = I.gmat_operator(8, 1.0)
    bad = at.copy()
    bad[3, 2] = np.nan
    assert orc.downcast(bad, orc.F32)[2] == orc.ERR_NONFINITE
    big = at * 1e5
    assert orc.downcast(big, orc.F16)[2] == orc.ERR_RANGE
    assert orc.downcast(big, orc.F32)[2] == 0


def test_anorm_is_max_row_sum(orc):
    at = I.random_dense(50, 9)
    _, anorm, _ = orc.downcast(at, orc.F32)
    assert anorm == pytest.approx(np.abs(at.T).sum(1).max(), rel=1e-15)


@pytest.mark.parametrize("kind,n,alpha", [("gauss", 700, 0.0), ("gmat", 1300, 10.0),
                                          ("gmat", 800, 1.0)])
def test_f16mixed_backward_error_with_underflow(orc, kind, n, alpha):
    # binary16 factors, binary32 updates: one binary16 rounding per L and U
    # entry (relative u_h, or absolute 2^-25 in the subnormal range) plus the
    # binary32 update errors, valid at any n:
    #   |L U - P A_F| <= (3 u_h + gamma_3n(u_s)) |L||U| + 2^-24 (1 + max|u_kk|)
    at = I.random_dense(n, 5) if kind == "gauss" else I.gmat_operator(n, alpha)
    af, _, _ = orc.downcast(at, orc.F16)
    lu, ipiv, info, _ = orc.lu(af, orc.LU_F16MIXED)
    assert info == 0
    L, U = _unpack(lu)
    lhs = np.abs(L @ U - af[_perm_from_ipiv(ipiv)])
    rhs = (3 * 2.0**-11 + _gamma(3 * n, 2.0**-24)) * (np.abs(L) @ np.abs(U)) \
        + 2.0**-24 * (1 + np.abs(np.diag(U)).max())
    assert np.all(lhs <= rhs)
