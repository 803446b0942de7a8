"""Pins of the BiCGSTAB-IR oracle (section "Krylov-IR"): the inner BiCGSTAB
against scipy's independent implementation (same start, same shadow vector)
iterate by iterate, finite termination on small systems, its recurrence
residual against the true one, the identity and exact preconditioners, and
the outer loop against the paper's claim that a Krylov correction recovers
the residual where half-precision IR does not."""
import numpy as np
import pytest
from scipy.sparse.linalg import bicgstab as sp_bicgstab

from paper_2311_14616_amd import inputs as I


@pytest.fixture(scope="module")
def B():
    from oracle import bicgstab_ir
    return bicgstab_ir


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_iterates_match_scipy(B, k):
    rng = np.random.default_rng(3)
    n = 12
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    rhs = rng.standard_normal(n)
    d, kk, est = B.bicgstab(lambda v: A @ v, rhs, k, 0.0)
    xs, _ = sp_bicgstab(A, rhs, x0=np.zeros(n), rtol=1e-300, atol=0.0, maxiter=k)
    assert kk == k
    assert np.abs(d - xs).max() <= 1e-14 * np.abs(xs).max()
    # the recurrence residual is the true residual of the iterate
    assert abs(est - np.linalg.norm(rhs - A @ d)) <= 1e-12 * np.linalg.norm(rhs)


def test_identity_operator_converges_in_one_step(B):
    rhs = np.random.default_rng(1).standard_normal(20)
    d, k, est = B.bicgstab(lambda v: v.copy(), rhs, 10, 1e-12)
    assert k == 1 and est == 0.0
    assert np.abs(d - rhs).max() <= 1e-15 * np.abs(rhs).max()


def test_small_system_solved(B):
    rng = np.random.default_rng(2)
    n = 6
    A = rng.standard_normal((n, n)) + 5 * np.eye(n)
    rhs = rng.standard_normal(n)
    d, k, _ = B.bicgstab(lambda v: A @ v, rhs, 30, 1e-14)
    assert k <= 30
    assert np.abs(d - np.linalg.solve(A, rhs)).max() <= 1e-12 * np.abs(np.linalg.solve(A, rhs)).max()


def test_exact_preconditioner_one_step(B, orc):
    n = 200
    at = I.gmat_operator(n, 1.0)
    b = I.rhs_ones(at)
    r = B.bicgstab_ir_solve(at, b, orc.F64, tol_rel=1e-14, litmax=5)
    assert r.khist[0] == 1 and r.stop == 0
    assert np.abs(r.x - 1).max() <= 1e-13


def test_matches_ir_where_ir_works(B, orc):
    n = 300
    at = I.gmat_operator(n, 1.0)
    b = I.rhs_ones(at)
    g = B.bicgstab_ir_solve(at, b, orc.F32, tol_rel=1e-14, litmax=20)
    ir = orc.ir_solve(at, b, orc.F32, tol_rel=1e-14, litmax=20)
    assert g.stop == 0 and ir.stop_name == "converged"
    assert np.abs(g.x - ir.x).max() <= 1e-13
    assert g.n_iter <= ir.n_iter
    assert len(g.khist) == g.n_iter and all(1 <= k <= 10 for k in g.khist)


@pytest.mark.parametrize("tf", ["f16", "bf16"])
def test_recovers_where_half_ir_fails(B, orc, tf):
    # the ill-conditioned example (I - 799 Gmat): 16-bit IR stalls,
    # BiCGSTAB-IR meets the 1e-14 rule
    n = 512
    at = I.gmat_operator(n, 799.0)
    b = I.rhs_ones(at)
    T = orc.F16 if tf == "f16" else orc.BF16
    ir = orc.ir_solve(at, b, T, tol_rel=1e-14, litmax=20)
    g = B.bicgstab_ir_solve(at, b, T, tol_rel=1e-14, litmax=20)
    assert ir.stop_name != "converged"
    assert g.stop == 0 and g.relres <= 1e-14
