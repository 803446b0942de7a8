"""Pins of the GMRES-IR oracle (sections "Krylov-IR" and "GMRES-IR"): the
inner GMRES against properties that fix it independently of its own code
(exact termination, the minimal-residual property over the Krylov space
built explicitly, the exact preconditioner), and the outer loop against the
paper's claim that GMRES-IR recovers the residual where half-precision IR
does not."""
import json
import os

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


@pytest.fixture(scope="module")
def G():
    from oracle import gmres_ir
    return gmres_ir


def test_givens_zeroes_second_entry(G):
    for a, b in [(3.0, 4.0), (-1.0, 2.0), (5.0, 0.0), (0.0, -2.0)]:
        c, s = G.givens(a, b)
        assert abs(c * c + s * s - 1.0) <= 1e-15
        assert abs(-s * a + c * b) <= 1e-15
        assert abs(c * a + s * b - np.hypot(a, b)) <= 1e-14


def test_identity_operator_converges_in_one_step(G):
    rng = np.random.default_rng(1)
    rhs = rng.standard_normal(20)
    d, k, est = G.gmres(lambda v: v.copy(), rhs, 10, 1e-12)
    assert k == 1
    assert np.abs(d - rhs).max() <= 1e-14 * np.abs(rhs).max()


def test_full_krylov_space_solves_exactly(G):
    # m = n steps on a nonsingular 8 x 8 system: the exact solution
    rng = np.random.default_rng(2)
    n = 8
    A = rng.standard_normal((n, n)) + 4 * np.eye(n)
    rhs = rng.standard_normal(n)
    d, k, _ = G.gmres(lambda v: A @ v, rhs, n, 1e-15)
    assert k <= n
    assert np.abs(A @ d - rhs).max() <= 1e-12 * np.abs(rhs).max()
    assert np.abs(d - np.linalg.solve(A, rhs)).max() <= 1e-11


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_minimal_residual_over_explicit_krylov_space(G, k):
    # after k steps GMRES minimises ||rhs - A d||_2 over span{rhs, ..., A^{k-1} rhs}:
    # compare with the least-squares minimiser over the explicit power basis
    rng = np.random.default_rng(3)
    n = 12
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)
    rhs = rng.standard_normal(n)
    d, kk, est = G.gmres(lambda v: A @ v, rhs, k, 0.0)
    assert kk == k
    K = np.empty((n, k))
    K[:, 0] = rhs
    for j in range(1, k):
        K[:, j] = A @ K[:, j - 1]
    c, *_ = np.linalg.lstsq(A @ K, rhs, rcond=None)
    d_ls = K @ c
    assert np.abs(d - d_ls).max() <= 1e-10 * np.abs(d_ls).max()
    # the estimate |g_k| is the true residual norm of the iterate
    assert abs(est - np.linalg.norm(rhs - A @ d)) <= 1e-10 * np.linalg.norm(rhs)


def test_exact_preconditioner_one_krylov_step(G, orc):
    # TF = F64: P A = I up to rounding, one GMRES step per correction and
    # the first correction already solves the system
    n = 200
    at = I.gmat_operator(n, 1.0)
    b = I.rhs_ones(at)
    r = G.gmres_ir_solve(at, b, orc.F64, tol_rel=1e-14, litmax=5)
    assert r.khist[0] == 1
    assert r.rhist[1] <= 1e-14 * r.rhist[0]
    assert np.abs(r.x - 1).max() <= 1e-13


def test_matches_ir_where_ir_works(G, orc):
    # well conditioned, TF = F32: both converge to the 1e-14 rule, the
    # solutions agree to the refinement's accuracy
    n = 300
    at = I.gmat_operator(n, 1.0)
    b = I.rhs_ones(at)
    g = G.gmres_ir_solve(at, b, orc.F32, tol_rel=1e-14, litmax=20)
    ir = orc.ir_solve(at, b, orc.F32, tol_rel=1e-14, litmax=20)
    assert g.stop == 0 and ir.stop_name == "converged"
    assert np.abs(g.x - ir.x).max() <= 1e-13
    assert g.n_iter <= ir.n_iter
    assert len(g.khist) == g.n_iter and all(1 <= k <= 10 for k in g.khist)


def test_recovers_where_half_ir_fails(G, orc):
    # the paper's ill-conditioned example (I - 799 Gmat) with a binary16
    # factorization: IR does not reach the tolerance, GMRES-IR does
    n = 512
    at = I.gmat_operator(n, 799.0)
    b = I.rhs_ones(at)
    ir = orc.ir_solve(at, b, orc.F16, tol_rel=1e-14, litmax=20)
    g = G.gmres_ir_solve(at, b, orc.F16, tol_rel=1e-14, litmax=20)
    assert ir.stop_name != "converged"
    assert g.stop == 0 and g.relres <= 1e-14
    assert max(g.khist) >= 3


def test_printed_statistics_session(G, orc):
    """The printed mpglu session (tests/golden E_gmres_stats): N = 4096,
    A = I - Gmat, FP32 factors, TW = TR = F64.  The same initial residual to
    the printed six digits (it fixes the grid), two corrections as printed,
    the residual after the first within a factor 2 of the printed 7.48e-14 and
    the final one at the binary64 floor near the printed 1.44e-15 (both are
    rounding-level quantities, so only their size is fixed), each correction
    within one Krylov step of the printed count.  The printed session stops
    at 1.44e-15, above eps(F64) ||b||, so the 1e-14 rule of the workloads
    stands in for the package's stopping test here."""
    g = GOLD["E_gmres_stats"]
    n = g["n"]
    at = I.gmat_operator(n, g["alpha"])
    b = I.rhs_ones(at)
    r = G.gmres_ir_solve(at, b, orc.F32, tol_rel=1e-14, litmax=10)
    assert r.stop == 0
    assert abs(r.rhist[0] - g["rhist"][0]) <= 5e-7
    assert r.n_iter == len(g["khist"]) == 2
    assert 0.5 <= r.rhist[1] / g["rhist"][1] <= 2.0
    assert 0.5 <= r.rhist[2] / g["rhist"][2] <= 2.0
    assert all(abs(k - kp) <= 1 for k, kp in zip(r.khist, g["khist"]))
