"""Pins of the oracle's refinement loop (Algorithm IR, low-precision solve of
eqs. vdlow/promotevd, residual in TR by eq. xferrule, termination rules of
section "Terminating the while loop") against the paper's printed sessions,
closed forms, special cases and metamorphic relations."""
import json
import os

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def test_config0_plain_ir(orc):
    n = 512
    at = I.gmat_operator(n, 1.0)
    b = I.rhs_ones(at)
    r = orc.ir_solve(at, b, orc.F32, tol_rel=1e-14, litmax=20)
    assert r.status == 0 and r.stop_name == "converged"
    assert r.rhist[-1] <= 1e-14 * r.rhist[0]
    assert r.bwd_err <= 1e-14
    assert 2 <= r.n_iter <= 5
    assert np.abs(r.x - 1).max() <= 1e-14
    assert len(r.rhist) == r.n_iter + 1 and len(r.dhist) == r.n_iter


def test_all_double_first_correction_is_plain_lu_solve(orc):
    # TF = TW = TR = F64: the first correction is the binary64 LU solve (the
    # power-of-two scaling commutes with rounding).
    n = 200
    at = I.random_dense(n, 21)
    b = np.random.default_rng(2).standard_normal(n) * 3.7
    r = orc.ir_solve(at, b, orc.F64, litmax=1)
    x, info, st = orc.solve_f64(at, b)
    assert r.n_iter == 1 and np.array_equal(r.x, x)


@pytest.mark.parametrize("tf", ["F32", "F16"])
def test_power_of_two_scaling_of_b(orc, tf):
    n = 300
    at = I.gmat_operator(n, 10.0)
    b = I.rhs_ones(at)
    t = getattr(orc, tf)
    r0 = orc.ir_solve(at, b, t, tol_rel=1e-14, litmax=20)
    for k in (-40, 7, 300):
        rk = orc.ir_solve(at, b * 2.0**k, t, tol_rel=1e-14, litmax=20)
        assert rk.n_iter == r0.n_iter and rk.stop == r0.stop
        assert np.array_equal(rk.x, r0.x * 2.0**k)


def test_row_permutation_gives_same_solution(orc):
    n = 257
    a = I.gmat_operator(n, 100.0).T
    b = I.rhs_ones(np.ascontiguousarray(a.T))
    perm = np.random.default_rng(8).permutation(n)
    r0 = orc.ir_solve(np.ascontiguousarray(a.T), b, orc.F32, tol_rel=1e-14, litmax=20)
    r1 = orc.ir_solve(np.ascontiguousarray(a[perm].T), b[perm], orc.F32, tol_rel=1e-14, litmax=20)
    assert r1.n_iter == r0.n_iter and np.array_equal(r0.x, r1.x)


@pytest.mark.slow
def test_paper_double_single_history(orc):
    g = GOLD["E4_double_single"]
    n = g["n"]
    at = I.gmat_operator(n, g["alpha"], grid="endpoint")
    b = I.rhs_ones(at)
    r = orc.ir_solve(at, b, orc.F32)          # the paper's default termination
    rh = np.array(g["rhist"])
    assert r.n_iter == len(rh) - 1 == 5
    assert r.rhist[0] == 1.0
    assert 0.5 < r.rhist[1] / rh[1] < 2.0     # first FP32 solve: same error level
    assert r.rhist[-1] <= 4 * 2.0**-52
    assert 0.5 < r.dhist[0] / g["dhist"][0] < 2.0
    err = np.abs(r.x - 1).max()
    assert err <= 4 * g["ir_error_inf"]
    # plain binary64 LU solve error, printed next to it
    x, _, _ = orc.solve_f64(at, b)
    assert 0.1 < np.abs(x - 1).max() / g["lu_error_inf"] < 10.0


@pytest.mark.slow
def test_paper_extended_residual_example(orc):
    g = GOLD["E5_extended_residual"]
    n, alpha = g["n"], g["alpha"]
    ad = I.gmat_operator(n, alpha, grid="endpoint")
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    bd = 1.0 - alpha * x * (1.0 - x) * 0.5
    a32, b32 = ad.astype(np.float32), bd.astype(np.float32)
    r = orc.ir_solve(a32, b32, orc.F32, tr=orc.F64)
    assert r.stop_name == "dstagnated" and r.n_iter == len(g["rhist"]) - 1
    assert r.rhist[0] == pytest.approx(g["rhist"][0], rel=1e-5)
    assert r.rhist[-1] == pytest.approx(g["rhist"][-1], rel=0.05)
    xp, info, _ = orc.solve_f64(a32, b32)
    assert np.abs(xp - 1).max() == pytest.approx(g["promoted_minus_ones_inf"], rel=1e-4)
    assert np.abs(r.x - xp).max() == pytest.approx(g["sol_minus_promoted_inf"], rel=0.02)
    # eq. irterm: forward error of the promoted problem <= 4 (N+1) kappa u_r + u_w
    kappa = g["cond_inf"]
    ferr = np.abs(r.x - xp).max() / np.abs(xp).max()
    assert ferr <= 4 * (n + 1) * kappa * 2.0**-53 + 2.0**-23


@pytest.mark.parametrize("rmax,key", [(0.5, "rhist_rmax_0_5"), (0.1, "rhist_rmax_0_1")])
def test_paper_stagnation_example(orc, rmax, key):
    g = GOLD["E11_stagnation"]
    n = g["n"]
    at = I.gmat_operator(n, g["alpha"], grid="endpoint")
    r = orc.ir_solve(at, np.ones(n), orc.F32, Rmax=rmax)
    rh = np.array(g[key])
    assert r.stop_name == "stagnated"
    assert len(r.rhist) == len(rh)
    assert 0.3 < r.rhist[-1] / rh[-1] < 3.0       # stall level ~ 6e-12
    assert r.rhist[-1] >= rmax * r.rhist[-2]


def test_stagnation_level_matches_theory(orc):
    # eq. stagterm: the stall is O(gamma_N(u_w) (||A|| ||x|| + ||b||))
    n = 512
    at = I.gmat_operator(n, 799.0)
    b = np.ones(n)
    r = orc.ir_solve(at, b, orc.F32, tol_rel=1e-16, litmax=20)
    assert r.stop_name == "stagnated"
    xi = n * 2.0**-53 * (r.anorm * r.xnorm + r.bnorm)
    assert r.rhist[-1] <= xi


def test_half_factorization_converges_on_well_conditioned(orc):
    n = 256
    for alpha in (1.0, 10.0, 100.0):
        at = I.gmat_operator(n, alpha)
        b = I.rhs_ones(at)
        r = orc.ir_solve(at, b, orc.F16, tol_rel=1e-14, litmax=20)
        assert r.stop_name == "converged" and r.bwd_err <= 1e-14
        r32 = orc.ir_solve(at, b, orc.F32, tol_rel=1e-14, litmax=20)
        assert r.n_iter >= r32.n_iter


def test_backward_error_termination(orc):
    n = 300
    at = I.gmat_operator(n, 10.0)
    b = I.rhs_ones(at)
    r = orc.ir_solve(at, b, orc.F32, residterm=False)
    assert r.stop_name in ("converged", "stagnated")
    r2 = orc.ir_solve(at, b, orc.F32, residterm=True)
    assert r.n_iter <= r2.n_iter


def test_zero_rhs_and_error_paths(orc):
    n = 16
    at = I.gmat_operator(n, 1.0)
    r = orc.ir_solve(at, np.zeros(n), orc.F32)
    assert r.status == 0 and r.n_iter == 0 and np.all(r.x == 0)
    b = I.rhs_ones(at)
    b[3] = np.inf
    assert orc.ir_solve(at, b, orc.F32).status == orc.ERR_NONFINITE
    sing = at.copy()
    sing[4] = 0.0      # column 4 of A is zero
    r = orc.ir_solve(sing, I.rhs_ones(at), orc.F32)
    assert r.status == orc.SINGULAR and r.info == 5
    assert orc.ir_solve(at * 1e6, I.rhs_ones(at), orc.F16).status == orc.ERR_RANGE


def test_tiny_rhs_is_scaled_before_half_downcast(orc):
    # unscaled, 1e-10 * b underflows in binary16 (smallest subnormal 6e-8)
    n = 128
    at = I.gmat_operator(n, 1.0)
    b = I.rhs_ones(at) * 1e-10
    r = orc.ir_solve(at, b, orc.F16, tol_rel=1e-14, litmax=20)
    assert r.stop_name == "converged" and np.abs(r.x - 1e-10).max() <= 1e-23


@pytest.mark.parametrize("tf", ["F32", "F16"])
def test_onthefly_first_correction_is_binary64_solve_with_tf_factors(orc, tf):
    """MPS (the onthefly solve): the first correction is b pushed through the
    TF factors in binary64 arithmetic, without rounding b to TF.  Pinned
    against scipy's triangular solves (LAPACK trtrs) on the same factors."""
    sl = pytest.importorskip("scipy.linalg")
    n = 160
    at = I.random_dense(n, 31, diag_shift=4.0 * np.sqrt(n))
    b = np.random.default_rng(4).standard_normal(n)
    T = getattr(orc, tf)
    r = orc.ir_solve(at, b, T, litmax=1, onthefly=True)
    af, _, _ = orc.downcast(at, T)
    lu, ipiv, info, _ = orc.lu(af, {"F32": orc.LU_F32, "F16": orc.LU_F16MIXED}[tf])
    y = b.copy()
    for k, p in enumerate(ipiv):
        y[[k, p]] = y[[p, k]]
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    ref = sl.solve_triangular(U, sl.solve_triangular(L, y, lower=True, unit_diagonal=True))
    assert r.n_iter == 1
    assert np.abs(r.x - ref).max() <= 1e-12 * np.abs(ref).max()
    # the low-precision solve rounds b to TF first: visibly different for F16
    r_lps = orc.ir_solve(at, b, T, litmax=1)
    if tf == "F16":
        assert np.abs(r_lps.x - ref).max() > 1e3 * np.abs(r.x - ref).max()


def test_onthefly_equals_lps_when_tf_is_tw(orc):
    n = 120
    at = I.random_dense(n, 8)
    b = np.random.default_rng(9).standard_normal(n)
    a = orc.ir_solve(at, b, orc.F64, litmax=3)
    c = orc.ir_solve(at, b, orc.F64, litmax=3, onthefly=True)
    assert np.array_equal(a.x, c.x) and a.n_iter == c.n_iter


def test_onthefly_half_converges_at_least_as_fast(orc):
    """On the paper's operator with alpha = 10 the half-precision MPS solve
    needs no more corrections than LPS (the residual is not rounded to FP16)."""
    n = 1024
    at = I.gmat_operator(n, 10.0)
    b = I.rhs_ones(at)
    lps = orc.ir_solve(at, b, orc.F16, tol_rel=1e-14, litmax=20)
    mps = orc.ir_solve(at, b, orc.F16, tol_rel=1e-14, litmax=20, onthefly=True)
    assert lps.stop_name == mps.stop_name == "converged"
    assert mps.n_iter <= lps.n_iter
    assert mps.bwd_err <= 1e-14
