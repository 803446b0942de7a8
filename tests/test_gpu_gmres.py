"""GPU parity of GMRES-IR (sections "Krylov-IR" and "GMRES-IR") against the
oracle in oracle/gmres_ir.py, through the C ABI.

GMRES-IR reaches the binary64 residual floor after one or two corrections,
so the outer stop is usually decided by residuals of a few ulps of ||b||,
which the two sides (different summation orders, factors equal only up to
binary32 rounding) do not share.  The bars therefore compare what rounding
does not decide:
  - the first residual (x = 0) bit for bit;
  - the first correction's GMRES iteration count within +-1, and every
    common correction's count within +-1 and within the basis;
  - the residual after the first correction within a factor 3 of the
    oracle's when it lies above the floor (a truncated basis);
  - outer iteration counts within +-1 and both final residuals at the
    floor (<= 1e-13 ||b||); the same stop reason whenever the oracle's
    residual history clears the tolerance and the stagnation ratio by a
    margin (factor 3, ratio <= 0.3);
  - the solutions within the accuracy the refinement reaches (a forward
    error bounded by kappa_inf(A) times the tolerance).
"""
import sys

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"
TF = {"f64": 0, "f32": 1, "f16": 2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_14616_amd import mpir
    mpir.lib()
    return mpir


@pytest.fixture(scope="module")
def G():
    from oracle import gmres_ir
    return gmres_ir


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _operator(name, n, alpha):
    if name == "gmat":
        return I.gmat_operator(n, alpha)
    return I.random_dense(n, 17, diag_shift=2.0 * np.sqrt(n))


CASES = [("gmat", 512, 1.0, "f32", 10), ("gmat", 512, 799.0, "f16", 10),
         ("gmat", 1100, 10.0, "f16", 20), ("rand", 650, 0.0, "f16", 10),
         ("gmat", 300, 1.0, "f64", 10), ("gmat", 777, 100.0, "f16", 3),
         ("gmat", 640, 799.0, "f16", 3), ("gmat", 1100, 10.0, "f16", 3),
         ("rand", 1100, 0.0, "f16", 10), ("gmat", 4096, 1.0, "f32", 10)]

TOL = 1e-14


def _stop_has_margin(ref):
    """True when the oracle's stop does not hang on rounding: every
    intermediate residual at least 3x above the tolerance, the last at least
    3x below, and every ratio of successive residuals at most 0.3."""
    rel = np.asarray(ref.rhist) / ref.rhist[0]
    ratios = rel[2:] / rel[1:-1]
    return (ref.stop == 0 and rel[-1] <= TOL / 3 and bool(np.all(rel[1:-1] >= 3 * TOL))
            and bool(np.all(ratios <= 0.3)))


@pytest.mark.parametrize("name,n,alpha,tf,m", CASES)
def test_gmres_ir_parity(M, G, orc, name, n, alpha, tf, m):
    say(f"gmres-ir {name} n={n} alpha={alpha} tf={tf} basis={m}")
    at = _operator(name, n, alpha)
    b = I.rhs_ones(at)
    tp = M.term(tol_rel=TOL, litmax=20)
    x, rep, kh = M.gmres_ir_solve(dev(at), dev(b), TF[tf], term_parms=tp, basissize=m)
    ref = G.gmres_ir_solve(at, b, TF[tf], basissize=m, tol_rel=TOL, litmax=20)
    rg = [rep.rhist[k] / rep.rhist[0] for k in range(rep.n_iter + 1)]
    ro = list(np.asarray(ref.rhist) / ref.rhist[0])
    say(f"  gpu n_iter={rep.n_iter} stop={rep.stop} khist={kh} rhist={['%.1e' % v for v in rg]} | "
        f"oracle n_iter={ref.n_iter} stop={ref.stop} khist={[int(k) for k in ref.khist]} "
        f"rhist={['%.1e' % v for v in ro]}")
    # x = 0: the first residual is b itself
    assert rep.rhist[0] == ref.rhist[0]
    assert len(kh) == rep.n_iter and rep.n_iter >= 1
    assert abs(kh[0] - ref.khist[0]) <= 1
    for kg, ko in zip(kh, ref.khist):
        assert abs(kg - ko) <= 1 and 1 <= kg <= m
    if ro[1] >= 1e-12:
        assert 1 / 3 <= rg[1] / ro[1] <= 3
    assert abs(rep.n_iter - ref.n_iter) <= 1
    assert rg[-1] <= 1e-13 and ro[-1] <= 1e-13
    assert rep.stop in (0, 1) and ref.stop in (0, 1)
    if _stop_has_margin(ref):
        assert rep.stop == ref.stop == 0 and rg[-1] <= TOL
    xg = x.cpu().numpy()
    kappa = np.abs(at).sum(0).max() * np.abs(np.linalg.inv(at.T)).sum(1).max()
    assert np.abs(xg - ref.x).max() <= 10 * kappa * TOL * np.abs(ref.x).max()


def test_gmres_ir_exact_preconditioner_one_step(M):
    """TF = F64: P A = I up to rounding, one GMRES step per correction."""
    say("gmres-ir tf=f64 one step")
    at = I.gmat_operator(400, 1.0)
    b = I.rhs_ones(at)
    x, rep, kh = M.gmres_ir_solve(dev(at), dev(b), M.F64, term_parms=M.term(tol_rel=1e-14, litmax=5))
    assert kh[0] == 1 and rep.stop_name == "converged"
    assert np.abs(x.cpu().numpy() - 1).max() <= 1e-13


def test_gmres_ir_recovers_where_half_ir_stalls(M):
    """The ill-conditioned example (I - 799 Gmat), binary16 factors: IR stops
    short of the 1e-14 residual rule, GMRES-IR meets it."""
    say("gmres-ir vs ir, alpha=799 tf=f16")
    at = I.gmat_operator(512, 799.0)
    b = I.rhs_ones(at)
    tp = M.term(tol_rel=1e-14, litmax=20)
    f = M.Factorization(dev(at), M.F16, M.F64)
    try:
        _, rep_ir = f.ir_solve(dev(b), term_parms=tp)
        _, rep_g, kh = f.gmres_ir_solve(dev(b), term_parms=tp)
        # the workspace of a larger basis, then a smaller one again
        _, rep_g2, kh2 = f.gmres_ir_solve(dev(b), term_parms=tp, basissize=30)
        _, rep_g3, kh3 = f.gmres_ir_solve(dev(b), term_parms=tp, basissize=10)
    finally:
        f.destroy()
    assert rep_ir.stop_name != "converged"
    assert rep_g.stop_name == "converged" and rep_g.relres <= 1e-14
    assert rep_g2.stop_name == "converged" and max(kh2) <= 30
    assert (rep_g3.n_iter, kh3) == (rep_g.n_iter, kh)
    assert list(rep_g3.rhist[:rep_g3.n_hist]) == list(rep_g.rhist[:rep_g.n_hist])


def test_gmres_ir_zero_rhs(M):
    say("gmres-ir zero rhs")
    at = I.gmat_operator(64, 1.0)
    x, rep, kh = M.gmres_ir_solve(dev(at), dev(np.zeros(64)), M.F32)
    assert rep.n_iter == 0 and rep.stop_name == "converged" and kh == []
    assert torch.all(x == 0)


def test_gmres_ir_argument_errors(M):
    say("gmres-ir argument errors")
    at = I.gmat_operator(64, 1.0)
    b = I.rhs_ones(at)
    f = M.Factorization(dev(at), M.F32, M.F64)
    try:
        for m in (0, 65):
            with pytest.raises(M.MpirError):
                f.gmres_ir_solve(dev(b), basissize=m)
    finally:
        f.destroy()
    # TR must be F64
    f = M.Factorization(dev(at.astype(np.float32)), M.F16, M.F32)
    try:
        with pytest.raises(M.MpirError):
            f.gmres_ir_solve(dev(b.astype(np.float32)))
    finally:
        f.destroy()


def test_gmres_ir_full_size(M):
    """N = 32768, A = I - Gmat, binary16 factors, TW = TR = F64: too large
    for the oracle, so checked by properties that hold at any size: the
    residual rule by an independent FP64 residual, every correction within
    the basis, x* = ones recovered."""
    n = 32768
    say(f"gmres-ir full size tf=f16 n={n}")
    At = I.gmat_operator_torch(n, 1.0, DEV)
    b = I.rhs_ones_torch(At)
    x, rep, kh = M.gmres_ir_solve(At, b, M.F16, term_parms=M.term(tol_rel=1e-14, litmax=20))
    say(f"  n_iter={rep.n_iter} khist={kh} relres={rep.relres:.2e}")
    assert rep.stop_name == "converged" and all(1 <= k <= 10 for k in kh)
    r = b.clone()
    for c0 in range(0, n, 4096):
        r -= At[c0:c0 + 4096].t().matmul(x[c0:c0 + 4096])
    assert float(r.abs().max()) / float(b.abs().max()) <= 2e-14
    assert float((x - 1.0).abs().max()) <= 1e-11


TW32_CASES = [("gmres", 700, 10.0, "f16"), ("gmres", 1100, 799.0, "f16"), ("gmres", 600, 100.0, "bf16"),
              ("bicgstab", 700, 10.0, "f16"), ("bicgstab", 1100, 799.0, "f16")]


@pytest.mark.parametrize("method,n,alpha,tf", TW32_CASES)
def test_krylov_ir_tw32_parity(M, orc, method, n, alpha, tf):
    """TW = F32, TR = F64: x kept in binary32, stop by eq. wilkterm.  Bars:
    the same stop and first residual, outer counts and the first correction's
    Krylov count within +-1, the final residual within a factor 3 of the
    oracle's (both at the binary32 floor), x within two binary32 ulps."""
    from oracle import bicgstab_ir, gmres_ir
    say(f"krylov tw=f32 {method} n={n} alpha={alpha} tf={tf}")
    T = {"f16": M.F16, "bf16": M.BF16}[tf]
    at = I.gmat_operator(n, alpha).astype(np.float32)
    b = (at.T.astype(np.float64) @ np.ones(n)).astype(np.float32)
    tp = M.term(litmax=10)
    f = M.Factorization(dev(at), T, M.F64)
    try:
        if method == "gmres":
            x, rep, kh = f.gmres_ir_solve(dev(b), term_parms=tp)
            ref = gmres_ir.gmres_ir_solve(at, b, T, litmax=10)
        else:
            x, rep, kh = f.bicgstab_ir_solve(dev(b), term_parms=tp)
            ref = bicgstab_ir.bicgstab_ir_solve(at, b, T, litmax=10)
    finally:
        f.destroy()
    say(f"  gpu n_iter={rep.n_iter} stop={rep.stop} khist={kh} rfinal={rep.rhist[rep.n_iter]:.2e} | "
        f"oracle n_iter={ref.n_iter} stop={ref.stop} khist={[int(k) for k in ref.khist]} rfinal={ref.rhist[-1]:.2e}")
    assert x.dtype == torch.float32
    assert rep.stop == ref.stop and rep.rhist[0] == ref.rhist[0]
    assert abs(rep.n_iter - ref.n_iter) <= 1 and abs(kh[0] - ref.khist[0]) <= 1
    assert 1 / 3 <= rep.rhist[rep.n_iter] / ref.rhist[-1] <= 3
    xg = x.cpu().numpy()
    assert np.abs(xg - ref.x).max() <= 2 * 2.0**-23 * np.abs(ref.x).max()


def test_printed_krylov_sessions_tw32(M, orc):
    """The printed IR-GMRES (basis 20) and IR-BiCGSTAB sessions (N = 4096,
    A = Float32(I - 799 Gmat) on the endpoint grid, binary16 factors,
    TR = F64) on the GPU: the final residual at the printed binary32 floor
    and the printed distance to the solution of the promoted problem."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))["E_krylov_tw32"]
    n, alpha = g["n"], g["alpha"]
    say(f"printed krylov sessions tw=f32 n={n}")
    ad = I.gmat_operator(n, alpha, grid="endpoint")
    h = 1.0 / (n - 1)
    xs = np.arange(n) * h
    a32 = ad.astype(np.float32)
    b32 = (1.0 - alpha * xs * (1.0 - xs) * 0.5).astype(np.float32)
    xp, info, _ = orc.solve_f64(a32, b32)
    f = M.Factorization(dev(a32), M.F16, M.F64)
    try:
        xg, rg, khg = f.gmres_ir_solve(dev(b32), term_parms=M.term(litmax=10), basissize=g["gmres_basissize"])
        xb, rb, khb = f.bicgstab_ir_solve(dev(b32), term_parms=M.term(litmax=10))
    finally:
        f.destroy()
    for x, rep, key in ((xg, rg, "gmres_rhist"), (xb, rb, "bicgstab_rhist")):
        say(f"  {key}: n_iter={rep.n_iter} stop={rep.stop_name} rfinal={rep.rhist[rep.n_iter]:.5e} "
            f"(printed {g[key][-1]:.5e}) |x - xp| = {np.abs(x.cpu().numpy() - xp).max():.5e}")
        assert rep.stop_name == "dstagnated"
        assert rep.rhist[0] == pytest.approx(g[key][0], rel=1e-5)
        assert 1 / 1.5 <= rep.rhist[rep.n_iter] / g[key][-1] <= 1.5
        assert np.abs(x.cpu().numpy() - xp).max() == pytest.approx(g["gmres_sol_minus_promoted_inf"], rel=0.01)


@pytest.mark.parametrize("method,limit", [("gmres", 1), ("gmres", 64), ("bicgstab", 1), ("bicgstab", 1000)])
def test_krylov_limits(M, method, limit):
    """The smallest and largest basis / iteration limit: every correction
    within the limit, the 1e-14 rule met (a one-step basis is IR with a
    minimal-residual step length)."""
    say(f"krylov limits {method} {limit}")
    at = I.gmat_operator(700, 10.0)
    b = I.rhs_ones(at)
    tp = M.term(tol_rel=1e-14, litmax=30)
    if method == "gmres":
        _, rep, kh = M.gmres_ir_solve(dev(at), dev(b), M.F16, term_parms=tp, basissize=limit)
    else:
        _, rep, kh = M.bicgstab_ir_solve(dev(at), dev(b), M.F16, term_parms=tp, maxit=limit)
    say(f"  n_iter={rep.n_iter} khist={kh} relres={rep.relres:.2e}")
    assert rep.stop_name == "converged" and rep.relres <= 1e-14
    assert all(1 <= k <= limit for k in kh)
