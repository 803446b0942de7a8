"""GPU parity of GMRES-IR (sections "Krylov-IR" and "GMRES-IR") against the
oracle in oracle/gmres_ir.py, through the C ABI.

Bars: the same stop reason; outer iteration counts within +-1; the GMRES
iteration counts of the corrections both runs take within +-1 each (the two
sides sum their inner products in different orders, so the inner stopping
test can fall one iteration apart); the residual rule met by both; the
solutions within the accuracy the refinement reaches (a forward error
bounded by kappa_inf(A) times the tolerance).
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
         ("gmat", 4096, 1.0, "f32", 10)]


@pytest.mark.parametrize("name,n,alpha,tf,m", CASES)
def test_gmres_ir_parity(M, G, orc, name, n, alpha, tf, m):
    say(f"gmres-ir {name} n={n} alpha={alpha} tf={tf} basis={m}")
    at = _operator(name, n, alpha)
    b = I.rhs_ones(at)
    tp = M.term(tol_rel=1e-14, litmax=20)
    x, rep, kh = M.gmres_ir_solve(dev(at), dev(b), TF[tf], term_parms=tp, basissize=m)
    ref = G.gmres_ir_solve(at, b, TF[tf], basissize=m, tol_rel=1e-14, litmax=20)
    say(f"  gpu n_iter={rep.n_iter} khist={kh} relres={rep.relres:.2e} | "
        f"oracle n_iter={ref.n_iter} khist={list(ref.khist)} relres={ref.relres:.2e}")
    assert rep.stop == ref.stop
    assert abs(rep.n_iter - ref.n_iter) <= 1
    assert len(kh) == rep.n_iter
    for kg, ko in zip(kh, ref.khist):
        assert abs(kg - ko) <= 1 and 1 <= kg <= m
    if ref.stop == 0:
        assert rep.relres <= 1e-14 and ref.relres <= 1e-14
        assert rep.rhist[rep.n_iter] <= 1e-14 * rep.rhist[0]
    xg = x.cpu().numpy()
    kappa = np.abs(at).sum(0).max() * np.abs(np.linalg.inv(at.T)).sum(1).max()
    assert np.abs(xg - ref.x).max() <= 10 * kappa * 1e-14 * np.abs(ref.x).max()
    # the GPU's first residual is the oracle's: both start from x = 0
    assert rep.rhist[0] == ref.rhist[0]


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
    f = M.Factorization(dev(at.astype(np.float32)), M.F16, M.F64)
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
