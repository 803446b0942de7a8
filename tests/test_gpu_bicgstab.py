"""GPU parity of BiCGSTAB-IR (section "Krylov-IR") against the oracle in
oracle/bicgstab_ir.py, through the C ABI.

As for GMRES-IR, the refinement reaches the binary64 residual floor after
one or two corrections, so the bars compare what rounding does not decide:
the first residual bit for bit; every common correction's BiCGSTAB count
within +-1 and within the limit; the residual after the first correction
within a factor 3 of the oracle's when it lies above 1e-12 ||b||; outer
counts within +-1; both final residuals at the floor (<= 1e-13 ||b||); the
same stop where the oracle's history has margin; the solutions within
10 kappa_inf(A) 1e-14 of the oracle's.
"""
import sys

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"
TOL = 1e-14


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
def B():
    from oracle import bicgstab_ir
    return bicgstab_ir


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _stop_has_margin(ref):
    rel = np.asarray(ref.rhist) / ref.rhist[0]
    ratios = rel[2:] / rel[1:-1]
    return (ref.stop == 0 and rel[-1] <= TOL / 3 and bool(np.all(rel[1:-1] >= 3 * TOL))
            and bool(np.all(ratios <= 0.3)))


CASES = [("gmat", 512, 1.0, "f32", 10), ("gmat", 512, 799.0, "f16", 10),
         ("gmat", 1100, 10.0, "f16", 10), ("rand", 650, 0.0, "f16", 10),
         ("gmat", 300, 1.0, "f64", 10), ("gmat", 777, 100.0, "f16", 2),
         ("gmat", 640, 799.0, "bf16", 10), ("gmat", 1100, 10.0, "f16", 1),
         ("gmat", 4096, 1.0, "f32", 10)]


@pytest.mark.parametrize("name,n,alpha,tf,m", CASES)
def test_bicgstab_ir_parity(M, B, orc, name, n, alpha, tf, m):
    say(f"bicgstab-ir {name} n={n} alpha={alpha} tf={tf} maxit={m}")
    T = {"f64": M.F64, "f32": M.F32, "f16": M.F16, "bf16": M.BF16}[tf]
    at = I.gmat_operator(n, alpha) if name == "gmat" else I.random_dense(n, 17, diag_shift=2.0 * np.sqrt(n))
    b = I.rhs_ones(at)
    tp = M.term(tol_rel=TOL, litmax=20)
    x, rep, kh = M.bicgstab_ir_solve(dev(at), dev(b), T, term_parms=tp, maxit=m)
    ref = B.bicgstab_ir_solve(at, b, T, maxit=m, tol_rel=TOL, litmax=20)
    rg = [rep.rhist[k] / rep.rhist[0] for k in range(rep.n_iter + 1)]
    ro = list(np.asarray(ref.rhist) / ref.rhist[0])
    say(f"  gpu n_iter={rep.n_iter} stop={rep.stop} khist={kh} rhist={['%.1e' % v for v in rg]} | "
        f"oracle n_iter={ref.n_iter} stop={ref.stop} khist={[int(k) for k in ref.khist]} "
        f"rhist={['%.1e' % v for v in ro]}")
    assert rep.rhist[0] == ref.rhist[0]
    assert len(kh) == rep.n_iter and rep.n_iter >= 1
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


def test_bicgstab_ir_recovers_where_half_ir_stalls(M):
    say("bicgstab-ir vs ir, alpha=799 tf=f16")
    at = I.gmat_operator(512, 799.0)
    b = I.rhs_ones(at)
    tp = M.term(tol_rel=TOL, litmax=20)
    f = M.Factorization(dev(at), M.F16, M.F64)
    try:
        _, rep_ir = f.ir_solve(dev(b), term_parms=tp)
        _, rep_b, kh = f.bicgstab_ir_solve(dev(b), term_parms=tp)
        _, rep_b2, kh2 = f.bicgstab_ir_solve(dev(b), term_parms=tp)
    finally:
        f.destroy()
    assert rep_ir.stop_name != "converged"
    assert rep_b.stop_name == "converged" and rep_b.relres <= TOL
    # deterministic: the same call twice gives the same history
    assert (rep_b2.n_iter, kh2) == (rep_b.n_iter, kh)
    assert list(rep_b2.rhist[:rep_b2.n_hist]) == list(rep_b.rhist[:rep_b.n_hist])


def test_bicgstab_ir_errors_and_zero_rhs(M):
    say("bicgstab-ir errors / zero rhs")
    at = I.gmat_operator(64, 1.0)
    x, rep, kh = M.bicgstab_ir_solve(dev(at), dev(np.zeros(64)), M.F32)
    assert rep.n_iter == 0 and rep.stop_name == "converged" and kh == [] and torch.all(x == 0)
    f = M.Factorization(dev(at), M.F32, M.F64)
    try:
        for m in (0, 1001):
            with pytest.raises(M.MpirError):
                f.bicgstab_ir_solve(dev(I.rhs_ones(at)), maxit=m)
    finally:
        f.destroy()


def test_bicgstab_ir_full_size(M):
    n = 32768
    say(f"bicgstab-ir full size tf=f16 n={n}")
    At = I.gmat_operator_torch(n, 1.0, DEV)
    b = I.rhs_ones_torch(At)
    x, rep, kh = M.bicgstab_ir_solve(At, b, M.F16, term_parms=M.term(tol_rel=TOL, litmax=20))
    say(f"  n_iter={rep.n_iter} khist={kh} relres={rep.relres:.2e} t_ir={rep.t_ir_ms:.1f} ms")
    assert rep.stop_name == "converged" and all(1 <= k <= 10 for k in kh)
    r = b.clone()
    for c0 in range(0, n, 4096):
        r -= At[c0:c0 + 4096].t().matmul(x[c0:c0 + 4096])
    assert float(r.abs().max()) / float(b.abs().max()) <= 2e-14
    assert float((x - 1.0).abs().max()) <= 1e-11
