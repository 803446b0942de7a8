"""GPU parity of the bfloat16 factorization (TF = BF16: the 16-bit format of
section "Half Precision", binary32 exponent range and an 8-bit significand)
against the oracle's bf16mixed mode, through the C ABI.

Bars (as for binary16): the downcast bit for bit; factors that are bfloat16
numbers, satisfy the componentwise backward-error bound pinned on the oracle
((3 u_b + gamma_3n(u_s)) |L||U|, u_b = 2^-8), pivot like the oracle on
the operator matrices and then lie within the first-order perturbation bound
(from both factorizations' measured backward errors) of the oracle's factors
(on a random matrix the first differing pivot must be a near-tie within the
measured difference of the two sides' active columns); one low-precision solve within gamma_2n(u_s)
componentwise of the oracle's solve on the GPU factors; refinement with the
oracle's stop reason, iteration counts within +-1 and backward error
<= 1e-14.
"""
import sys

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I
from lu_checks import check_first_pivot_difference, lu_difference_bound

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _gamma(k, u):
    return k * u / (1 - k * u)


def _perm_from_ipiv(ipiv):
    perm = np.arange(len(ipiv))
    for k, p in enumerate(ipiv):
        perm[[k, p]] = perm[[p, k]]
    return perm


@pytest.mark.parametrize("n", [1, 65, 300])
@pytest.mark.parametrize("tw", ["f64", "f32"])
def test_downcast_bitwise(M, orc, n, tw):
    say(f"downcast bf16 tw={tw} n={n}")
    rng = np.random.default_rng(n)
    at = rng.standard_normal((n, n)) * 10.0 ** rng.integers(-30, 30, (n, n))
    # bfloat16 ties and their neighbours, subnormals, the overflow edge
    special = np.array([1 + 2.0**-8, 1 + 3 * 2.0**-8, 1 + 2.0**-8 + 2.0**-30, 2.0**-134,
                        3 * 2.0**-134, 3.38e38, -1.5 * 2.0**-126, 1 - 2.0**-9])
    at.flat[: min(n * n, len(special))] = special[: n * n]
    if tw == "f32":
        at = at.astype(np.float32)
    out, anorm, st = M.downcast(dev(at), M.BF16)
    af, anorm_ref, st_ref = orc.downcast(at, orc.BF16)
    assert st == 0 and st_ref == 0
    assert out.dtype == torch.bfloat16
    assert np.array_equal(out.double().cpu().numpy(), af)
    assert anorm == anorm_ref


def test_downcast_overflow(M):
    say("downcast bf16 overflow")
    at = I.gmat_operator(70, 1.0)
    at[3, 4] = 3.4e38                      # above (2 - 2^-8) 2^127
    assert M.downcast(dev(at), M.BF16)[2] == M.ERR_RANGE


@pytest.mark.parametrize("name,n,alpha", [("gmat", 257, 10.0), ("gmat", 1300, 10.0),
                                          ("gmat", 700, 1.0), ("rand", 600, 0.0)])
def test_factor_parity(M, orc, name, n, alpha):
    say(f"factor bf16 {name} n={n}")
    at = I.gmat_operator(n, alpha) if name == "gmat" else I.random_dense(n, 5)
    f = M.factor(dev(at), M.BF16)
    lu, ipiv = f.factors()
    f.destroy()
    assert f.info == 0 and lu.dtype == torch.bfloat16
    lu = lu.double().cpu().numpy()
    af, _, _ = orc.downcast(at, orc.BF16)
    lu_o, ipiv_o, info_o, _ = orc.lu(af, orc.LU_BF16MIXED)
    assert info_o == 0
    assert np.array_equal(orc.fl_b(lu), lu)
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    assert np.abs(np.tril(lu, -1)).max() <= 1.0
    bound = (3 * 2.0**-8 + _gamma(3 * n, 2.0**-24)) * (np.abs(L) @ np.abs(U))
    assert np.all(np.abs(L @ U - af[_perm_from_ipiv(ipiv)]) <= bound)
    # the operator matrices have no pivot near-ties; a random matrix's
    # pivot sequence can part at a near-tie, where both sides' choices are
    # the first maximum of their own active column and tied within the
    # measured difference of the two columns
    if name == "gmat":
        assert np.array_equal(ipiv, ipiv_o)
    d = np.nonzero(ipiv != ipiv_o)[0]
    if len(d):
        check_first_pivot_difference(af, lu, ipiv, lu_o, ipiv_o, int(d[0]), 2.0**-8, say)
    else:
        # identical pivots: the factors within the first-order perturbation
        # bound of the two factorizations' measured backward errors
        bound = lu_difference_bound(lu_o, lu, af[_perm_from_ipiv(ipiv)])
        diff = np.abs(lu - lu_o)
        say(f"  max |LU_gpu - LU_orc| / bound = {(diff / np.maximum(bound, 1e-300)).max():.3e}")
        assert np.all(diff <= bound)


def test_single_solve_parity(M, orc):
    say("solve bf16 n=333")
    n = 333
    at = I.gmat_operator(n, 10.0)
    b = np.random.default_rng(1).standard_normal(n) * 1e-3
    f = M.factor(dev(at), M.BF16)
    lu, ipiv = f.factors()
    x = f.solve(dev(b)).cpu().numpy()
    f.destroy()
    lu = lu.double().cpu().numpy()
    sigma = orc.pow2_ceil(np.abs(b).max())
    y = orc.fl_b(orc.apply_pivots(ipiv, b) / sigma)
    ref = sigma * orc.trsv_lu(lu, y, orc.TS_F32)
    L = np.tril(lu, -1) + np.eye(n)
    U = np.triu(lu)
    Li, Ui = np.linalg.inv(L), np.linalg.inv(U)
    bound = _gamma(2 * n + 2, 2.0**-24) * (np.abs(Ui) @ np.abs(Li) @ np.abs(L) @ np.abs(U) @ np.abs(ref))
    assert np.all(np.abs(x - ref) <= 4 * bound + 1e-300)


@pytest.mark.parametrize("n,alpha,onthefly", [(512, 1.0, False), (900, 10.0, False),
                                              (300, 100.0, False), (1100, 1.0, True),
                                              (900, 10.0, True)])
def test_ir_parity(M, orc, n, alpha, onthefly):
    say(f"ir bf16 n={n} alpha={alpha} onthefly={onthefly}")
    at = I.gmat_operator(n, alpha)
    b = I.rhs_ones(at)
    tp = M.term(tol_rel=1e-14, litmax=30, onthefly=onthefly)
    x, rep = M.ir_solve(dev(at), dev(b), M.BF16, term_parms=tp)
    ref = orc.ir_solve(at, b, orc.BF16, tol_rel=1e-14, litmax=30, onthefly=onthefly)
    say(f"  n_iter gpu={rep.n_iter} oracle={ref.n_iter} bwd={rep.bwd_err:.2e}")
    assert rep.stop_name == ref.stop_name == "converged"
    assert abs(rep.n_iter - ref.n_iter) <= 1
    assert rep.bwd_err <= 1e-14 and ref.bwd_err <= 1e-14
    assert rep.rhist[0] == ref.rhist[0]
    xg = x.cpu().numpy()
    kappa = np.abs(at).sum(0).max() * np.abs(np.linalg.inv(at.T)).sum(1).max()
    assert np.abs(xg - ref.x).max() <= 10 * kappa * 1e-14 * np.abs(ref.x).max()


def test_gmres_ir_recovers_where_bf16_ir_stalls(M, orc):
    """alpha = 799: bfloat16 IR stagnates far above the tolerance, GMRES-IR
    with the bfloat16 factors as preconditioner meets it."""
    say("gmres-ir bf16 n=640 alpha=799")
    from oracle import gmres_ir as G
    n = 640
    at = I.gmat_operator(n, 799.0)
    b = I.rhs_ones(at)
    tp = M.term(tol_rel=1e-14, litmax=20)
    _, rep_ir = M.ir_solve(dev(at), dev(b), M.BF16, term_parms=tp)
    x, rep, kh = M.gmres_ir_solve(dev(at), dev(b), M.BF16, term_parms=tp)
    ref = G.gmres_ir_solve(at, b, orc.BF16, tol_rel=1e-14, litmax=20)
    say(f"  ir stop={rep_ir.stop_name} | gmres gpu n_iter={rep.n_iter} khist={kh} "
        f"oracle n_iter={ref.n_iter} khist={list(map(int, ref.khist))}")
    assert rep_ir.stop_name != "converged"
    assert rep.stop_name == "converged" and rep.relres <= 1e-14
    assert abs(kh[0] - ref.khist[0]) <= 1 and abs(rep.n_iter - ref.n_iter) <= 1


def test_full_size(M):
    """N = 32768, A = I - Gmat, TW = TR = F64, TF = BF16 with the schedule the
    benchmark times: multipliers bounded by one, converged to the 1e-14 rule
    by an independent FP64 residual, x* = ones recovered."""
    n = 32768
    say(f"full size bf16 n={n}")
    At = I.gmat_operator_torch(n, 1.0, DEV)
    b = I.rhs_ones_torch(At)
    f = M.Factorization(At, M.BF16, M.F64)
    lu, _ = f.factors()
    assert float(torch.tril(lu.float(), -1).abs().max()) <= 1.0
    del lu
    x, rep = f.ir_solve(b, term_parms=M.term(tol_rel=1e-14, litmax=30))
    f.destroy()
    say(f"  n_iter={rep.n_iter} stop={rep.stop_name} relres={rep.relres:.2e}")
    assert rep.stop_name == "converged"
    r = b.clone()
    for c0 in range(0, n, 4096):
        r -= At[c0:c0 + 4096].t().matmul(x[c0:c0 + 4096])
    assert float(r.abs().max()) / float(b.abs().max()) <= 2e-14
    assert float((x - 1.0).abs().max()) <= 1e-11
