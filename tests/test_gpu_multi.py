"""GPU tests of mpir_ir_solve_multi (several right-hand sides with one
factorization).  Every column must be refined exactly as mpir_ir_solve
refines it alone (that path is parity-tested against the oracle): the same
x bit for bit and the same report, for every precision triple, both solves
(LPS and onthefly), chunks of the residual (4 columns) and of the
triangular solves (4, or 2 for binary64 solves), columns that stop at
different iterations, a zero column and a non-finite one.
"""
import sys

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I

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


def _rhs(at, nrhs, dt):
    """Columns that converge at different speeds: A*ones, A*x* for random
    x*, small random vectors, a zero column, a power-of-two multiple."""
    n = at.shape[1]
    rng = np.random.default_rng(nrhs)
    out = []
    for c in range(nrhs):
        k = c % 5
        if k == 0:
            b = I.rhs_ones(at)
        elif k == 1:
            b = at.T.astype(np.float64) @ rng.standard_normal(n)
        elif k == 2:
            b = rng.standard_normal(n) * 1e-3
        elif k == 3:
            b = np.zeros(n)
        else:
            b = 2.0**10 * I.rhs_ones(at)
        out.append(np.asarray(b, dtype=dt))
    return np.ascontiguousarray(np.stack(out))


CASES = [  # (tw, tf, tr, onthefly, n, alpha, nrhs)
    ("f64", "f32", "f64", False, 700, 10.0, 6),
    ("f64", "f16", "f64", False, 300, 100.0, 5),
    ("f64", "bf16", "f64", False, 257, 1.0, 4),
    ("f64", "f64", "f64", False, 200, 10.0, 3),
    ("f64", "f16", "f64", True, 333, 10.0, 5),
    ("f32", "f32", "f64", False, 400, 1.0, 3),
    ("f32", "f16", "f32", False, 129, 1.0, 2),
    ("f64", "f32", "f64", False, 1, 1.0, 1),
]


@pytest.mark.parametrize("tw,tf,tr,otf,n,alpha,nrhs", CASES)
def test_multi_equals_single_columns(M, tw, tf, tr, otf, n, alpha, nrhs):
    say(f"multi tw={tw} tf={tf} tr={tr} onthefly={otf} n={n} nrhs={nrhs}")
    P = {"f64": M.F64, "f32": M.F32, "f16": M.F16, "bf16": M.BF16}
    dt = np.float64 if tw == "f64" else np.float32
    at = I.gmat_operator(n, alpha).astype(dt)
    B = _rhs(at, nrhs, dt)
    tp = M.term(tol_rel=1e-14 if tr == "f64" and tw == "f64" else 0.0, litmax=25, onthefly=otf)
    At = torch.from_numpy(np.ascontiguousarray(at)).to(DEV)
    Bd = torch.from_numpy(B).to(DEV)
    f = M.Factorization(At, P[tf], P[tr])
    try:
        X, reps = f.ir_solve_multi(Bd, term_parms=tp)
        for c in range(nrhs):
            x1, rep1 = f.ir_solve(Bd[c].contiguous(), term_parms=tp)
            r = reps[c]
            assert torch.equal(X[c], x1), c
            assert (r.n_iter, r.stop) == (rep1.n_iter, rep1.stop), c
            assert list(r.rhist[:r.n_hist]) == list(rep1.rhist[:rep1.n_hist]), c
            assert list(r.dhist[:r.n_iter]) == list(rep1.dhist[:rep1.n_iter]), c
            assert (r.relres, r.bwd_err) == (rep1.relres, rep1.bwd_err), c
        say("  n_iter per column:", [r.n_iter for r in reps], "stops:", [r.stop_name for r in reps])
        zero = [c for c in range(nrhs) if c % 5 == 3]
        for c in zero:
            assert reps[c].n_iter == 0 and reps[c].stop_name == "converged" and torch.all(X[c] == 0)
    finally:
        f.destroy()


def test_multi_nonfinite_column(M):
    say("multi nonfinite column")
    n = 200
    at = I.gmat_operator(n, 1.0)
    B = _rhs(at, 3, np.float64)
    B[1, 17] = np.nan
    f = M.Factorization(torch.from_numpy(at).to(DEV), M.F32, M.F64)
    try:
        X, reps = f.ir_solve_multi(torch.from_numpy(B).to(DEV), term_parms=M.term(tol_rel=1e-14, litmax=20),
                                   allow=(M.OK, M.ERR_NONFINITE))
        assert reps[1].stop_name == "nonfinite" and reps[1].n_iter == 0
        for c in (0, 2):
            assert reps[c].stop_name == "converged" and reps[c].bwd_err <= 1e-14
    finally:
        f.destroy()


def test_multi_full_size(M):
    """N = 32768, TF = FP32, four right-hand sides in one call: each column
    bit-identical to its single solve (the benchmark's configuration)."""
    n = 32768
    say(f"multi full size n={n} nrhs=4")
    At = I.gmat_operator_torch(n, 1.0, DEV)
    b = I.rhs_ones_torch(At)
    B = torch.stack([b, 0.5 * b, -b, 4.0 * b]).contiguous()
    tp = M.term(tol_rel=1e-14, litmax=20)
    f = M.Factorization(At, M.F32, M.F64)
    try:
        X, reps = f.ir_solve_multi(B, term_parms=tp)
        for c in range(4):
            x1, rep1 = f.ir_solve(B[c].contiguous(), term_parms=tp)
            assert torch.equal(X[c], x1) and reps[c].n_iter == rep1.n_iter
            assert reps[c].stop_name == "converged" and reps[c].bwd_err <= 1e-14
        say(f"  multi refinement {reps[0].t_ir_ms:.2f} ms for 4 columns, single {rep1.t_ir_ms:.2f} ms")
    finally:
        f.destroy()


def test_multi_padded_leading_dimensions(M):
    """B and X as views of wider arrays (ldb = n + 7, ldx = n + 3): the
    columns are read and written at their strides and equal the contiguous
    call bit for bit; the padding is left untouched."""
    say("multi padded leading dimensions")
    n, nrhs = 333, 5
    at = I.gmat_operator(n, 10.0)
    B = _rhs(at, nrhs, np.float64)
    Bbig = torch.zeros((nrhs, n + 7), dtype=torch.float64, device=DEV)
    Bbig[:, :n] = torch.from_numpy(B).to(DEV)
    Xbig = torch.full((nrhs, n + 3), 7.0, dtype=torch.float64, device=DEV)
    tp = M.term(tol_rel=1e-14, litmax=20)
    f = M.Factorization(torch.from_numpy(at).to(DEV), M.F16, M.F64)
    try:
        Xv, reps = f.ir_solve_multi(Bbig[:, :n], X=Xbig[:, :n], term_parms=tp)
        Xc, repc = f.ir_solve_multi(torch.from_numpy(B).to(DEV), term_parms=tp)
    finally:
        f.destroy()
    assert torch.equal(Xbig[:, :n], Xc)
    assert torch.all(Xbig[:, n:] == 7.0)
    assert [r.n_iter for r in reps] == [r.n_iter for r in repc]


def test_multi_after_refactor_equals_fresh_handle(M):
    """mpir_refactor reuses the handle (factors and the several-column
    workspace): refactoring a BF16 handle with a new matrix and solving three
    columns gives bit for bit what a fresh handle gives."""
    say("multi after refactor (bf16)")
    n = 400
    a1 = I.gmat_operator(n, 1.0)
    a2 = I.gmat_operator(n, 10.0)
    B = torch.from_numpy(_rhs(a2, 3, np.float64)).to(DEV)
    tp = M.term(tol_rel=1e-14, litmax=30)
    A1, A2 = torch.from_numpy(a1).to(DEV), torch.from_numpy(a2).to(DEV)
    f = M.Factorization(A1, M.BF16, M.F64)
    try:
        f.ir_solve_multi(torch.from_numpy(_rhs(a1, 3, np.float64)).to(DEV), term_parms=tp)
        f.refactor(A2)
        X1, r1 = f.ir_solve_multi(B, term_parms=tp)
    finally:
        f.destroy()
    g = M.Factorization(A2, M.BF16, M.F64)
    try:
        X2, r2 = g.ir_solve_multi(B, term_parms=tp)
    finally:
        g.destroy()
    assert torch.equal(X1, X2)
    assert [r.n_iter for r in r1] == [r.n_iter for r in r2]
