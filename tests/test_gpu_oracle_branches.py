"""GPU parity against the oracle for the termination rules, the reuse of a
factorization and the error states of a handle, through the C ABI.

  - termination (section "Terminating the while loop"): the paper's
    stagnation example (eq. stag at Rmax = .5 and .1), the small-backward-
    error rule (eq. term, residterm = 0) in cases where it stops earlier than
    eq. residterm, and the litmax stop;
  - several right-hand sides (sections "Memory Allocations: I" and
    "Double-Single IR"): every column of mpir_ir_solve_multi against the
    oracle's refinement of that column alone;
  - mplu! (mpir_refactor) followed by a refinement, against the oracle on the
    second matrix; a refactor that fails leaves the handle refusing every
    solve until a refactor succeeds;
  - the batched call without reports still returns a failing system's status.

Bars: the same stop reason, the iteration count within +-1 of the oracle's,
and where the refinement converges the backward error <= 1e-14 and x within
the forward-error bound B_fwd = 1e-12 kappa_inf(A) (u_d / 1e-16) of the
oracle's x (TW = F32 with TR = F64: a few units of 2^-24, the storage of x).
"""
import ctypes as C
import json
import os
import sys

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_examples.json")))


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


def _kappa_inf(at):
    a = at.T.astype(np.float64)
    return np.abs(a).sum(1).max() * np.abs(np.linalg.inv(a)).sum(1).max()


def _b_fwd(at):
    return 1e-12 * _kappa_inf(at) * (2.0**-53 / 1e-16)


# ------------------------------------------------------------------ eq. stag
@pytest.mark.parametrize("rmax,key", [(0.5, "rhist_rmax_0_5"), (0.1, "rhist_rmax_0_1")])
def test_paper_stagnation_example(M, orc, rmax, key):
    """Section "Changing the parameters": N = 512, A = I - 799 Gmat (endpoint
    grid), b = ones, TF = F32, default termination except Rmax.  The
    refinement stagnates (eq. stag) near 6e-12 after 5 (Rmax = .5) or 4
    (Rmax = .1) corrections in the printed sessions."""
    g = GOLD["E11_stagnation"]
    n = g["n"]
    say(f"paper stagnation example rmax={rmax}")
    at = I.gmat_operator(n, g["alpha"], grid="endpoint")
    b = np.ones(n)
    x, rep = M.ir_solve(dev(at), dev(b), M.F32, term_parms=M.term(Rmax=rmax))
    ref = orc.ir_solve(at, b, orc.F32, Rmax=rmax)
    rh, _ = rep.history()
    printed = np.array(g[key])
    say(f"  gpu n_iter={rep.n_iter} stop={rep.stop_name} rhist[-1]={rh[-1]:.3e}; oracle "
        f"{ref.n_iter} {ref.stop_name} {ref.rhist[-1]:.3e}; printed {len(printed) - 1} {printed[-1]:.3e}")
    assert rep.stop_name == ref.stop_name == "stagnated"
    assert abs(rep.n_iter - ref.n_iter) <= 1
    assert abs(len(rh) - len(printed)) <= 1
    assert rh[-1] >= rmax * rh[-2]                      # the rule that fired
    assert 1 / 3 < rh[-1] / printed[-1] < 3 and 1 / 3 < rh[-1] / ref.rhist[-1] < 3
    # the first correction's residual is the rounding error of a binary32
    # solve amplified by kappa_inf ~ 2e5: GPU and oracle (different summation
    # orders) agree on its size, not its digits
    assert 1 / 3 < rh[1] / ref.rhist[1] < 3


# ------------------------------------------------------------------ eq. term
TERM_CASES = [  # (n, alpha, tf, tol_rel): eq. term stops before eq. residterm would
    (700, 799.0, "f32", 0.0),      # residterm = 1 stagnates after 5; eq. term converges after 4
    (900, 10.0, "f16", 1e-14),     # residterm = 1 stagnates after 7; eq. term converges after 5
]


@pytest.mark.parametrize("n,alpha,tf,tol", TERM_CASES)
def test_small_backward_error_rule(M, orc, n, alpha, tf, tol):
    """eq. term: stop when ||r|| <= tol_e (||b|| + ||A|| ||x||), with ||A||
    the binary64 infinity norm formed by the downcast."""
    say(f"eq. term n={n} alpha={alpha} tf={tf} tol={tol}")
    T = {"f32": M.F32, "f16": M.F16}[tf]
    at = I.gmat_operator(n, alpha)
    b = np.ones(n)
    tp = M.term(residterm=False, tol_rel=tol, litmax=20)
    x, rep = M.ir_solve(dev(at), dev(b), T, term_parms=tp)
    ref = orc.ir_solve(at, b, T, residterm=False, tol_rel=tol, litmax=20)
    res1 = orc.ir_solve(at, b, T, residterm=True, tol_rel=tol, litmax=20)
    say(f"  gpu n_iter={rep.n_iter} {rep.stop_name}; oracle {ref.n_iter} {ref.stop_name} "
        f"(eq. residterm: {res1.n_iter} {res1.stop_name})")
    assert ref.stop_name == "converged" and ref.n_iter < res1.n_iter
    assert rep.stop_name == "converged"
    assert abs(rep.n_iter - ref.n_iter) <= 1
    assert rep.anorm_inf == ref.anorm                  # same binary64 row sums
    # the rule that fired, evaluated on the reported norms
    rh, _ = rep.history()
    tol_e = tol if tol > 0 else 2.0**-52
    assert rh[-1] <= tol_e * (rep.bnorm_inf + rep.anorm_inf * rep.xnorm_inf) * (1 + 1e-12)
    xg = x.cpu().numpy()
    assert np.abs(xg - ref.x).max() / np.abs(ref.x).max() <= _b_fwd(at)


# ------------------------------------------------------------------ litmax
@pytest.mark.parametrize("tf,litmax", [("f16", 3), ("f32", 1)])
def test_litmax_stop(M, orc, tf, litmax):
    """A refinement cut off by litmax returns after exactly litmax
    corrections with stop = litmax on both sides, and the residual history
    agrees with the oracle's to the accuracy of the low-precision solves."""
    n, alpha = 900, 10.0
    say(f"litmax tf={tf} litmax={litmax}")
    T = {"f32": M.F32, "f16": M.F16}[tf]
    at = I.gmat_operator(n, alpha)
    b = I.rhs_ones(at)
    tp = M.term(tol_rel=1e-14, litmax=litmax)
    x, rep = M.ir_solve(dev(at), dev(b), T, term_parms=tp)
    ref = orc.ir_solve(at, b, T, tol_rel=1e-14, litmax=litmax)
    rh, dh = rep.history()
    say(f"  gpu rhist {['%.3e' % v for v in rh]}; oracle {['%.3e' % v for v in ref.rhist]}")
    assert rep.stop_name == ref.stop_name == "litmax"
    assert rep.n_iter == ref.n_iter == litmax
    assert rh[0] == ref.rhist[0]
    # each correction contracts the residual by a factor of the order of
    # kappa u_F; the two sides' factors differ by rounding order only, so
    # every history entry agrees within a factor 4 and ||d_1|| closely
    assert np.all(np.abs(np.log(rh[1:] / ref.rhist[1:])) <= np.log(4.0))
    assert dh[0] == pytest.approx(ref.dhist[0], rel=1e-2)


# ------------------------------------------------------------------ several right-hand sides
def _columns(at, nrhs, dt):
    """A*ones, A*x* for Gaussian x*, small Gaussian vectors, a zero column
    and a power-of-two multiple of A*ones."""
    n = at.shape[1]
    rng = np.random.default_rng(100 + nrhs)
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


MULTI_CASES = [  # (tw, tf, tr, onthefly, n, alpha, nrhs)
    ("f64", "f32", "f64", False, 700, 10.0, 6),
    ("f64", "f16", "f64", False, 300, 100.0, 5),
    ("f64", "bf16", "f64", False, 257, 1.0, 5),
    ("f64", "f16", "f64", True, 333, 10.0, 5),
    ("f64", "f64", "f64", False, 200, 10.0, 3),
    ("f32", "f32", "f64", False, 400, 1.0, 4),
]


@pytest.mark.parametrize("tw,tf,tr,otf,n,alpha,nrhs", MULTI_CASES)
def test_multi_columns_against_oracle(M, orc, tw, tf, tr, otf, n, alpha, nrhs):
    say(f"multi vs oracle tw={tw} tf={tf} tr={tr} onthefly={otf} n={n} nrhs={nrhs}")
    P = {"f64": M.F64, "f32": M.F32, "f16": M.F16, "bf16": M.BF16}
    O = {"f64": orc.F64, "f32": orc.F32, "f16": orc.F16, "bf16": orc.BF16}
    dt = np.float64 if tw == "f64" else np.float32
    at = I.gmat_operator(n, alpha).astype(dt)
    B = _columns(at, nrhs, dt)
    wide = tw == "f32" and tr == "f64"
    tol = 0.0 if wide else 1e-14
    tp = M.term(tol_rel=tol, litmax=25, onthefly=otf)
    f = M.Factorization(dev(at), P[tf], P[tr])
    try:
        X, reps = f.ir_solve_multi(dev(B), term_parms=tp)
    finally:
        f.destroy()
    Xg = X.cpu().numpy().astype(np.float64)
    bfwd = _b_fwd(at)
    for c in range(nrhs):
        ref = orc.ir_solve(at, B[c], O[tf], tr=O[tr], tol_rel=tol, litmax=25, onthefly=otf)
        r = reps[c]
        say(f"  column {c}: gpu {r.n_iter} {r.stop_name} bwd={r.bwd_err:.1e}; "
            f"oracle {ref.n_iter} {ref.stop_name} bwd={ref.bwd_err:.1e}")
        assert r.stop_name == ref.stop_name, c
        assert abs(r.n_iter - ref.n_iter) <= 1, c
        assert r.rhist[0] == ref.rhist[0], c
        xs = np.abs(ref.x).max()
        if xs == 0:
            assert np.all(Xg[c] == 0)
            continue
        err = np.abs(Xg[c] - ref.x).max() / xs
        if wide:
            assert err <= 4 * 2.0**-24, c
        else:
            assert r.bwd_err <= 1e-14 and ref.bwd_err <= 1e-14, c
            assert err <= bfwd, c


# ------------------------------------------------------------------ mplu!
@pytest.mark.parametrize("tf", ["f32", "f16", "bf16"])
def test_refactor_against_oracle(M, orc, tf):
    """Factor A1, refactor A2 into the same handle, refine A2 x = A2*ones:
    the result matches the oracle's refinement of A2 (the first matrix
    leaves no trace)."""
    say(f"refactor vs oracle tf={tf}")
    P = {"f32": M.F32, "f16": M.F16, "bf16": M.BF16}[tf]
    O = {"f32": orc.F32, "f16": orc.F16, "bf16": orc.BF16}[tf]
    n = 450
    a1 = I.random_dense(n, 31, diag_shift=3.0 * np.sqrt(n))
    a2 = I.gmat_operator(n, 50.0)
    b2 = I.rhs_ones(a2)
    f = M.Factorization(dev(a1), P, M.F64)
    try:
        A2 = dev(a2)
        f.refactor(A2)
        assert f.status == M.OK and f.info == 0
        lu, ipiv = f.factors()
        x, rep = f.ir_solve(dev(b2), term_parms=M.term(tol_rel=1e-14, litmax=20))
    finally:
        f.destroy()
    af, anorm, _ = orc.downcast(a2, O)
    lu_o, ipiv_o, _, _ = orc.lu(af, orc.default_lu_mode(O))
    assert np.array_equal(ipiv, ipiv_o)                 # Gmat: no pivot near-ties
    ref = orc.ir_solve(a2, b2, O, tol_rel=1e-14, litmax=20)
    say(f"  gpu {rep.n_iter} {rep.stop_name} bwd={rep.bwd_err:.1e}; oracle {ref.n_iter} {ref.stop_name}")
    assert rep.anorm_inf == anorm
    assert rep.stop_name == ref.stop_name == "converged"
    assert abs(rep.n_iter - ref.n_iter) <= 1
    assert rep.bwd_err <= 1e-14
    xg = x.cpu().numpy()
    assert np.abs(xg - ref.x).max() / np.abs(ref.x).max() <= _b_fwd(a2)


def test_failed_refactor_empties_handle(M, orc):
    """mpir_refactor with an entry that overflows binary16 fails with
    MPIR_ERR_RANGE; the handle then refuses every solve (MPIR_ERR_STATE)
    instead of solving with stale factors, until a refactor succeeds."""
    say("failed refactor")
    n = 200
    a1 = I.gmat_operator(n, 1.0)
    bad = a1.copy()
    bad[17, 3] = 1.0e5
    b = I.rhs_ones(a1)
    f = M.Factorization(dev(a1), M.F16, M.F64)
    try:
        with pytest.raises(M.MpirError) as e:
            f.refactor(dev(bad))
        assert e.value.status == M.ERR_RANGE
        bt = dev(b)
        for call in (lambda: f.solve(bt), lambda: f.ir_solve(bt),
                     lambda: f.ir_solve_multi(bt.reshape(1, n).contiguous()),
                     lambda: f.gmres_ir_solve(bt), lambda: f.bicgstab_ir_solve(bt),
                     lambda: f.factors()):
            with pytest.raises(M.MpirError) as e:
                call()
            assert e.value.status == M.ERR_STATE
        nan = a1.copy()
        nan[5, 5] = np.nan
        with pytest.raises(M.MpirError) as e:
            f.refactor(dev(nan))
        assert e.value.status == M.ERR_NONFINITE
        with pytest.raises(M.MpirError) as e:
            f.ir_solve(bt)
        assert e.value.status == M.ERR_STATE
        # a good matrix makes the handle usable again
        A1 = dev(a1)
        f.refactor(A1)
        x, rep = f.ir_solve(bt, term_parms=M.term(tol_rel=1e-14, litmax=20))
    finally:
        f.destroy()
    ref = orc.ir_solve(a1, b, orc.F16, tol_rel=1e-14, litmax=20)
    assert rep.stop_name == ref.stop_name == "converged"
    assert abs(rep.n_iter - ref.n_iter) <= 1


# ------------------------------------------------------------------ batched status
def test_batched_without_reports_returns_failing_status(M):
    """mpir_ir_solve_batched with reps = NULL: a system with a zero column
    (exactly singular) still makes the call return MPIR_ERR_SINGULAR."""
    say("batched reps=NULL singular")
    L = M.lib()
    ns = [40, 65, 33]
    As, bs, xs = [], [], []
    for k, n in enumerate(ns):
        a = I.gmat_operator(n, 2.0)
        if k == 1:
            a[7, :] = 0.0                                  # column 7 of A (column-major storage)
        As.append(dev(a))
        bs.append(dev(np.ones(n)))
        xs.append(torch.zeros(n, dtype=torch.float64, device=DEV))
    kk = len(ns)
    n_arr = (C.c_int64 * kk)(*ns)
    lda = (C.c_int64 * kk)(*ns)
    pa = (C.c_void_p * kk)(*[a.data_ptr() for a in As])
    pb = (C.c_void_p * kk)(*[b.data_ptr() for b in bs])
    px = (C.c_void_p * kk)(*[x.data_ptr() for x in xs])
    st = L.mpir_ir_solve_batched(kk, n_arr, pa, lda, pb, px, M.F64, M.F32, M.F64, None, None,
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == M.ERR_SINGULAR
    # and with reports: the same status, the failing system identified
    st2, reps = M.ir_solve_batched(As, bs, xs, M.F32)
    assert st2 == M.ERR_SINGULAR
    assert [r.reserved for r in reps] == [M.OK, M.ERR_SINGULAR, M.OK]
    assert reps[1].info == 8
