"""Pins of the Krylov-IR oracles with TW = F32 and TR = F64 (the outer loop
of oracle/krylov_ir.py): the paper's printed IR-GMRES and IR-BiCGSTAB
sessions (tests/golden, E_krylov_tw32).

The printed intermediate residuals come from the package's binary16 LU,
which rounds every operation to binary16; the oracle's binary16 mode keeps
the trailing matrix in binary32 (the mode the GPU implements), so it reaches
the binary32 floor after one correction where the printed GMRES session
needs seven.  What the factorization does not decide is pinned: the initial
residual, the stop by eq. wilkterm on the corrections, the final residual at
the binary32 storage floor, and the distance of the returned x from the
solution of the promoted problem (x is stored in binary32)."""
import json
import os

import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


@pytest.fixture(scope="module")
def problem(orc):
    g = GOLD["E_krylov_tw32"]
    n, alpha = g["n"], g["alpha"]
    ad = I.gmat_operator(n, alpha, grid="endpoint")
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    bd = 1.0 - alpha * x * (1.0 - x) * 0.5
    a32, b32 = ad.astype(np.float32), bd.astype(np.float32)
    xp, info, _ = orc.solve_f64(a32, b32)
    assert info == 0
    return g, a32, b32, xp


def _check(r, g, key):
    printed = g[key]
    assert r.stop == 2                                   # dstagnated (eq. wilkterm)
    assert r.x.dtype == np.float32
    assert r.rhist[0] == pytest.approx(printed[0], rel=1e-5)
    assert 1 / 1.5 <= r.rhist[-1] / printed[-1] <= 1.5    # the binary32 floor
    # the corrections after the first are at the binary32 floor of x
    assert np.all(r.dhist[1:] <= 1e-6 * r.dhist[0])


def test_printed_ir_gmres_session(G, orc, problem):
    g, a32, b32, xp = problem
    r = G.gmres_ir_solve(a32, b32, orc.F16, basissize=g["gmres_basissize"], litmax=10)
    _check(r, g, "gmres_rhist")
    assert np.abs(r.x - xp).max() == pytest.approx(g["gmres_sol_minus_promoted_inf"], rel=0.01)


def test_printed_ir_bicgstab_session(B, orc, problem):
    g, a32, b32, xp = problem
    r = B.bicgstab_ir_solve(a32, b32, orc.F16, litmax=10)
    _check(r, g, "bicgstab_rhist")
    assert np.abs(r.x - xp).max() == pytest.approx(g["gmres_sol_minus_promoted_inf"], rel=0.01)


@pytest.fixture(scope="module")
def G():
    from oracle import gmres_ir
    return gmres_ir


@pytest.fixture(scope="module")
def B():
    from oracle import bicgstab_ir
    return bicgstab_ir
