"""Write oracle_scale_refs.json: the oracle's results at the configurations'
real sizes, which the oracle needs minutes for (too slow to run inside the
GPU test session).

Only the oracle (``oracle/``) and the seeded input generators are called;
nothing here touches the GPU library.  Run from the repository root:

    python tests/golden/make_scale_refs.py [half] [single] [wilkinson] [fingerprints]

Stored per case:
  * half (A = I - alpha*Gmat, N = 8192, TW = TR = F64, TF in {F16, BF16},
    alpha in {1, 10, 100}, ||r||/||b|| <= 1e-14, litmax 30) and single (the
    same operator with alpha = 1, TF = F32, litmax 20): the oracle's
    refinement -- corrections, stop reason, residual and correction
    histories, relres, backward error and ||x - 1||_inf;
  * wilkinson (A = H1 diag(sigma) H2 rounded to binary32, N = 16384,
    kappa in {1e4, 1e6, 1e7}, TW = TF = F32, TR = F64, litmax 20): the
    oracle's refinement as above, and its binary64 LU solve x_ref of the same
    binary32 system, stored at 1024 seeded indices (exact binary64 values as
    hex) with ||x_ref||_inf, so that a test can form the forward error of any
    x against it on that sample.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2311_14616_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_scale_refs.json")
SAMPLE = 1024


def _ir_record(r, x_exact=None):
    rec = {"n_iter": int(r.n_iter), "stop": r.stop_name,
           "rhist": [float(v) for v in r.rhist], "dhist": [float(v) for v in r.dhist],
           "relres": float(r.relres), "bwd_err": float(r.bwd_err)}
    if x_exact is not None:
        rec["xerr_inf"] = float(np.abs(r.x.astype(np.float64) - x_exact).max())
    return rec


def half_cases(out):
    n = 8192
    for tf, name in ((O.F16, "f16"), (O.BF16, "bf16")):
        for alpha in (1.0, 10.0, 100.0):
            at = I.gmat_operator(n, alpha)
            b = I.rhs_ones(at)
            t0 = time.time()
            r = O.ir_solve(at, b, tf, tol_rel=1e-14, litmax=30)
            key = f"half_n{n}_{name}_alpha{alpha:g}"
            out[key] = _ir_record(r, np.ones(n))
            out[key]["oracle_s"] = round(time.time() - t0, 2)
            print(key, out[key]["n_iter"], out[key]["stop"], out[key]["oracle_s"], "s", flush=True)


def single_cases(out):
    n = 8192
    at = I.gmat_operator(n, 1.0)
    b = I.rhs_ones(at)
    t0 = time.time()
    r = O.ir_solve(at, b, O.F32, tol_rel=1e-14, litmax=20)
    key = f"single_n{n}_f32_alpha1"
    out[key] = _ir_record(r, np.ones(n))
    out[key]["oracle_s"] = round(time.time() - t0, 2)
    print(key, out[key]["n_iter"], out[key]["stop"], out[key]["oracle_s"], "s", flush=True)


def wilkinson_cases(out):
    import torch
    n = 16384
    idx = np.sort(np.random.default_rng(7).choice(n, SAMPLE, replace=False))
    for kappa in (1e4, 1e6, 1e7):
        at_t, b_t, _, _ = I.wilkinson_operator_torch(n, kappa, "cpu")
        at32, b32 = at_t.numpy(), b_t.numpy()
        t0 = time.time()
        r = O.ir_solve(at32, b32, O.F32, tr=O.F64, litmax=20)
        t1 = time.time()
        xr, info, st = O.solve_f64(at32, b32)
        t2 = time.time()
        assert st == 0 and info == 0
        key = f"wilkinson_n{n}_kappa{kappa:.0e}"
        rec = out.get(key, {})
        rec.update(_ir_record(r))
        rec["xref_inf"] = float(np.abs(xr).max())
        rec["ferr_vs_xref"] = float(np.abs(r.x.astype(np.float64) - xr).max() / np.abs(xr).max())
        rec["sample_idx"] = [int(i) for i in idx]
        rec["xref_sample_hex"] = [float(v).hex() for v in xr[idx]]
        rec["oracle_ir_s"] = round(t1 - t0, 2)
        rec["oracle_f64_s"] = round(t2 - t1, 2)
        out[key] = rec
        print(key, rec["n_iter"], rec["stop"], f"ferr {rec['ferr_vs_xref']:.2e}",
              rec["oracle_ir_s"], rec["oracle_f64_s"], "s", flush=True)
        del at_t, b_t, at32, b32, xr


def fingerprints(out):
    """A few input values of the at-scale cases, so that a test can confirm
    that the device-side generators built the same matrices and vectors."""
    import torch
    rng = np.random.default_rng(11)
    n = 16384
    for kappa in (1e4, 1e6, 1e7):
        at_t, b_t, _, _ = I.wilkinson_operator_torch(n, kappa, "cpu")
        ii = rng.integers(0, n, 16)
        jj = rng.integers(0, n, 16)
        key = f"wilkinson_n{n}_kappa{kappa:.0e}"
        out.setdefault(key, {})["input_fingerprint"] = {
            "at_idx": [[int(j), int(i)] for j, i in zip(jj, ii)],
            "at_hex": [float(at_t[j, i]).hex() for j, i in zip(jj, ii)],
            "b_idx": [int(i) for i in ii],
            "b_hex": [float(b_t[i]).hex() for i in ii]}
        del at_t, b_t


def main(parts):
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    out["_about"] = ("Oracle results at the configurations' real sizes, written by "
                     "make_scale_refs.py (oracle and input generators only).")
    out["_threads"] = O.num_threads()
    steps = {"half": half_cases, "single": single_cases, "wilkinson": wilkinson_cases,
             "fingerprints": fingerprints}
    for p in parts or list(steps):
        steps[p](out)
        with open(OUT, "w") as fh:
            json.dump(out, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
