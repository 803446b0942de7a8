"""Benchmark: mixed-precision IR time-to-solve vs an FP64 LU solve, one GPU.

Workload (default): A = I - alpha*G (the paper's integral-equation operator,
interior grid), alpha = 1, N = 32768, b = A*ones, TW = FP64, TF = FP32,
TR = FP64; stop when ||r||/||b|| <= 1e-14 (litmax 20).  A step is one full
pass of the hot path: mpir_factor (downcast + blocked LU on the matrix cores)
followed by mpir_ir_solve (triangular solves, update, FP64 residual,
termination) with A and b already resident in HBM.  The comparator is an FP64
LU factorization + solve (mpir_factor with TF = FP64, then mpir_solve) on the
same GPU, timed the same way.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IR vs FP64-LU time-to-solve at 1e-14 backward err; batched solves/s"
PEAK = {"f32": 157.3, "f16": 2516.6, "f64": 78.6}     # dense matrix TFLOP/s (MI355X)
HBM_PEAK = 8000.0                                     # GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def trailing_bytes(n: int, nb: int, esz: int) -> float:
    """Algorithmic HBM bytes of all trailing-update launches of one
    factorization (the same two launches per step as the library: the next
    panel's columns, then the rest): A21 and U12 read once, A22 read and
    written once."""
    tot = 0.0
    for K in range(0, n, nb):
        w = min(nb, n - K)
        K1 = K + w
        w1 = min(nb, n - K1) if K1 < n else 0
        K2 = K1 + w1
        m = n - K1
        for nc in (w1, n - K2):
            if m > 0 and nc > 0:
                tot += esz * (m * w + w * nc + 2.0 * m * nc)
    return tot


def counter_traffic(tf_name: str, n: int):
    """HBM bytes per trailing-update launch from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary of this workload, scaled by the copy
    calibration it records; None if there is none or if the GEMM source has
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"trailing_gemm_{tf_name}_n{n}_counters.json")
    src = os.path.join(ROOT, "paper_2311_14616_amd", "csrc", "k_gemm.hip")
    if not os.path.exists(path):
        return None, None
    with open(path) as fp:
        rec = json.load(fp)
    with open(src, "rb") as fp:
        sha = hashlib.sha256(fp.read()).hexdigest()
    if rec.get("source_sha256") != sha:
        return None, rec
    return rec.get("hbm_bytes_per_launch"), rec


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fp:
            for line in fp:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_sample: int, n_full: int, at_full=None):
    """Time the oracle (plain C, OpenMP on the host cores) on a bounded sample
    of the workload and scale it to the full size N: the downcast and LU of
    the same operator at N = n_sample by (N/n)^3, and one correction (the
    FP64 residual and the substitutions with the factors) times the sample's
    number of corrections.  With the full matrix given (at_full, a device
    tensor in column-major storage) the correction is timed at the full size
    itself -- its O(N^2) work takes seconds -- because a correction timed at
    a power-of-two sample size does not scale by (N/n)^2: the oracle's
    strided column accesses make its cache behaviour depend on the size
    (5.3 s at N = 8192 against 0.09 s at N = 8000 on the same host).  The
    substitutions there run on the operator's own triangles with the
    identity permutation: the same work as with the factors.  The whole
    Algorithm IR solve of the sample is timed too, for reference."""
    from oracle import oracle as O
    from paper_2311_14616_amd import inputs as I
    import numpy as np
    at = I.gmat_operator(n_sample, 1.0)
    b = I.rhs_ones(at)
    t0 = time.perf_counter()
    af, _, _ = O.downcast(at, O.F32)
    lu_rm, ipiv, _, _ = O.lu(af, O.LU_F32)
    t_lu = time.perf_counter() - t0
    del af
    t0 = time.perf_counter()
    r = O.ir_solve(at, b, O.F32, tol_rel=1e-14, litmax=20)
    t_all = time.perf_counter() - t0
    s3, s2 = (n_full / n_sample) ** 3, (n_full / n_sample) ** 2
    if at_full is not None:
        ah = at_full.cpu().numpy()
        bh = ah.sum(axis=0)                      # A * ones (A in column-major storage)
        t0 = time.perf_counter()
        res = O.residual(ah, bh, np.zeros(n_full))
        O.lu_solve(ah, np.arange(n_full, dtype=np.int32), res, O.default_ts(O.F32))
        t_corr = time.perf_counter() - t0
        del ah, bh, res
        corr_scale, corr_at = 1.0, n_full
    else:
        x = np.zeros(n_sample)
        t_corr = float("inf")
        for _ in range(2):
            t0 = time.perf_counter()
            res = O.residual(at, b, x)
            O.lu_solve(lu_rm, ipiv, res, O.default_ts(O.F32))
            t_corr = min(t_corr, time.perf_counter() - t0)
        corr_scale, corr_at = s2, n_sample
    value_s = t_lu * s3 + r.n_iter * t_corr * corr_scale
    corr_txt = (f"{r.n_iter} corrections of {t_corr:.3f} s (FP64 residual + substitutions, timed at N={n_full})"
                if corr_at == n_full else
                f"{r.n_iter} corrections of {t_corr:.3f} s (FP64 residual + substitutions) x (N/{n_sample})^2")
    out = {"value": round(value_s * 1e3, 1), "unit": "ms", "cores": O.num_threads(), "kind": "oracle",
           "host_cpu": host_cpu_model(), "host_nproc": os.cpu_count(),
           "sample": f"oracle on the same operator: downcast + LU at N={n_sample} {t_lu:.2f} s x (N/{n_sample})^3, "
                     f"{corr_txt}, to N={n_full}",
           "sample_n_iter": int(r.n_iter), "sample_factor_s": round(t_lu, 3),
           "sample_correction_s": round(t_corr, 4), "correction_timed_at_n": int(corr_at),
           "sample_ir_solve_s": round(t_all, 3)}
    # the one full-size run of the oracle on a GPU host's CPU, if recorded
    # (oracle/time_full_size.py)
    full = os.path.join(ROOT, "oracle", f"cpu_time_n{n_full}.json")
    if os.path.exists(full):
        with open(full) as fp:
            out["measured_full_size"] = json.load(fp)
    return out


def gmat_kappa_inf(n: int, alpha: float, anorm: float):
    """kappa_inf(A) for A = I - alpha*G (interior grid, 0 < alpha below the
    smallest eigenvalue of T): G is the inverse of T = h^-2 tridiag(-1, 2, -1),
    so A^-1 = I + alpha (T - alpha I)^-1; T - alpha I is a nonsingular
    M-matrix with a nonnegative inverse, hence ||A^-1||_inf = max_i
    (1 + alpha y_i) with (T - alpha I) y = ones, one tridiagonal solve."""
    import numpy as np
    from scipy.linalg import solve_banded
    h = 1.0 / (n + 1)
    lam_min = 4.0 / h**2 * np.sin(np.pi * h / 2) ** 2
    if not (0.0 < alpha < lam_min):
        return None
    ab = np.zeros((3, n))
    ab[0, 1:] = -1.0 / h**2
    ab[1, :] = 2.0 / h**2 - alpha
    ab[2, :-1] = -1.0 / h**2
    y = solve_banded((1, 1), ab, np.ones(n))
    return anorm * float(np.max(1.0 + alpha * y))


def accuracy(x, rep, kappa):
    """Forward error of x against x* = ones and against the bound
    B_fwd = 1e-12 kappa_inf(A) (u_d / 1e-16), u_d = 2^-53."""
    ferr = float((x - 1.0).abs().max())          # ||x*||_inf = 1
    out = {"ferr_vs_ones": ferr}
    if kappa is not None:
        bf = 1e-12 * kappa * (2.0**-53 / 1e-16)
        out.update({"kappa_inf": kappa, "b_fwd": bf, "ferr_over_b_fwd": ferr / bf})
    return out


def batched_bench(M, I, torch, dev, tf_name: str, reps: int = 3):
    """Solves/s of the uneven batch (4096 systems, N_k in [32, 1024], seed
    2311) in one persistent launch replayed from a hipGraph, with the
    per-system forward error against x* = ones (b = A*ones)."""
    import numpy as np
    ns, alphas, ds = I.batched_spec()
    As, bs, xs = [], [], []
    for n, al, d in zip(ns, alphas, ds):
        at = I.gmat_operator_torch(int(n), float(al), dev)
        at[torch.arange(int(n)), torch.arange(int(n))] += torch.from_numpy(d).to(dev)
        As.append(at)
        bs.append(at.sum(0))
        xs.append(torch.empty(int(n), dtype=torch.float64, device=dev))
    tf = {"f32": M.F32, "f16": M.F16, "bf16": M.BF16}[tf_name]
    # panel width and update form per size class: measured on this device
    # (or read from the cache file) before the batch is created
    t0 = time.perf_counter()
    tuning = M.batch_autotune(M.F64, tf, os.environ.get("MPIR_TUNE_CACHE"))
    tune_s = time.perf_counter() - t0
    bt = M.Batch(As, bs, xs, tf, term_parms=M.term(tol_rel=1e-14, litmax=20), use_graph=True)
    bt.run()                                    # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st, rep = bt.run()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    bt.destroy()
    ferr = np.array([float((x - 1.0).abs().max()) for x in xs])
    bwd = np.array([r.bwd_err for r in rep])
    iters = np.array([r.n_iter for r in rep])
    return {"tf": tf_name, "systems": len(ns), "ms": round(ms, 3),
            "solves_per_s": round(len(ns) / (ms * 1e-3), 1),
            "all_converged": bool(all(r.stop == 0 for r in rep)),
            "n_iter_mean": float(iters.mean()), "n_iter_max": int(iters.max()),
            "ferr_p50": float(np.percentile(ferr, 50)), "ferr_p99": float(np.percentile(ferr, 99)),
            "bwd_err_max": float(bwd.max()),
            "device_factor_ms_sum": round(float(sum(r.t_factor_ms for r in rep)), 1),
            "device_ir_ms_sum": round(float(sum(r.t_ir_ms for r in rep)), 1),
            "autotune_s": round(tune_s, 2), "tuning": tuning.as_dict()}


def experiments(M, I, torch, dev):
    """The remaining workloads of the method, one JSON line each:
    (i)   TF=F32 IR at N=8192 against the FP64 LU solve;
    (ii)  TF=F16 IR at N in {8192, 32768}, alpha in {1, 10, 100}: iteration
          counts, stop reason and the level where it stalls, beside the
          onthefly (mixed-precision) solve, TF=BF16 and TF=F32;
    (iii) the Wilkinson-type matrices A = H1 diag(sigma) H2 at N=16384,
          kappa in {1e4, 1e6, 1e7}, TW=TF=F32, TR=F64: forward error of IR
          against x* and against the FP64 LU solve of the same matrix, and
          of one plain FP32 LU solve;
    (iv)  GMRES-IR (the factors as left preconditioner, basissize 10) and
          BiCGSTAB-IR (at most 10 iterations) against IR with TF=F16 at
          N=32768, alpha in {1, 10, 799}: corrections, Krylov iterations per
          correction, stop reason, time;
    (v)   several right-hand sides with one factorization (TF=F32, N=32768,
          nrhs in {4, 16}): refinement time of one mpir_ir_solve_multi call
          against nrhs single-column refinements."""
    import numpy as np
    tp = M.term(tol_rel=1e-14, litmax=20)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) * 1e3

    tp_mps = M.term(tol_rel=1e-14, litmax=20, onthefly=True)
    tp30 = M.term(tol_rel=1e-14, litmax=30)

    def ir(At, b, tf, tr=M.F64, term=tp):
        x = torch.empty_like(b)

        def go():
            f = M.Factorization(At, tf, tr)
            _, rep = f.ir_solve(b, x, term)
            f.destroy()
            return rep
        timed(go)                                   # warm-up
        rep, ms = timed(go)
        return x, rep, ms

    def lu64(At64, b64):
        x = torch.empty_like(b64)

        def go():
            f = M.Factorization(At64, M.F64, M.F64)
            f.solve(b64, x)
            f.destroy()
        timed(go)
        _, ms = timed(go)
        return x, ms

    def rec(rep):
        return {"n_iter": rep.n_iter, "stop": rep.stop_name, "relres": rep.relres,
                "bwd_err": rep.bwd_err, "rhist_rel": [v / rep.rhist[0] for v in rep.rhist[:rep.n_iter + 1]]}

    out = []
    # (i)
    n = 8192
    At = I.gmat_operator_torch(n, 1.0, dev)
    b = I.rhs_ones_torch(At)
    x, rep, ms = ir(At, b, M.F32)
    x64, ms64 = lu64(At, b)
    out.append({"experiment": "plain IR TF=F32 vs FP64 LU", "n": n, "alpha": 1.0, "ir_ms": round(ms, 3),
                "fp64_lu_ms": round(ms64, 3), "speedup": round(ms64 / ms, 3), **rec(rep),
                "ferr_vs_ones": float((x - 1).abs().max()), "ferr_fp64_lu_vs_ones": float((x64 - 1).abs().max())})
    print(json.dumps(out[-1]), flush=True)
    del At, b
    # (ii)
    for n in (8192, 32768):
        for alpha in (1.0, 10.0, 100.0):
            At = I.gmat_operator_torch(n, alpha, dev)
            b = I.rhs_ones_torch(At)
            row = {"experiment": "half-precision factorization", "n": n, "alpha": alpha}
            for name, tf, tpar in (("f16", M.F16, tp), ("f16_onthefly", M.F16, tp_mps),
                                   ("bf16", M.BF16, tp30), ("f32", M.F32, tp)):
                x, rep, ms = ir(At, b, tf, M.F64, tpar)
                r = rec(rep)
                r["ms"] = round(ms, 3)
                r["ferr_vs_ones"] = float((x - 1).abs().max())
                r["stall_relres"] = min(r["rhist_rel"])
                row[name] = r
            print(json.dumps(row), flush=True)
            out.append(row)
            del At, b
    # (iii)
    n = 16384
    for kappa in (1e4, 1e6, 1e7):
        at32, b32, xstar, _ = I.wilkinson_operator_torch(n, kappa, dev)
        wt = M.term(litmax=20)                      # TR wider than TW: eq. wilkterm
        x, rep, ms = ir(at32, b32, M.F32, M.F64, wt)
        x64, _ = lu64(at32.to(torch.float64), b32.to(torch.float64))
        xp = torch.empty_like(b32)
        f = M.Factorization(at32, M.F32, M.F32)
        f.solve(b32, xp)
        f.destroy()
        xsn = float(xstar.abs().max())
        row = {"experiment": "Wilkinson-type, TW=TF=F32, TR=F64", "n": n, "kappa": kappa, "ms": round(ms, 3),
               "n_iter": rep.n_iter, "stop": rep.stop_name,
               "ferr_ir_vs_xstar": float((x.double() - xstar).abs().max()) / xsn,
               "ferr_ir_vs_fp64_lu": float((x.double() - x64).abs().max()) / float(x64.abs().max()),
               "ferr_fp64_lu_vs_xstar": float((x64 - xstar).abs().max()) / xsn,
               "ferr_plain_f32_lu_vs_xstar": float((xp.double() - xstar).abs().max()) / xsn,
               "dhist": list(rep.dhist[:rep.n_iter])}
        print(json.dumps(row), flush=True)
        out.append(row)
        del at32, b32
    # (iv)
    n = 32768
    for alpha in (1.0, 10.0, 799.0):
        At = I.gmat_operator_torch(n, alpha, dev)
        b = I.rhs_ones_torch(At)
        row = {"experiment": "GMRES-IR and BiCGSTAB-IR vs IR, TF=F16", "n": n, "alpha": alpha}
        x, rep, ms = ir(At, b, M.F16, M.F64, tp)
        row["ir"] = {**rec(rep), "ms": round(ms, 3), "ferr_vs_ones": float((x - 1).abs().max())}
        xg = torch.empty_like(b)

        def go():
            f = M.Factorization(At, M.F16, M.F64)
            _, rp, kh = f.gmres_ir_solve(b, xg, tp)
            f.destroy()
            return rp, kh
        timed(go)
        (rep, kh), ms = timed(go)
        row["gmres_ir"] = {**rec(rep), "khist": kh, "ms": round(ms, 3),
                           "factor_ms": round(rep.t_factor_ms, 3), "refine_ms": round(rep.t_ir_ms, 3),
                           "ferr_vs_ones": float((xg - 1).abs().max())}

        def go_b():
            f = M.Factorization(At, M.F16, M.F64)
            _, rp, kh = f.bicgstab_ir_solve(b, xg, tp)
            f.destroy()
            return rp, kh
        timed(go_b)
        (rep, kh), ms = timed(go_b)
        row["bicgstab_ir"] = {**rec(rep), "khist": kh, "ms": round(ms, 3),
                              "factor_ms": round(rep.t_factor_ms, 3), "refine_ms": round(rep.t_ir_ms, 3),
                              "ferr_vs_ones": float((xg - 1).abs().max())}
        print(json.dumps(row), flush=True)
        out.append(row)
        del At, b
    # (v)
    n = 32768
    At = I.gmat_operator_torch(n, 1.0, dev)
    b = I.rhs_ones_torch(At)
    f = M.Factorization(At, M.F32, M.F64)
    for nrhs in (4, 16):
        scales = [2.0 ** (k % 7 - 3) * (-1) ** k for k in range(nrhs)]
        B = torch.stack([s * b for s in scales]).contiguous()
        X, reps = f.ir_solve_multi(B, term_parms=tp)            # warm-up
        (X, reps), ms_multi = timed(lambda: f.ir_solve_multi(B, term_parms=tp))
        ms_single = 0.0
        for c in range(nrhs):
            _, ms = timed(lambda: f.ir_solve(B[c].contiguous(), term_parms=tp))
            ms_single += ms
        row = {"experiment": "several right-hand sides, TF=F32", "n": n, "nrhs": nrhs,
               "multi_ms": round(ms_multi, 3), "single_ms_sum": round(ms_single, 3),
               "speedup": round(ms_single / ms_multi, 3),
               "n_iter": [r.n_iter for r in reps], "all_converged": all(r.stop == 0 for r in reps),
               "bwd_err_max": max(r.bwd_err for r in reps)}
        print(json.dumps(row), flush=True)
        out.append(row)
        del B, X
    f.destroy()
    del At, b
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--alpha", type=float, default=1.0)
    ap.add_argument("--tf", choices=["f32", "f16"], default="f32")
    ap.add_argument("--fp64-runs", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=8192)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--experiments", action="store_true",
                    help="run the N=8192 comparison, the half-precision alpha sweep and the "
                         "Wilkinson-type cases instead of the benchmark (one JSON line each)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device to device once (the reference kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU benchmark: --gpus must be 1 (sharding the "
                                   "factorization over several GPUs is not implemented)"}))
        sys.exit(2)

    import torch
    import paper_2311_14616_amd.mpir as M
    from paper_2311_14616_amd import inputs as I

    dev = torch.device("cuda:0")
    if args.experiments:
        experiments(M, I, torch, dev)
        return
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 1 GiB read, 1 GiB written")
        del src, dst
    n = args.n
    tf = {"f32": M.F32, "f16": M.F16}[args.tf]
    log(f"[bench] generating A (N={n}) on the device")
    At = I.gmat_operator_torch(n, args.alpha, dev)
    b = I.rhs_ones_torch(At)
    x = torch.empty_like(b)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    tp = M.term(tol_rel=1e-14, litmax=20)

    def step():
        f = M.Factorization(At, tf, M.F64, stream)
        _, rep = f.ir_solve(b, x, tp)
        f.destroy()
        return rep

    for w in range(args.warmup):
        log(f"[bench] warmup {w}")
        step()
    torch.cuda.synchronize()
    M.prof_reset()
    M.prof_enable(True)
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    reps = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    M.prof_enable(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    rep = reps[-1]
    g_ms, g_cnt, g_flops = M.prof_get(M.PROF_GEMM)
    p_ms, p_cnt, _ = M.prof_get(M.PROF_PANEL)
    t_ms, t_cnt, _ = M.prof_get(M.PROF_TRSV)
    v_ms, v_cnt, v_bytes = M.prof_get(M.PROF_GEMV)
    d_ms, d_cnt, d_bytes = M.prof_get(M.PROF_DOWNCAST)
    gemm_tflops = g_flops / (g_ms * 1e-3) / 1e12 if g_ms > 0 else 0.0
    # algorithmic bytes of the trailing updates: A21, U12 read, A22 read and
    # written, in the working precision of the factorization (4 B; 8 B F64)
    g_bytes = trailing_bytes(n, int(os.environ.get("MPIR_NB", "512")), 4) * args.steps
    traffic, trec = counter_traffic(args.tf, n)
    traffic_src = (f"profiles/trailing_gemm_{args.tf}_n{n}_counters.json"
                   + ("" if traffic is not None else " (absent or stale)")) if trec is not None or traffic is None else None
    gemv_gbs = v_bytes / (v_ms * 1e-3) / 1e9 if v_ms > 0 else 0.0
    trsv_bytes_per = (4 if args.tf == "f32" else 2) * n * n
    trsv_gbs = trsv_bytes_per * t_cnt / (t_ms * 1e-3) / 1e9 if t_ms > 0 else 0.0
    kappa = gmat_kappa_inf(n, args.alpha, rep.anorm_inf)
    log(f"[bench] IR step {ms_step:.2f} ms  n_iter={rep.n_iter} stop={rep.stop_name} "
        f"bwd={rep.bwd_err:.2e}  gemm {gemm_tflops:.1f} TF/s  panel {p_ms / args.steps:.1f} ms/step")

    out = {
        "metric": METRIC, "value": round(ms_step, 3), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": f"{args.tf}+f64", "data": "synthetic",
        "config": {"workload": f"IR solve of A = I - {args.alpha:g}*Gmat(N), b = A*ones, "
                               f"N={n}, TW=FP64, TF={args.tf.upper()}, TR=FP64, "
                               f"tol ||r||/||b|| <= 1e-14, litmax 20",
                   "n": n, "alpha": args.alpha, "tw": "f64", "tf": args.tf, "tr": "f64"},
        "ir": {"n_iter": rep.n_iter, "stop": rep.stop_name, "bwd_err": rep.bwd_err,
               "relres": rep.relres, "t_factor_ms": rep.t_factor_ms, "t_ir_ms": rep.t_ir_ms,
               **accuracy(x, rep, kappa)},
        "roofline": {"bound": "mfma", "achieved": round(gemm_tflops, 2), "peak": PEAK[args.tf],
                     "unit": "TFLOP/s", "frac": round(gemm_tflops / PEAK[args.tf], 4),
                     "traffic": traffic, "kernel": f"trailing-update GEMM ({args.tf} MFMA)",
                     "launches": g_cnt, "avg_launch_ms": g_ms / max(g_cnt, 1),
                     "algorithmic_bytes_per_launch": g_bytes / max(g_cnt, 1),
                     "traffic_source": traffic_src},
        "kernels": {
            "gemm_ms_per_step": g_ms / args.steps, "panel_ms_per_step": p_ms / args.steps,
            "trsv_ms_per_step": t_ms / args.steps, "gemv_ms_per_step": v_ms / args.steps,
            "downcast_ms_per_step": d_ms / args.steps,
            "gemv_GBps": round(gemv_gbs, 1), "gemv_hbm_frac": round(gemv_gbs / HBM_PEAK, 4),
            "trsv_GBps": round(trsv_gbs, 1),
        },
    }
    if args.tf == "f32":
        # the same solve with the 16-bit factorizations (binary16 or bfloat16
        # L and U, binary32 trailing matrix, 16-bit MFMA with binary32
        # accumulation)
        xh = torch.empty_like(b)
        for key, tfh in (("f16_factorization", M.F16), ("bf16_factorization", M.BF16)):
            log(f"[bench] {key}: solve of the same system")

            def step_h():
                f = M.Factorization(At, tfh, M.F64, stream)
                _, rh = f.ir_solve(b, xh, M.term(tol_rel=1e-14, litmax=30))
                f.destroy()
                return rh
            step_h()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rh = step_h()
            torch.cuda.synchronize()
            hms = (time.perf_counter() - t0) * 1e3
            out[key] = {"ms": round(hms, 3), "n_iter": rh.n_iter, "stop": rh.stop_name,
                        "bwd_err": rh.bwd_err, "relres": rh.relres,
                        "t_factor_ms": rh.t_factor_ms, "t_ir_ms": rh.t_ir_ms,
                        **accuracy(xh, rh, kappa)}
            log(f"[bench] {key}: {hms:.2f} ms, n_iter={rh.n_iter}, bwd={rh.bwd_err:.2e}")
    if not args.no_fp64:
        log("[bench] FP64 LU comparator")
        xs = torch.empty_like(b)

        def fp64_step():
            f = M.Factorization(At, M.F64, M.F64, stream)
            f.solve(b, xs)
            f.destroy()

        fp64_step()            # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.fp64_runs):
            fp64_step()
        torch.cuda.synchronize()
        fp64_ms = (time.perf_counter() - t0) * 1e3 / args.fp64_runs
        r64, rn64 = M.residual(At, b, xs, M.F64)
        bn = float(b.abs().max())
        out["fp64_lu_ms"] = round(fp64_ms, 3)
        out["speedup_vs_fp64_lu"] = round(fp64_ms / ms_step, 3)
        for key in ("f16_factorization", "bf16_factorization"):
            if key in out:
                out[key]["speedup_vs_fp64_lu"] = round(fp64_ms / out[key]["ms"], 3)
        out["fp64_lu_relres"] = rn64 / bn
        out["fp64_lu_ferr_vs_ones"] = float((xs - 1.0).abs().max())
        log(f"[bench] FP64 LU solve {fp64_ms:.2f} ms  relres={rn64 / bn:.2e}")
    if not args.no_batched:
        out["batched"] = []
        for tfn in ("f32", "f16", "bf16"):
            log(f"[bench] batched 4096 uneven systems, TF={tfn}")
            out["batched"].append(batched_bench(M, I, torch, dev, tfn))
            log(f"[bench]   {out['batched'][-1]}")
    if not args.no_cpu:
        log(f"[bench] CPU oracle sample N={args.cpu_sample}")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample, n, At if args.alpha == 1.0 else None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
