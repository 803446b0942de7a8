"""Time the oracle on the full benchmark workload once and cache the result.

Runs the oracle's Algorithm IR (emulated binary32 LU, binary64 residual,
the 1e-14 rule, litmax 20) on A = I - Gmat(N), b = A*ones at N = 32768 on
every host core (OpenMP), and writes oracle/cpu_time_n32768.json with the
wall time of the factorization and of the whole solve, the corrections, the
host CPU model, the core count and the OpenMP thread count.  bench.py
reports that file beside its bounded sample.  The oracle is test
infrastructure; this script only measures it.

    ORC_PROGRESS=1 python oracle/time_full_size.py [N]
"""
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2311_14616_amd import inputs as I  # noqa: E402


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fp:
            for line in fp:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main(n: int = 32768) -> None:
    os.environ.setdefault("ORC_PROGRESS", "1")
    print(f"[oracle timing] building A = I - Gmat({n})", flush=True)
    at = I.gmat_operator(n, 1.0)
    b = I.rhs_ones(at)
    print("[oracle timing] factorization alone", flush=True)
    t0 = time.perf_counter()
    af, _, _ = O.downcast(at, O.F32)
    O.lu(af, O.LU_F32)
    t_lu = time.perf_counter() - t0
    del af
    print(f"[oracle timing] factorization {t_lu:.1f} s; whole solve", flush=True)
    t0 = time.perf_counter()
    r = O.ir_solve(at, b, O.F32, tol_rel=1e-14, litmax=20)
    t_all = time.perf_counter() - t0
    out = {"n": n, "workload": f"A = I - Gmat({n}), b = A*ones, TW=F64 TF=F32 TR=F64, "
                               "||r||/||b|| <= 1e-14, litmax 20",
           "solve_s": round(t_all, 2), "factorization_s": round(t_lu, 2),
           "n_iter": int(r.n_iter), "stop": r.stop_name, "bwd_err": float(r.bwd_err),
           "host_cpu": cpu_model(), "host_nproc": os.cpu_count(), "omp_threads": O.num_threads()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"cpu_time_n{n}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 32768)
