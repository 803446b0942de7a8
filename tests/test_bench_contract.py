"""CPU checks of bench.py's contract: a request for several GPUs is refused
with a message (this benchmark runs one GPU), the algorithmic bytes the
roofline divides by follow the stated formula, and the CPU baseline scales
its bounded oracle sample as stated."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "error" in msg and "--gpus must be 1" in msg["error"]


def test_trailing_bytes_formula():
    import bench
    # one step with a look-ahead panel: n = 2 nb.  The update of panel 0
    # touches the trailing nb x nb block in two launches (next panel's
    # columns, then nothing else): (m k + k nc + 2 m nc) * esz
    nb, esz = 8, 4
    n = 2 * nb
    got = bench.trailing_bytes(n, nb, esz)
    m, k, nc = nb, nb, nb
    assert got == (m * k + k * nc + 2 * m * nc) * esz
    # a single panel: nothing to update
    assert bench.trailing_bytes(nb, nb, esz) == 0.0


def test_cpu_baseline_scaling():
    # the oracle's bounded sample scaled to the full size: the factorization
    # part by (N/n)^3, the corrections timed at the full size when the full
    # matrix is given (else by (N/n)^2); the value is the sum of the two
    import bench
    from paper_2311_14616_amd import inputs as I
    n_s, n_f = 96, 160
    at_full = I.gmat_operator_torch(n_f, 1.0, "cpu")
    for full in (at_full, None):
        r = bench.cpu_baseline(n_s, n_f, full)
        assert r["kind"] == "oracle" and r["unit"] == "ms" and r["cores"] >= 1
        assert r["correction_timed_at_n"] == (n_f if full is not None else n_s)
        scale = 1.0 if full is not None else (n_f / n_s) ** 2
        s3 = (n_f / n_s) ** 3
        want = r["sample_factor_s"] * s3 + r["sample_n_iter"] * r["sample_correction_s"] * scale
        # the reported parts are rounded (to 1 ms and 0.1 ms), the value to 0.1 ms
        tol = 1e3 * (0.0005 * s3 + r["sample_n_iter"] * 0.00005 * scale) + 0.1
        assert abs(r["value"] - 1e3 * want) <= tol, (r, want)
        assert f"N={n_f}" in r["sample"]
