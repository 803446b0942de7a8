"""CPU checks of bench.py's contract: a request for several GPUs is refused
with a message (this benchmark runs one GPU), and the algorithmic bytes the
roofline divides by follow the stated formula."""
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
