"""Exact factorizations: a matrix built as A = L U with L unit lower
triangular (off-diagonal entries 0, +-1/4, +-1/2), U upper triangular with
integer entries and |u_jj| >= 40, scaled by a power of two.  Partial
pivoting then keeps every row in place (after j elimination steps column j
holds l_ij u_jj below u_jj, and |l_ij| <= 1/2), each multiplier is l_ij
exactly, and every product and sum of the elimination is a multiple of
2^(s-2) below 2^(s+8): exact in binary32 and binary64.  So the factors of
an IEEE implementation of the factorization step of Algorithm IR are L and
2^s U bit for bit, whatever order the trailing updates sum in.  The scale
puts the entries in and around the subnormal range of TF, where a unit that
flushed subnormal operands or results to zero would show."""
import sys

import numpy as np
import pytest

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


def exact_lu(n, seed, sparse=False):
    """sparse: few nonzeros of L and U (off-diagonal U entries +-1, pivots
    +-8 or +-16), so that every entry of A and of the factors has at most
    eight significant bits (exact in bfloat16)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, n)) < (0.002 if sparse else 0.05)
    vals = rng.choice([-0.5, -0.25, 0.25, 0.5], size=(n, n))
    L = np.eye(n) + np.tril(mask * vals, -1)
    if sparse:
        um = rng.random((n, n)) < 0.05
        U = np.triu(um * rng.choice([-1.0, 1.0], size=(n, n)), 1)
        U[np.diag_indices(n)] = rng.choice([-16.0, -8.0, 8.0, 16.0], size=n)
    else:
        U = np.triu(rng.integers(-8, 9, size=(n, n)).astype(np.float64), 1)
        U[np.diag_indices(n)] = rng.choice([-64.0, -48.0, -40.0, 40.0, 48.0, 64.0], size=n)
    A = L @ U                       # exact: multiples of 1/4 well below 2^53
    assert np.abs(A).max() < 2.0**8
    return L, U, A


# (TF, scale exponent s): binary32 subnormals lie below 2^-126, binary64
# below 2^-1022, binary16 below 2^-14; the entries span 2^(s-2) .. 2^(s+7),
# so with s = -128 (-1024, -16) about a third of the entries of A and of U
# are subnormal.  Binary16 factors (f16mixed: binary16 L and U, binary32
# trailing matrix) are exact too: every entry is a multiple of 2^(s-2)
# below 2^(s+7), within binary16's 11 significant bits; bfloat16 factors
# (8 significant bits) take the sparse matrix, with s = -130 reaching
# bfloat16's subnormal range (below 2^-126).
CASES = [("f32", -128), ("f64", -1024), ("f32", 0), ("f64", 0), ("f16", 0), ("f16", -16),
         ("bf16", 0), ("bf16", -130)]


def _representable(x, tfname):
    if tfname == "bf16":
        y = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    else:
        y = x.astype({"f32": np.float32, "f64": np.float64, "f16": np.float16}[tfname]).astype(np.float64)
    return np.array_equal(y, x)


@pytest.mark.parametrize("tfname,s", CASES, ids=[f"{t}_s{s}" for t, s in CASES])
def test_exact_factors(M, tfname, s):
    n = 1600        # several 512-column panels: leaves, in-panel and trailing updates
    say(f"exact LU tf={tfname} n={n} scale=2^{s}")
    L, U, A = exact_lu(n, seed=11, sparse=tfname == "bf16")
    As = A * 2.0**s
    assert np.array_equal(As / 2.0**s, A)            # the scaling is exact in binary64
    assert _representable(As, tfname)                # the downcast is exact
    tf = {"f32": M.F32, "f64": M.F64, "f16": M.F16, "bf16": M.BF16}[tfname]
    At = torch.from_numpy(np.ascontiguousarray(As.T)).to(DEV)   # column-major A
    f = M.Factorization(At, tf, M.F64)
    assert f.info == 0
    lu, ipiv = f.factors()
    f.destroy()
    assert np.array_equal(ipiv, np.arange(n, dtype=np.int32))
    want64 = np.tril(L, -1) + U * 2.0**s
    assert _representable(want64, tfname)            # the factors are representable in TF
    want = want64.astype(np.float64 if tfname == "f64" else np.float32)
    got = lu.float().cpu().numpy() if tfname in ("f16", "bf16") else lu.cpu().numpy()
    bad = np.argwhere(got != want)
    assert bad.size == 0, (len(bad), bad[:5].tolist(), [(float(got[i, j]), float(want[i, j])) for i, j in bad[:5]])


def test_handles_alive_together(M):
    # each handle owns its leaf exchange area (a pooled area comes back only
    # when its handle is destroyed): factorizations of handles alive at the
    # same time, and of a handle created after one of them was destroyed,
    # stay exact
    n = 1100
    say(f"exact LU, several handles alive, n={n}")
    cases = [exact_lu(n, seed) for seed in (21, 22, 23, 24)]
    def make(k):
        L, U, A = cases[k]
        At = torch.from_numpy(np.ascontiguousarray(A.T)).to(DEV)
        return M.Factorization(At, M.F32, M.F64), (np.tril(L, -1) + U).astype(np.float32)
    def check(f, want):
        lu, ipiv = f.factors()
        assert np.array_equal(ipiv, np.arange(n, dtype=np.int32))
        assert np.array_equal(lu.cpu().numpy(), want)
    hs = [make(k) for k in range(3)]
    for f, want in hs:
        check(f, want)
    hs[1][0].destroy()
    h3 = make(3)
    check(h3[0], h3[1])
    for f, want in (hs[0], hs[2]):
        check(f, want)
        f.destroy()
    h3[0].destroy()
