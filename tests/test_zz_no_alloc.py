"""mpir_residual_noalloc (the allocation-free residual, scratch in a fixed
device array of the library) against mpir_residual, through the C ABI: the
same kernels in the same order, so the residual and its norm are equal bit
for bit.  Two calls in a row on one GPU, the second smaller, show that the
scratch left by a call does not leak into the next; sizes beyond the
documented maximum are refused."""
import ctypes as C
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


def _case(n, tw, seed):
    """Seeded Gaussian A (column-major storage), x and b, drawn on the device."""
    dt = torch.float64 if tw == "f64" else torch.float32
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    at = torch.randn((n, n), generator=g, dtype=dt, device=DEV)
    b = torch.randn(n, generator=g, dtype=dt, device=DEV)
    x = torch.randn(n, generator=g, dtype=dt, device=DEV)
    return at, b, x


@pytest.mark.parametrize("tw,tr", [("f64", "f64"), ("f32", "f64"), ("f32", "f32")])
def test_noalloc_residual_equals_allocating_call(M, tw, tr):
    P = {"f64": M.F64, "f32": M.F32}
    rdt = torch.float64 if tr == "f64" else torch.float32
    # the largest size first, then a smaller one with a ragged chunk
    for n, seed in ((M.RESIDUAL_NOALLOC_MAX_N, 3), (1000, 4)):
        say(f"noalloc residual tw={tw} tr={tr} n={n}")
        At, b, x = _case(n, tw, seed)
        r_ref, rn_ref = M.residual(At, b, x, P[tr])
        r = torch.full((n,), float("nan"), dtype=rdt, device=DEV)
        rn = M.residual_noalloc(At, b, x, r, P[tr])
        torch.cuda.synchronize()
        assert torch.equal(r, r_ref)
        assert rn == rn_ref and rn == float(r.abs().max())


def test_noalloc_residual_strided_and_limits(M):
    """lda > n (a sub-block of a larger matrix) and the size limit."""
    say("noalloc residual lda > n, limits")
    n, lda = 777, 1024
    full = torch.from_numpy(np.random.default_rng(9).standard_normal((n, lda))).to(DEV)
    b = torch.ones(n, dtype=torch.float64, device=DEV)
    x = torch.linspace(-1, 1, n, dtype=torch.float64, device=DEV)
    r_ref, rn_ref = M.residual(full, b, x, M.F64)
    r = torch.empty(n, dtype=torch.float64, device=DEV)
    assert M.residual_noalloc(full, b, x, r, M.F64) == rn_ref
    assert torch.equal(r, r_ref)
    L = M.lib()
    big = M.RESIDUAL_NOALLOC_MAX_N + 1
    rn = C.c_double(0.0)
    p = C.c_void_p(r.data_ptr())
    st = L.mpir_residual_noalloc(big, p, big, M.F64, M.F64, p, p, p, C.byref(rn),
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == M.ERR_ARG
    st = L.mpir_residual_noalloc(n, p, n, M.F64, M.F32, p, p, p, C.byref(rn), None)
    assert st == M.ERR_ARG                                  # TR narrower than TW
