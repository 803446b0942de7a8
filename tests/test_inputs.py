"""Closed-form checks of the workload generators (CPU only).

G is the trapezoid-rule discretisation of the Green's operator of -d^2/dx^2 on
[0,1] (paper, section "Integral Equations Example").  On the interior grid
h = 1/(N+1) it is exactly the inverse of T = h^-2 tridiag(-1, 2, -1), so its
spectrum is known in closed form, and G*1 = x(1-x)/2 exactly because the
trapezoid rule integrates the piecewise-linear kernel exactly.
"""
import numpy as np
import pytest

from paper_2311_14616_amd import inputs as I


def _tridiag(n):
    h = 1.0 / (n + 1)
    t = np.zeros((n, n))
    t[np.arange(n), np.arange(n)] = 2.0
    t[np.arange(n - 1), np.arange(1, n)] = -1.0
    t[np.arange(1, n), np.arange(n - 1)] = -1.0
    return t / h**2


@pytest.mark.parametrize("n", [5, 8, 33])
def test_gmat_is_inverse_of_second_difference(n):
    g = np.eye(n) - I.gmat_operator(n, 1.0)          # alpha = 1 -> G = I - A
    err = np.abs(g @ _tridiag(n) - np.eye(n)).max()
    assert err < 64 * n * np.finfo(float).eps


@pytest.mark.parametrize("n", [7, 64, 1000])
def test_gmat_times_ones_closed_form(n):
    h, x = I.gmat_grid(n)
    g = np.eye(n) - I.gmat_operator(n, 1.0)
    assert np.abs(g.sum(axis=1) - x * (1 - x) / 2).max() < 8 * n * np.finfo(float).eps


@pytest.mark.parametrize("alpha", [1.0, 10.0, 100.0])
def test_rhs_closed_form(alpha):
    n = 257
    at = I.gmat_operator(n, alpha)
    b = I.rhs_ones(at)
    _, x = I.gmat_grid(n)
    assert np.abs(b - (1.0 - alpha * x * (1 - x) / 2)).max() < 1e-13 * max(1, alpha)


def test_spectrum_closed_form():
    # eig(I - alpha G) = 1 - alpha h^2 / (4 sin^2(k pi h / 2)), k = 1..N
    n, alpha = 200, 10.0
    h = 1.0 / (n + 1)
    k = np.arange(1, n + 1)
    lam = np.sort(1.0 - alpha * h**2 / (4 * np.sin(k * np.pi * h / 2) ** 2))
    ev = np.sort(np.linalg.eigvalsh(I.gmat_operator(n, alpha)))
    assert np.abs(ev - lam).max() < 1e-12 * alpha


@pytest.mark.slow
def test_condition_number_printed_in_paper():
    # section "Evaluating the residual in extended precision": cond(I - 799 G, Inf)
    # printed as 2.35899e+05 at N = 4096.
    n = 4096
    a = I.gmat_operator(n, 799.0)
    kinf = np.abs(a).sum(1).max() * np.abs(np.linalg.inv(a)).sum(1).max()
    assert abs(kinf - 2.35899e5) / 2.35899e5 < 5e-6


def test_endpoint_grid_has_identity_rows():
    a = I.gmat_operator(16, 3.0, grid="endpoint")
    e = np.zeros(16)
    e[0] = 1.0
    assert np.array_equal(a[0], e) and np.array_equal(a[:, 0], e)


@pytest.mark.parametrize("grid", ["interior", "endpoint"])
def test_torch_generator_bitwise(grid):
    torch = pytest.importorskip("torch")
    n = 300
    a_np = I.gmat_operator(n, 7.5, grid=grid)
    a_t = I.gmat_operator_torch(n, 7.5, "cpu", grid=grid, cols_per_chunk=64).numpy()
    assert np.array_equal(a_np.view(np.uint64), a_t.view(np.uint64))
    b_np = I.rhs_ones(a_np)
    b_t = I.rhs_ones_torch(torch.from_numpy(a_np)).numpy()
    assert np.array_equal(b_np.view(np.uint64), b_t.view(np.uint64))


def test_batched_spec_is_seeded_and_in_range():
    ns, alphas, ds = I.batched_spec()
    ns2, alphas2, ds2 = I.batched_spec()
    assert len(ns) == 4096 and ns.min() >= 32 and ns.max() <= 1024
    assert np.array_equal(ns, ns2) and np.array_equal(alphas, alphas2)
    assert alphas.min() >= 0.5 and alphas.max() <= 5.0
    assert all(len(d) == n for d, n in zip(ds, ns))
    assert min(d.min() for d in ds) >= 0.0 and max(d.max() for d in ds) <= 0.1


def test_batched_system_is_spd():
    ns, alphas, ds = I.batched_spec(count=4, nmin=32, nmax=64)
    for n, al, d in zip(ns, alphas, ds):
        a = I.batched_system(int(n), float(al), d)
        assert np.array_equal(a, a.T)
        assert np.linalg.eigvalsh(a).min() > 0


def test_wilkinson_singular_values():
    n, kappa = 96, 1e6
    at32, b, xstar, sigma = I.wilkinson_operator(n, kappa)
    sv = np.linalg.svd(at32.T.astype(np.float64), compute_uv=False)
    # rounding A to binary32 perturbs each singular value by at most ||dA||_2
    da = np.linalg.norm(at32.astype(np.float64), 2) * 2.0**-24 * n
    assert np.abs(np.sort(sv) - np.sort(sigma)).max() <= da
    assert abs(sigma[0] - 1.0) < 1e-15 and abs(sigma[-1] - 1 / kappa) < 1e-15 / kappa
    assert b.dtype == np.float32


def test_wilkinson_torch_matches_host_generator():
    """The device-side Wilkinson generator gives the same A32 bits as the
    host one (same draws, same elementwise FP64 operations); b agrees to
    FP32 rounding (its FP64 sum runs in another order)."""
    torch = pytest.importorskip("torch")
    for n, kappa in ((7, 1e4), (130, 1e7)):
        at, b, xs, sg = I.wilkinson_operator(n, kappa, seed=5)
        at2, b2, xs2, sg2 = I.wilkinson_operator_torch(n, kappa, "cpu", seed=5, cols_per_chunk=48)
        assert np.array_equal(at, at2.numpy())
        assert np.array_equal(xs, xs2.numpy()) and np.array_equal(sg, sg2.numpy())
        assert np.allclose(b, b2.numpy(), rtol=2e-7, atol=0)


def test_random_dense_is_seeded_column_major():
    a = I.random_dense(5, 3)
    b = I.random_dense(5, 3)
    assert a.shape == (5, 5) and a.flags["C_CONTIGUOUS"] and np.array_equal(a, b)
    c = I.random_dense(5, 3, dtype=np.float32, diag_shift=10.0)
    assert c.dtype == np.float32 and np.all(np.diag(c) > 5.0)
