"""Seeded synthetic inputs for the iterative-refinement workloads.

This module only builds test and benchmark matrices; it holds none of the
method's arithmetic (no factorization, no solve, no refinement step), so the
CPU oracle and the GPU path can both be fed from it without sharing code.

Storage convention: every matrix is returned in *column-major* storage, i.e.
as an array ``At`` with ``At[j, i] == A[i, j]`` (shape ``(n, n)``, C-contiguous),
which is what the library's C ABI takes (LAPACK/Julia layout, ``lda = n``).

Workloads (paper: section "Integral Equations Example", Gmat; experiments in
"Double-Single Precision" and "Interprecision Transfers: Part II"):

* ``gmat_operator`` -- A = I - alpha*G, G the trapezoid-rule discretisation of
  the Green's operator of -d^2/dx^2 on [0,1] with kernel g(x,y) = x(1-y) for
  x <= y and y(1-x) otherwise.  Grid: interior nodes h = 1/(N+1), x_i = i*h,
  i = 1..N (the endpoint grid h = 1/(N-1), x_i = (i-1)*h, used by some of the
  paper's printed examples, is available as ``grid="endpoint"``; its first and
  last rows are then identity rows because g vanishes at both ends).
  Expression order, fixed so that the NumPy and the torch versions agree bit
  for bit:  xi = (double)i*h;  G_ij = h*(min(xi,xj)*(1.0-max(xi,xj)));
  A_ij = (i==j) - alpha*G_ij.
* ``batched_systems`` -- 4096 uneven systems A_k = I - alpha_k G_{N_k} + D_k.
* ``wilkinson_operator`` -- A = H1 diag(sigma) H2 with Householder reflectors
  from seeded Gaussian vectors, rounded to FP32.

Right-hand sides are b = A*ones unless stated, accumulated in FP64 in
increasing column order (``rhs_ones``).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gmat_grid", "gmat_operator", "gmat_operator_torch", "rhs_ones",
    "rhs_ones_torch", "batched_spec", "batched_systems", "wilkinson_operator",
    "random_dense",
]


def gmat_grid(n: int, grid: str = "interior") -> tuple[float, np.ndarray]:
    """Return (h, x) with x the n quadrature nodes of the chosen grid."""
    if grid == "interior":
        h = 1.0 / (n + 1)
        x = np.arange(1, n + 1, dtype=np.float64) * h
    elif grid == "endpoint":
        h = 1.0 / (n - 1)
        x = np.arange(0, n, dtype=np.float64) * h
    else:
        raise ValueError(f"unknown grid {grid!r}")
    return h, x


def gmat_operator(n: int, alpha: float, grid: str = "interior",
                  dtype=np.float64) -> np.ndarray:
    """Column-major storage of A = I - alpha*G (A is symmetric, so At == A)."""
    h, x = gmat_grid(n, grid)
    mn = np.minimum.outer(x, x)
    mx = np.maximum.outer(x, x)
    g = h * (mn * (1.0 - mx))
    a = np.eye(n, dtype=np.float64) - alpha * g
    return np.ascontiguousarray(a.astype(dtype))


def gmat_operator_torch(n: int, alpha: float, device, grid: str = "interior",
                        cols_per_chunk: int = 2048):
    """Same matrix as ``gmat_operator`` (bit for bit), built on a torch device
    in column chunks so that N = 32768 (8 GiB in FP64) needs no host copy."""
    import torch
    if grid == "interior":
        h = 1.0 / (n + 1)
        x = torch.arange(1, n + 1, dtype=torch.float64, device=device) * h
    elif grid == "endpoint":
        h = 1.0 / (n - 1)
        x = torch.arange(0, n, dtype=torch.float64, device=device) * h
    else:
        raise ValueError(f"unknown grid {grid!r}")
    at = torch.empty((n, n), dtype=torch.float64, device=device)
    for j0 in range(0, n, cols_per_chunk):
        j1 = min(n, j0 + cols_per_chunk)
        xj = x[j0:j1, None]
        mn = torch.minimum(xj, x[None, :])
        mx = torch.maximum(xj, x[None, :])
        g = h * (mn * (1.0 - mx))
        blk = 0.0 - alpha * g
        idx = torch.arange(j0, j1, device=device)
        blk[idx - j0, idx] = 1.0 - alpha * g[idx - j0, idx]
        at[j0:j1] = blk
        del mn, mx, g, blk
    return at


def rhs_ones(at: np.ndarray) -> np.ndarray:
    """b = A*ones in FP64, each b_i summed over j in increasing order.

    ``at`` is column-major storage (At[j, i] = A[i, j]); the loop adds column
    after column, which is the left-to-right order for every row."""
    n = at.shape[1]
    b = np.zeros(n, dtype=np.float64)
    for j in range(at.shape[0]):
        b += at[j].astype(np.float64)
    return b


def rhs_ones_torch(at):
    """Same as ``rhs_ones`` on a torch device (same order, same bits)."""
    import torch
    b = torch.zeros(at.shape[1], dtype=torch.float64, device=at.device)
    for j in range(at.shape[0]):
        b += at[j].to(torch.float64)
    return b


def batched_spec(count: int = 4096, nmin: int = 32, nmax: int = 1024,
                 seed: int = 2311):
    """Sizes, alphas and diagonal shifts of the uneven batch.

    Draw order (one generator): all N_k, then all alpha_k, then the
    concatenated diagonals D_k."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, count)
    alphas = rng.uniform(0.5, 5.0, count)
    diag = rng.uniform(0.0, 0.1, int(ns.sum()))
    offs = np.concatenate([[0], np.cumsum(ns)])
    ds = [diag[offs[k]:offs[k + 1]] for k in range(count)]
    return ns.astype(np.int64), alphas, ds


def batched_system(n: int, alpha: float, d: np.ndarray) -> np.ndarray:
    """Column-major storage of A = (I - alpha*G_n) + diag(d) (symmetric)."""
    a = gmat_operator(n, alpha)
    a[np.arange(n), np.arange(n)] += d
    return a


def batched_systems(count: int = 4096, nmin: int = 32, nmax: int = 1024,
                    seed: int = 2311):
    """Yield (n, At, b) for every system of the uneven batch (host arrays)."""
    ns, alphas, ds = batched_spec(count, nmin, nmax, seed)
    for k in range(count):
        at = batched_system(int(ns[k]), float(alphas[k]), ds[k])
        yield int(ns[k]), at, rhs_ones(at)


def wilkinson_operator(n: int, kappa: float, seed: int = 14616):
    """Ill-conditioned test matrix A = H1 diag(sigma) H2, rounded to FP32.

    H_m = I - 2 v_m v_m^T / (v_m^T v_m) with v1, v2 ~ N(0,1) and the exact
    solution x* ~ N(0,1), drawn in that order from one generator;
    sigma_i = kappa^(-(i-1)/(n-1)).  A is assembled in FP64 from the rank-one
    expansion of the product, then rounded to FP32; b = fl32(A32 * x*) with
    the product in FP64.  Returns (At32 column-major, b32, xstar64, sigma)."""
    rng = np.random.default_rng(seed)
    v1 = rng.standard_normal(n)
    v2 = rng.standard_normal(n)
    xstar = rng.standard_normal(n)
    i = np.arange(n, dtype=np.float64)
    sigma = kappa ** (-(i / (n - 1)))
    c1 = 2.0 / np.dot(v1, v1)
    c2 = 2.0 / np.dot(v2, v2)
    s = np.dot(v1 * sigma, v2)
    # A = S - c2 (S v2) v2^T - c1 v1 (v1^T S) + c1 c2 s v1 v2^T, S = diag(sigma)
    a = (-c2 * np.outer(sigma * v2, v2) - c1 * np.outer(v1, v1 * sigma)
         + (c1 * c2 * s) * np.outer(v1, v2))
    a[np.arange(n), np.arange(n)] += sigma
    a32 = a.astype(np.float32)
    at32 = np.ascontiguousarray(a32.T)
    b = (a32.astype(np.float64) @ xstar).astype(np.float32)
    return at32, b, xstar, sigma


def wilkinson_operator_torch(n: int, kappa: float, device, seed: int = 14616,
                             cols_per_chunk: int = 2048):
    """``wilkinson_operator`` built on a torch device in column chunks (the
    same draws; A32 bit for bit: the same elementwise FP64 operations in the
    same order).  b = fl32(A32 * x*) is summed over columns in increasing
    order in FP64 on the device.  Returns (At32 column-major, b32, xstar64,
    sigma) as device tensors."""
    import torch
    rng = np.random.default_rng(seed)
    v1 = rng.standard_normal(n)
    v2 = rng.standard_normal(n)
    xstar = rng.standard_normal(n)
    i = np.arange(n, dtype=np.float64)
    sigma = kappa ** (-(i / (n - 1)))
    c1 = 2.0 / np.dot(v1, v1)
    c2 = 2.0 / np.dot(v2, v2)
    s = np.dot(v1 * sigma, v2)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    v1t, v2t, sgt, xt = T(v1), T(v2), T(sigma), T(xstar)
    sv2, v1s = sgt * v2t, v1t * sgt
    at = torch.empty((n, n), dtype=torch.float32, device=device)
    b = torch.zeros(n, dtype=torch.float64, device=device)
    for j0 in range(0, n, cols_per_chunk):
        j1 = min(n, j0 + cols_per_chunk)
        # column j of A: rows i -> a[i, j]; stored as at[j, i]
        blk = ((-c2 * (sv2[None, :] * v2t[j0:j1, None])) - c1 * (v1t[None, :] * v1s[j0:j1, None])
               + (c1 * c2 * s) * (v1t[None, :] * v2t[j0:j1, None]))
        idx = torch.arange(j0, j1, device=device)
        blk[idx - j0, idx] += sgt[idx]
        at[j0:j1] = blk.to(torch.float32)
        del blk
    for j in range(n):
        b += at[j].to(torch.float64) * xt[j]
    return at, b.to(torch.float32), xt, sgt


def random_dense(n: int, seed: int, dtype=np.float64, diag_shift: float = 0.0):
    """Gaussian matrix (column-major storage) for generic parity cases."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    if diag_shift:
        a[np.arange(n), np.arange(n)] += diag_shift
    return np.ascontiguousarray(a.T.astype(dtype))
