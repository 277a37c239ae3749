"""Seeded synthetic SPD inputs shared by the oracle and the HIP path.

This module holds input recipes only: no step of the factorization is here.
The paper factors randomly generated SPD matrices (Results, first paragraph)
and motivates the method with Gaussian-process kernels (Introduction); the
recipes below are those workloads at fixed seeds:

  gg_plus_identity(n, seed)   A = G G^T / n + I, G iid N(0,1); spectrum in
                              about [1, 5] (kappa ~ 5).
  se_kernel(n, seed, ...)     squared-exponential kernel on n points uniform
                              in [0,1]^2, A_ij = exp(-|x_i-x_j|^2/(2 l^2)) +
                              nugget * delta_ij (lengthscale 0.1, nugget 1e-2).
  integer_factor(n, seed)     an integer lower-triangular L0 with positive
                              diagonal and A = L0 L0^T computed exactly; every
                              correct FP64 Cholesky returns L0 bit for bit.
  integer_factor_norm4(n, seed)
                              the same with every row of L0 of Euclidean
                              norm 4 (diag(A) = 16), so that diagonal scaling
                              divides by powers of two and L0 / 4 has
                              quarter-integer entries: exact in FP32 and BF16.

  batch_sizes(count, seed, lo, hi)
                              orders log-uniform in [lo, hi]:
                              round(exp(U(ln lo, ln hi))) from numpy's
                              default_rng(seed).
  gg_batch_device(sizes, seed)
                              the G G^T / n + I recipe for every order of a
                              batch, built on the device (matrix i from
                              torch's generator seeded seed * 1000003 + i).

Both sides of a parity test receive the identical FP64 bytes produced here.
"""
from __future__ import annotations

import numpy as np


def gg_plus_identity(n: int, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    A = G @ G.T / n + np.eye(n)
    return np.ascontiguousarray((A + A.T) * 0.5)


def se_points(n: int, seed: int = 1) -> np.ndarray:
    return np.random.default_rng(seed).random((n, 2))


def se_kernel(n: int, seed: int = 1, lengthscale: float = 0.1, nugget: float = 1e-2,
              rows: slice | None = None) -> np.ndarray:
    """SE kernel matrix (or the row block `rows` of it).  Squared distances are
    formed coordinate-wise, never through the |x|^2+|y|^2-2xy expansion, so
    they are never negative."""
    x = se_points(n, seed)
    r = rows if rows is not None else slice(0, n)
    xr = x[r]
    d0 = xr[:, 0:1] - x[None, :, 0]
    d1 = xr[:, 1:2] - x[None, :, 1]
    K = np.exp(-(d0 * d0 + d1 * d1) / (2.0 * lengthscale * lengthscale))
    idx = np.arange(r.start, r.start + xr.shape[0])
    K[np.arange(xr.shape[0]), idx] += nugget
    return np.ascontiguousarray(K)


def se_kernel_device(n: int, seed: int = 1, lengthscale: float = 0.1, nugget: float = 1e-2,
                     device="cuda", lda: int | None = None, block: int = 4096):
    """Same recipe as se_kernel, built row block by row block on the device
    with torch (for n where a host copy would be slow).  Returns an (n, lda)
    float64 tensor whose first n columns hold A; the points come from the
    same numpy seed."""
    import torch
    lda = lda or n
    x = torch.from_numpy(se_points(n, seed)).to(device)
    A = torch.empty((n, lda), dtype=torch.float64, device=device)
    inv = 1.0 / (2.0 * lengthscale * lengthscale)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        d0 = x[r0:r1, 0:1] - x[None, :, 0]
        d1 = x[r0:r1, 1:2] - x[None, :, 1]
        blk = torch.exp(-(d0 * d0 + d1 * d1) * inv)
        ii = torch.arange(r1 - r0, device=device)
        blk[ii, ii + r0] += nugget
        A[r0:r1, :n] = blk
    return A


def integer_factor(n: int, seed: int = 0, diag_max: int = 3, off_max: int = 2,
                   band: int | None = None):
    """Return (A, L0): L0 integer lower triangular, diagonal in [1, diag_max],
    off-diagonals in [-off_max, off_max] (within `band` of the diagonal if
    given), and A = L0 L0^T formed exactly in int64.  Every partial sum of the
    factorization is then an integer far below 2^53, each square root is of a
    perfect square and each division is exact, so any correct FP64 Cholesky
    in any summation order reproduces L0 exactly."""
    rng = np.random.default_rng(seed)
    L0 = rng.integers(-off_max, off_max + 1, size=(n, n), dtype=np.int64)
    L0 = np.tril(L0, -1)
    if band is not None:
        i, j = np.indices((n, n))
        L0[(i - j) > band] = 0
    L0 += np.diag(rng.integers(1, diag_max + 1, size=n, dtype=np.int64))
    A = L0 @ L0.T
    assert np.abs(A).max() < 2 ** 40
    return np.ascontiguousarray(A.astype(np.float64)), np.ascontiguousarray(L0.astype(np.float64))


# (diagonal, off-diagonal magnitudes) of an integer row with squared norm 16
_NORM4_ROWS = [(4, ()), (2, (2, 2, 2)), (3, (2, 1, 1, 1)), (3, (1,) * 7), (1, (3, 2, 1, 1)),
               (2, (1,) * 12), (1, (2, 2, 2, 1, 1, 1))]


def integer_factor_norm4(n: int, seed: int = 0):
    """Return (A, L0) with L0 integer lower triangular, positive diagonal,
    every row of squared norm 16, off-diagonal entries at random earlier
    columns with random signs, and A = L0 L0^T exact (so diag(A) = 16 and
    |A_ij| <= 16)."""
    rng = np.random.default_rng(seed)
    L0 = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        fits = [r for r in _NORM4_ROWS if len(r[1]) <= i]
        dg, offs = fits[int(rng.integers(len(fits)))]
        L0[i, i] = dg
        if offs:
            cols = rng.choice(i, size=len(offs), replace=False)
            L0[i, cols] = np.array(offs) * rng.choice([-1, 1], size=len(offs))
    A = L0 @ L0.T
    return np.ascontiguousarray(A.astype(np.float64)), np.ascontiguousarray(L0.astype(np.float64))


def batch_sizes(count: int, seed: int = 3, lo: int = 32, hi: int = 2048) -> list[int]:
    u = np.random.default_rng(seed).uniform(np.log(lo), np.log(hi), size=count)
    return [int(v) for v in np.rint(np.exp(u))]


def gg_batch_device(sizes, seed: int = 3, device="cuda"):
    """A_i = G_i G_i^T / n_i + I (symmetrised), G_i iid N(0,1) from torch's
    generator on `device` seeded seed * 1000003 + i; returns a list of
    contiguous (n_i, n_i) float64 tensors."""
    import torch
    out = []
    for i, n in enumerate(sizes):
        g = torch.Generator(device=device)
        g.manual_seed(seed * 1000003 + i)
        G = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
        A = G @ G.T / n
        A = (A + A.T) * 0.5
        A += torch.eye(n, dtype=torch.float64, device=device)
        out.append(A.contiguous())
    return out
