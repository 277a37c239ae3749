"""Mixed-precision factorization and refinement: plain CPU reference.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the HIP library never does, and the
two share no code.

The paper's factorization is FP64 throughout (Methods, "Tiled Cholesky
Decomposition"; Results).  This module is the reference for the precision
extension built on the same tiled right-looking algorithm (Fig. 1):

  * symmetric diagonal scaling  A^ = D^-1 A D^-1,  D = diag(A)^(1/2), and an
    optional diagonal shift  A^ + sigma I  (the usual remedy when a
    low-precision factorization breaks down; Higham and Pranesh, SIAM J. Sci.
    Comput. 2021);
  * the tile loop of Fig. 1 with POTRF and TRSM in FP64 and the trailing
    SYRK/GEMM products formed from panel entries rounded once to FP32 or
    BF16, each product entry summed in FP32 over the tile width, and the
    product subtracted from FP64 storage;
  * undoing the scaling, L = D L^;
  * two ways of solving A X = B in FP64 with such a factor: classical
    iterative refinement (Wilkinson; Moler 1967) and preconditioned conjugate
    gradients (Hestenes and Stiefel 1952) with L L^T as the preconditioner.

Everything here is plain numpy in FP64 (FP32 only where the method itself
rounds to FP32), slow and written for reading.  The FP64 tile POTRF is the C
oracle; the TRSM is a library triangular solve.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_triangular

from . import oracle as _plain

PRECISIONS = ("fp64", "fp32", "bf16")


# ------------------------------------------------------------------ rounding
def round_fp32(x) -> np.ndarray:
    """Nearest FP32 value, ties to even (IEEE 754 binary32), returned in FP64."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_to_odd_fp32(x) -> np.ndarray:
    """FP32 rounding to odd: truncate toward zero, and if anything was lost
    set the last significand bit.  Rounding this result once more to a format
    at least two bits shorter gives the correctly rounded value (Boldo and
    Melquiond, IEEE Trans. Computers 2008), which avoids double rounding in
    FP64 -> FP32 -> BF16."""
    x = np.asarray(x, dtype=np.float64)
    f = x.astype(np.float32)
    away = np.abs(f.astype(np.float64)) > np.abs(x)
    f = np.where(away, np.nextafter(f, np.float32(0.0)), f).astype(np.float32)
    inexact = f.astype(np.float64) != x
    u = f.view(np.uint32) | inexact.astype(np.uint32)
    return u.view(np.float32)


def round_bf16(x) -> np.ndarray:
    """Nearest BF16 value (8 significant bits, FP32 exponent range), ties to
    even, returned in FP64.  BF16 is the upper half of an FP32 word, so the
    round-to-nearest-even step adds 0x7FFF plus the lowest kept bit and
    clears the low 16 bits."""
    f = round_to_odd_fp32(x)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def rounder(prec: str):
    if prec == "fp64":
        return lambda v: np.asarray(v, dtype=np.float64)
    if prec == "fp32":
        return round_fp32
    if prec == "bf16":
        return round_bf16
    raise ValueError(f"unknown precision {prec!r}")


# ----------------------------------------------------------- scaling, shift
def scale_factors(A: np.ndarray) -> np.ndarray:
    """d_i = sqrt(A_ii).  A non-positive diagonal entry makes A not SPD."""
    dg = np.diag(np.asarray(A, dtype=np.float64)).copy()
    if not np.all(dg > 0):
        raise ValueError("diagonal entry not positive")
    return np.sqrt(dg)


def scaled_shifted(A: np.ndarray, d: np.ndarray | None, shift: float) -> np.ndarray:
    """Lower triangle of D^-1 A D^-1 + shift I (no scaling when d is None):
    entry (i, j) is A_ij / (d_i d_j), the product d_i d_j rounded once."""
    W = np.tril(np.asarray(A, dtype=np.float64))
    if d is not None:
        W = np.tril(W / (d[:, None] * d[None, :]))
    n = W.shape[0]
    W[np.arange(n), np.arange(n)] += shift
    return W


# ---------------------------------------------------------- the factorization
def potrf_mixed(A: np.ndarray, T: int, prec: str = "fp32", shift: float = 0.0, scale: bool = True):
    """Tiled right-looking Cholesky with low-precision trailing products.

    Returns (L, info).  L holds the factor of A + shift D^2 (of A + shift I
    without scaling) in its lower triangle, zeros above; info = 0 on success,
    else the 1-based global column whose pivot was not positive (L is then
    partial).

    Step J (Fig. 1):
      POTRF  L_JJ = chol(A_JJ) in FP64 (the C oracle on the tile);
      TRSM   L_IJ = A_IJ L_JJ^-T in FP64 for every tile row I > J;
      round  P = the entries of L_IJ, I > J, rounded to `prec`;
      update A_IK -= P_I P_K^T for J < K <= I, each product entry summed in
             FP32 (FP64 when prec is fp64) over the tile width, then
             subtracted in FP64.
    """
    rnd = rounder(prec)
    acc = np.float64 if prec == "fp64" else np.float32
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    d = scale_factors(A) if scale else None
    W = scaled_shifted(A, d, shift)
    M = -(-n // T) if n else 0
    info = 0
    for J in range(M):
        j0, j1 = J * T, min(n, (J + 1) * T)
        Ljj, tinfo = _plain.potrf(W[j0:j1, j0:j1])
        if tinfo:
            W[j0:j1, j0:j1] = np.tril(Ljj)
            info = j0 + tinfo
            break
        Ljj = np.tril(Ljj)
        W[j0:j1, j0:j1] = Ljj
        if j1 == n:
            break
        # rows are independent: X L_JJ^T = A_IJ  <=>  L_JJ X^T = A_IJ^T
        W[j1:, j0:j1] = solve_triangular(Ljj, W[j1:, j0:j1].T, lower=True).T
        P = rnd(W[j1:, j0:j1]).astype(acc)
        prod = (P @ P.T).astype(np.float64)
        W[j1:, j1:] = W[j1:, j1:] - np.tril(prod)
    L = np.tril(W)
    if d is not None:
        L = d[:, None] * L
    return L, info


# ------------------------------------------------------------- refinement
def _sym(A: np.ndarray) -> np.ndarray:
    low = np.tril(np.asarray(A, dtype=np.float64))
    return low + np.tril(low, -1).T


def eta_columns(As: np.ndarray, X: np.ndarray, B: np.ndarray, R: np.ndarray | None = None) -> np.ndarray:
    """Normwise backward error of every column: ||r||_inf / (||A||_inf ||x||_inf
    + ||b||_inf), with r = b - A x (computed here unless given)."""
    if R is None:
        R = B - As @ X
    anorm = np.abs(As).sum(axis=1).max()
    den = anorm * np.abs(X).max(axis=0) + np.abs(B).max(axis=0)
    num = np.abs(R).max(axis=0)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def refine_ir(A: np.ndarray, L: np.ndarray, B: np.ndarray, tol: float = 1e-12, max_iter: int = 30):
    """Classical iterative refinement in FP64 with the factor L:
        x_0 = (L L^T)^-1 b;  repeat  r = b - A x,  x <- x + (L L^T)^-1 r
    until every column's backward error is <= tol.  Returns (X, corrections
    applied, final backward error per column)."""
    As = _sym(A)
    B2 = np.asarray(B, dtype=np.float64).reshape(As.shape[0], -1)
    X = _plain.solve(L, B2)
    it = 0
    while True:
        R = B2 - As @ X
        eta = eta_columns(As, X, B2, R)
        if eta.max() <= tol or it == max_iter:
            return X, it, eta
        X = X + _plain.solve(L, R)
        it += 1


def pcg(A: np.ndarray, L: np.ndarray, B: np.ndarray, tol: float = 1e-12, max_iter: int = 200):
    """Preconditioned conjugate gradients in FP64, every column on its own,
    with M = L L^T (Hestenes and Stiefel 1952, preconditioned form):
        x = M^-1 b, r = b - A x, z = M^-1 r, p = z
        repeat: q = A p, alpha = r.z / p.q, x += alpha p, r -= alpha q,
                z = M^-1 r, beta = r.z(new) / r.z(old), p = z + beta p.
    A column stops when the backward error of its recurrence residual is
    <= tol; the true residual b - A x is then recomputed and, if it misses
    tol, replaces the recurrence residual and the column restarts its
    direction (p = z).  Returns (X, iterations of the slowest column, final
    true backward error per column)."""
    As = _sym(A)
    B2 = np.asarray(B, dtype=np.float64).reshape(As.shape[0], -1)
    nrhs = B2.shape[1]
    X = _plain.solve(L, B2)
    R = B2 - As @ X
    eta = eta_columns(As, X, B2, R)
    done = eta <= tol
    Z = _plain.solve(L, R)
    P = Z.copy()
    rz = np.einsum("ij,ij->j", R, Z)
    it = 0
    while not done.all() and it < max_iter:
        it += 1
        Q = As @ P
        pq = np.einsum("ij,ij->j", P, Q)
        alpha = np.where(done, 0.0, rz / np.where(pq != 0, pq, 1.0))
        X = X + alpha[None, :] * P
        R = R - alpha[None, :] * Q
        restart = np.zeros(nrhs, dtype=bool)
        eta_rec = eta_columns(As, X, B2, R)
        for c in range(nrhs):
            if not done[c] and eta_rec[c] <= tol:
                r_true = B2[:, c] - As @ X[:, c]
                e = eta_columns(As, X[:, c:c + 1], B2[:, c:c + 1], r_true[:, None])[0]
                if e <= tol:
                    done[c] = True
                else:
                    R[:, c] = r_true
                    restart[c] = True
        Z = _plain.solve(L, R)
        rz_new = np.einsum("ij,ij->j", R, Z)
        beta = np.where(restart | done, 0.0, rz_new / np.where(rz != 0, rz, 1.0))
        P = Z + beta[None, :] * P
        rz = rz_new
    return X, it, eta_columns(As, X, B2)


def nearest_on_grid(x: float, bits: int) -> float:
    """Nearest number with `bits` significant bits to a finite normal x, ties
    to the even significand: an independent statement of round-to-nearest
    in exact rational arithmetic, for pinning the bit-level rounders."""
    from fractions import Fraction
    if x == 0.0:
        return 0.0
    m, e = math.frexp(abs(x))        # |x| = m 2^e, 1/2 <= m < 1
    step = Fraction(2) ** (e - bits)  # spacing of the grid around |x|
    q = Fraction(abs(x)) / step
    lo = math.floor(q)
    rem = q - lo
    k = lo + 1 if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and lo % 2 == 1) else lo
    return math.copysign(float(k * step), x)
