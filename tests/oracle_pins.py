"""Pins that tie the CPU oracle to facts other than itself.

Each pin is a plain function taking the oracle's ctypes library handle (so the
same checks can be run against deliberately broken builds of the oracle in
test_oracle_mutants.py) and raising AssertionError on failure.  The pins are
chosen so that a dropped term, a wrong sign, a wrong index or a transposed
operand in the oracle makes at least one of them fail.

What pins what:
  golden_*          closed-form worked examples of the POTRF definition
                    (Methods) stored under tests/golden/;
  pascal            the symmetric Pascal matrix S_ij = C(i+j, i) has the lower
                    Pascal matrix L_ij = C(i, j) as its Cholesky factor
                    (Edelman and Strang, "Pascal Matrices", 2004);
  minij             A_ij = min(i, j) (1-based) has the all-ones lower
                    triangle as its factor;
  identity/diagonal special cases that reduce to elementwise sqrt;
  integer_factor    A = L0 L0^T with integer L0: exact arithmetic, so L0 is
                    returned bit for bit;
  mpmath            60-digit Cholesky from mpmath within a normwise forward
                    error bound c n u kappa(A);
  residual          ||A - L L^T||_F / (n u ||A||_F) <= 10 with u = 2^-53;
  non_spd           first failing pivot reported as info = j + 1;
  upper_untouched   the strict upper triangle is never read or written;
  crout             the two oracle forms agree bit for bit;
  leading_block     chol(A[:m,:m]) equals L[:m,:m] bit for bit;
  solve_*           exact integer solve and backward error <= 1e-12.
"""
from __future__ import annotations

import math
import os

import numpy as np

import oracle
from paper_2606_11937_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name: str):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    n = int(rows[0][0])
    A = np.array([[float(v) for v in r] for r in rows[1:1 + n]])
    L = np.array([[float(v) for v in r] for r in rows[1 + n:1 + 2 * n]])
    return A, L


def _ulps(x: np.ndarray, y: np.ndarray) -> float:
    return float(np.max(np.abs(x - y) / np.spacing(np.maximum(np.abs(y), 1e-300))))


def pin_golden_exact(lib):
    for name in ("chol_2x2_exact.txt", "chol_3x3_exact.txt"):
        A, L = read_golden(name)
        got, info = oracle.potrf(A, lib)
        assert info == 0, (name, info)
        assert np.array_equal(np.tril(got), L), (name, got)


def pin_golden_irrational(lib):
    A, L = read_golden("chol_2x2_irrational.txt")
    got, info = oracle.potrf(A, lib)
    assert info == 0
    assert _ulps(np.tril(got), L) <= 1.0, got


def pin_pascal(lib):
    n = 20
    S = np.array([[math.comb(i + j, i) for j in range(n)] for i in range(n)], dtype=np.float64)
    P = np.array([[math.comb(i, j) if j <= i else 0 for j in range(n)] for i in range(n)], dtype=np.float64)
    got, info = oracle.potrf(S, lib)
    assert info == 0
    assert np.array_equal(np.tril(got), P)


def pin_minij(lib):
    n = 37
    i, j = np.indices((n, n))
    A = np.minimum(i, j).astype(np.float64) + 1.0
    got, info = oracle.potrf(A, lib)
    assert info == 0
    assert np.array_equal(np.tril(got), np.tril(np.ones((n, n))))


def pin_identity_diagonal(lib):
    n = 9
    got, info = oracle.potrf(np.eye(n), lib)
    assert info == 0 and np.array_equal(np.tril(got), np.eye(n))
    d = np.array([4.0, 9.0, 2.0, 0.25, 1e-8, 3.0, 1e10, 7.0, 0.5])
    got, info = oracle.potrf(np.diag(d), lib)
    assert info == 0 and np.array_equal(np.tril(got), np.diag(np.sqrt(d)))


def pin_integer_factor(lib):
    for n, seed, band in ((1, 0, None), (5, 1, None), (64, 2, None), (97, 3, 4)):
        A, L0 = inputs.integer_factor(n, seed=seed, band=band)
        got, info = oracle.potrf(A, lib)
        assert info == 0
        assert np.array_equal(np.tril(got), L0), (n, seed)


def pin_mpmath(lib):
    import mpmath
    mpmath.mp.dps = 60
    for n, seed in ((6, 11), (24, 12), (48, 13)):
        A = inputs.gg_plus_identity(n, seed=seed)
        Lm = mpmath.cholesky(mpmath.matrix(A.tolist()))
        Lx = np.array([[float(Lm[r, c]) for c in range(n)] for r in range(n)])
        got, info = oracle.potrf(A, lib)
        assert info == 0
        kappa = np.linalg.cond(A)
        err = np.abs(np.tril(got) - Lx).max() / np.abs(Lx).max()
        assert err <= 10 * n * oracle.U64 * kappa, (n, err)


def pin_residual(lib):
    for n, gen in ((200, "gg"), (160, "se")):
        A = inputs.gg_plus_identity(n, seed=5) if gen == "gg" else inputs.se_kernel(n, seed=6)
        got, info = oracle.potrf(A, lib)
        assert info == 0
        rho = oracle.scaled_residual(A, got)
        assert rho <= 10.0, (gen, rho)


def pin_non_spd(lib):
    # indefinite diagonal: the third pivot is the first non-positive one
    A = np.diag([1.0, 2.0, -3.0, 4.0])
    _, info = oracle.potrf(A, lib)
    assert info == 3, info
    # a leading minor of order 4 is singular: A = L0 L0^T with row 3 replaced so
    # that a_33 equals the sum of squares already removed (pivot exactly 0)
    Aint, L0 = inputs.integer_factor(7, seed=4)
    B = Aint.copy()
    B[3, 3] = float(np.sum(L0[3, :3] ** 2))
    _, info = oracle.potrf(B, lib)
    assert info == 4, info
    # NaN on the diagonal is a failing pivot too
    C = np.eye(5)
    C[1, 1] = np.nan
    _, info = oracle.potrf(C, lib)
    assert info == 2, info


def pin_upper_untouched(lib):
    A = inputs.gg_plus_identity(33, seed=7)
    Am = A.copy()
    Am[np.triu_indices(33, 1)] = np.nan  # strict upper is garbage; must not be read
    got, info = oracle.potrf(Am, lib)
    assert info == 0
    ref, _ = oracle.potrf(A, lib)
    assert np.array_equal(np.tril(got), np.tril(ref))
    assert np.all(np.isnan(got[np.triu_indices(33, 1)]))


def pin_crout(lib):
    for n, seed in ((1, 0), (31, 8), (130, 9)):
        A = inputs.gg_plus_identity(n, seed=seed)
        a, ia = oracle.potrf(A, lib)
        b, ib = oracle.potrf_crout(A, lib)
        assert ia == ib == 0
        assert np.array_equal(np.tril(a), np.tril(b))
    Aint, L0 = inputs.integer_factor(40, seed=10)
    b, ib = oracle.potrf_crout(Aint, lib)
    assert ib == 0 and np.array_equal(np.tril(b), L0)
    b, ib = oracle.potrf_crout(np.diag([1.0, -1.0]), lib)
    assert ib == 2


def pin_leading_block(lib):
    A = inputs.gg_plus_identity(150, seed=14)
    full, _ = oracle.potrf(A, lib)
    for m in (1, 17, 64, 149):
        part, _ = oracle.potrf(A[:m, :m], lib)
        assert np.array_equal(np.tril(part), np.tril(full[:m, :m])), m


def pin_solve_exact(lib):
    # A = L0 L0^T with unit-diagonal integer L0 and integer x: every step of
    # both substitutions is exact, so x comes back exactly.
    rng = np.random.default_rng(15)
    A, L0 = inputs.integer_factor(50, seed=15, diag_max=1, band=3)
    X = rng.integers(-5, 6, size=(50, 3)).astype(np.float64)
    B = A @ X
    got = oracle.solve(L0, B, lib)
    assert np.array_equal(got, X)


def pin_solve_backward(lib):
    A = inputs.gg_plus_identity(120, seed=16)
    B = np.random.default_rng(17).standard_normal((120, 4))
    L, info = oracle.potrf(A, lib)
    assert info == 0
    X = oracle.solve(L, B, lib)
    assert oracle.backward_error(A, X, B) <= 1e-12
    # cross-check against an independent LAPACK solve
    Xs = np.linalg.solve(A, B)
    assert np.abs(X - Xs).max() <= 1e-12 * np.abs(Xs).max() * np.linalg.cond(A)


def pin_lapack_crosscheck(lib):
    import scipy.linalg
    A = inputs.se_kernel(300, seed=18)
    got, info = oracle.potrf(A, lib)
    assert info == 0
    ref = scipy.linalg.cholesky(A, lower=True)
    assert oracle.row_scaled_error(got, ref, A) <= 1e-13


ALL_PINS = [
    pin_golden_exact, pin_golden_irrational, pin_pascal, pin_minij,
    pin_identity_diagonal, pin_integer_factor, pin_mpmath, pin_residual,
    pin_non_spd, pin_upper_untouched, pin_crout, pin_leading_block,
    pin_solve_exact, pin_solve_backward, pin_lapack_crosscheck,
]
