"""Pins of the oracle's acceptance measures (scaled_residual,
backward_error, row_scaled_error): hand-worked examples stored under
tests/golden/ with their derivations, plus invariants that hold for any
correct implementation.

Each pin takes the module that provides the measures (so
test_oracle_mutants.py can run the same checks against copies of
oracle/oracle.py with planted mistakes) and raises AssertionError on failure.

What pins what:
  row_scaled_by_hand  e_row on a 2x2 with exact row norms 2 and 5 and a
                      known difference (golden/measure_row_scaled_error.txt);
  residual_by_hand    rho on a 2x2 whose residual is exactly 2^-39 [[0,-1],
                      [-1,-3]] (golden/measure_scaled_residual.txt);
  eta_by_hand         eta on a 2x2 with two right-hand sides whose worst
                      column is not the one with the largest ||x||
                      (golden/measure_backward_error.txt);
  exact_cases         an exact integer factor has rho = 0 and e_row = 0 against
                      itself, an exact solution has eta = 0;
  scale_invariance    rho and eta are unchanged when A (and b) are scaled by a
                      power of two and L (and x) accordingly.
"""
from __future__ import annotations

import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_measure_golden(name: str) -> dict:
    """Keyed rows of a measure fixture: `key v1 v2 ...` (floats, hex allowed)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out[key] = np.array([float.fromhex(v) if v.startswith(("0x", "-0x")) else float(v) for v in vals])
    return out


def _close(got: float, want: float, rel: float = 1e-14) -> bool:
    return abs(got - want) <= rel * abs(want)


def pin_row_scaled_by_hand(m):
    g = read_measure_golden("measure_row_scaled_error.txt")
    A, Lr, Lt = (g[k].reshape(2, 2) for k in ("A", "Lref", "Ltest"))
    got = m.row_scaled_error(Lt, Lr, A)
    assert got == g["expect"][0], got


def pin_residual_by_hand(m):
    g = read_measure_golden("measure_scaled_residual.txt")
    A, L = g["A"].reshape(2, 2), g["L"].reshape(2, 2)
    want = 2.0 ** 13 * math.sqrt(11.0 / 713.0)  # the closed form of the derivation
    assert _close(want, g["expect"][0], 1e-15)
    got = m.scaled_residual(A, L)
    assert _close(got, want), got


def pin_eta_by_hand(m):
    g = read_measure_golden("measure_backward_error.txt")
    A, X, B = (g[k].reshape(2, 2) for k in ("A", "X", "B"))
    got = m.backward_error(A, X, B)
    assert got == g["expect"][0], got
    # the worst column last: the maximum is over all columns
    assert m.backward_error(A, X[:, ::-1], B[:, ::-1]) == g["expect"][0]
    # column 1 alone: 0.25 / 12
    got1 = m.backward_error(A, X[:, 1:], B[:, 1:])
    assert _close(got1, 0.25 / 12.0), got1


def pin_exact_cases(m):
    # integer L0 with A = L0 L0^T exact in binary64
    L0 = np.array([[2.0, 0, 0, 0], [1, 3, 0, 0], [-1, 2, 4, 0], [0, -2, 1, 1]])
    A = L0 @ L0.T
    assert m.scaled_residual(A, L0) == 0.0
    assert m.row_scaled_error(L0, L0, A) == 0.0
    x = np.array([[1.0, -2.0], [0.5, 3.0], [-1.0, 0.0], [2.0, 1.0]])
    b = A @ x
    assert m.backward_error(A, x, b) == 0.0


def pin_scale_invariance(m):
    rng = np.random.default_rng(11)
    G = rng.standard_normal((6, 6))
    A = G @ G.T / 6 + np.eye(6)
    L = np.linalg.cholesky(A)
    L = L * (1.0 + 1e-9 * rng.standard_normal(L.shape))  # a perturbed factor
    x = rng.standard_normal((6, 2))
    b = A @ x + 1e-6 * rng.standard_normal((6, 2))
    r1, e1 = m.scaled_residual(A, L), m.backward_error(A, x, b)
    assert r1 > 0 and e1 > 0
    # scaling by powers of two is exact: A -> 4 A, L -> 2 L, b -> 4 b
    assert m.scaled_residual(4.0 * A, 2.0 * L) == r1
    assert m.backward_error(4.0 * A, x, 4.0 * b) == e1
    assert m.row_scaled_error(2.0 * L, 2.0 * np.linalg.cholesky(A), 4.0 * A) == m.row_scaled_error(
        L, np.linalg.cholesky(A), A)


ALL_PINS = [pin_row_scaled_by_hand, pin_residual_by_hand, pin_eta_by_hand, pin_exact_cases, pin_scale_invariance]
