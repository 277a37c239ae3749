"""Pins that tie the mixed-precision reference (oracle/mixed.py) to facts
other than itself.

Each pin takes the module under test (so test_mixed_oracle.py can run the
same checks against copies of the module with planted mistakes) and raises
AssertionError on failure.

What pins what:
  rounding_golden     hand-worked round-to-nearest-even cases from binary64
                      to binary32 and bfloat16, including the double-rounding
                      trap (tests/golden/rounding_bf16_fp32.txt);
  rounding_bruteforce both rounders against nearest_on_grid, an exact
                      rational statement of round-to-nearest-even;
  integer_exact       A = L0 L0^T with integer rows of norm 4: scaling divides
                      by powers of two and every operand and partial sum is
                      exact in FP32 and BF16, so L0 comes back bit for bit
                      in every precision, tile size and with/without scaling;
  fp64_is_plain       in FP64 the tiled form is a regrouping of the plain
                      definition: within 1e-13 (row-scaled) of the C oracle;
  shift               chol(A + s D^2) (chol(A + s I) unscaled) equals the C
                      oracle on the shifted matrix, in FP64;
  scale_power_of_two  L(4A) = 2 L(A) bit for bit (scaling absorbs the factor);
  rounding_applied    the factor error against FP64 is of the order of the
                      precision's unit roundoff on a well-conditioned matrix
                      (so the rounding really happens, at the right width);
  eta_by_hand         the backward-error formula on a 2x2 worked example;
  ir_exact            refinement with the exact factor applies no correction;
  ir_converges        an FP32 factor reaches eta <= 1e-12 in a few
                      corrections;
  cg_finite           with M = I, CG on a matrix with three distinct
                      eigenvalues converges in three steps (exact-arithmetic
                      property of Krylov methods), to rounding;
  pcg_exact           PCG with the exact factor needs no iteration.
"""
from __future__ import annotations

import os

import numpy as np

import oracle
from paper_2606_11937_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rounding_bf16_fp32.txt")


def _plain_factor(A):
    L, info = oracle.potrf(A)
    assert info == 0
    return np.tril(L)


def pin_rounding_golden(mx):
    for line in open(GOLDEN):
        f = line.split("#")[0].split()
        if not f:
            continue
        x, want = float.fromhex(f[1]), float.fromhex(f[2])
        rnd = mx.round_bf16 if f[0] == "bf16" else mx.round_fp32
        got = float(rnd(np.array([x]))[0])
        assert got == want, f"{f[0]}({f[1]}) = {got.hex()}, expected {want.hex()}"


def pin_rounding_bruteforce(mx):
    rng = np.random.default_rng(11)
    x = rng.standard_normal(400) * np.exp2(rng.integers(-30, 30, 400))
    # values one FP64 ulp either side of BF16 halfway points, and the halfway points
    base = mx.round_bf16(rng.standard_normal(100))
    half = base + np.spacing(base.astype(np.float32)).astype(np.float64) * 2 ** 15
    x = np.concatenate([x, half, np.nextafter(half, np.inf), np.nextafter(half, -np.inf)])
    for v in x:
        assert mx.round_bf16(np.array([v]))[0] == mx.nearest_on_grid(float(v), 8), v.hex()
        assert mx.round_fp32(np.array([v]))[0] == mx.nearest_on_grid(float(v), 24), v.hex()


def pin_integer_exact(mx):
    A, L0 = inputs.integer_factor_norm4(130, seed=3)
    for prec in ("fp64", "fp32", "bf16"):
        for T in (32, 100):
            for scale in (True, False):
                L, info = mx.potrf_mixed(A, T, prec, scale=scale)
                assert info == 0
                assert np.array_equal(L, L0), (prec, T, scale)


def pin_fp64_is_plain(mx):
    A = inputs.se_kernel(300, seed=1)
    L64 = _plain_factor(A)
    for scale in (False, True):
        L, info = mx.potrf_mixed(A, 64, "fp64", scale=scale)
        assert info == 0
        assert oracle.row_scaled_error(L, L64, A) <= 1e-13, scale


def pin_shift(mx):
    A = inputs.gg_plus_identity(200, seed=4)
    s = 0.37
    L, _ = mx.potrf_mixed(A, 48, "fp64", shift=s, scale=False)
    ref = _plain_factor(A + s * np.eye(200))
    assert oracle.row_scaled_error(L, ref, A) <= 1e-13
    L, _ = mx.potrf_mixed(A, 48, "fp64", shift=s, scale=True)
    ref = _plain_factor(A + s * np.diag(np.diag(A)))
    assert oracle.row_scaled_error(L, ref, A) <= 1e-13


def pin_scale_power_of_two(mx):
    A = inputs.se_kernel(200, seed=5)
    for prec in ("fp32", "bf16"):
        L1, _ = mx.potrf_mixed(A, 64, prec, shift=0.05)
        L4, _ = mx.potrf_mixed(4.0 * A, 64, prec, shift=0.05)
        assert np.array_equal(L4, 2.0 * L1), prec


def pin_rounding_applied(mx):
    A = inputs.gg_plus_identity(256, seed=6)
    L64 = _plain_factor(A)
    e32 = oracle.row_scaled_error(mx.potrf_mixed(A, 64, "fp32")[0], L64, A)
    e16 = oracle.row_scaled_error(mx.potrf_mixed(A, 64, "bf16")[0], L64, A)
    assert 1e-9 <= e32 <= 1e-5, e32          # u32 = 6e-8
    assert 1e-5 <= e16 <= 1e-1, e16          # u_bf16 = 3.9e-3
    assert e16 > 100 * e32


def pin_eta_by_hand(mx):
    # A = [[2,1],[1,3]], x = (1,1), b = (3.5, 4): r = (0.5, 0),
    # ||A||_inf = 4, ||x||_inf = 1, ||b||_inf = 4  =>  eta = 0.5 / 8
    As = np.array([[2.0, 1.0], [1.0, 3.0]])
    eta = mx.eta_columns(As, np.array([[1.0], [1.0]]), np.array([[3.5], [4.0]]))
    assert eta[0] == 0.0625, eta


def pin_ir_exact(mx):
    A = inputs.gg_plus_identity(128, seed=7)
    B = np.random.default_rng(8).standard_normal((128, 3))
    X, it, eta = mx.refine_ir(A, _plain_factor(A), B)
    assert it == 0 and eta.max() <= 1e-15


def pin_ir_converges(mx):
    A = inputs.se_kernel(384, seed=1)
    B = np.random.default_rng(2).standard_normal((384, 4))
    L, info = mx.potrf_mixed(A, 64, "fp32")
    assert info == 0
    X, it, eta = mx.refine_ir(A, L, B)
    assert eta.max() <= 1e-12 and 1 <= it <= 4, (it, eta.max())
    Xref = oracle.solve(_plain_factor(A), B)
    assert oracle.backward_error(A, X, B) <= 1e-12
    assert np.abs(X - Xref).max() / np.abs(Xref).max() <= 1e-8


def pin_cg_finite(mx):
    n = 60
    Q, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((n, n)))
    lam = np.array([1.0, 2.0, 5.0] * (n // 3))
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    B = np.random.default_rng(10).standard_normal((n, 2))
    X, it, eta = mx.pcg(A, np.eye(n), B, tol=1e-13)
    assert eta.max() <= 1e-13 and it <= 4, (it, eta.max())


def pin_pcg_exact(mx):
    A = inputs.gg_plus_identity(96, seed=12)
    B = np.random.default_rng(13).standard_normal((96, 2))
    X, it, eta = mx.pcg(A, _plain_factor(A), B)
    assert it == 0 and eta.max() <= 1e-15


# cheapest first (the mutant test stops at the first pin that fails)
ALL_PINS = [pin_rounding_golden, pin_rounding_bruteforce, pin_eta_by_hand, pin_cg_finite, pin_pcg_exact,
            pin_ir_exact, pin_rounding_applied, pin_ir_converges, pin_fp64_is_plain, pin_shift,
            pin_scale_power_of_two, pin_integer_exact]
