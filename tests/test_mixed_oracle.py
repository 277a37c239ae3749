"""The mixed-precision reference against its pins (mixed_pins.py), and the
pins against plausible mistakes planted in copies of the reference (CPU
only; the copies are imported from a temporary directory)."""
import importlib.util
import os
import sys

import pytest

import mixed_pins
from oracle import mixed as _mixed

SRC = _mixed.__file__


@pytest.mark.parametrize("pin", mixed_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin(_mixed)


# (name, text in oracle/mixed.py, replacement)
MUTANTS = [
    ("bf16_no_round_to_odd", "u = f.view(np.uint32) | inexact.astype(np.uint32)", "u = f.view(np.uint32)"),
    ("bf16_truncate", "u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000", "u = u & 0xFFFF0000"),
    ("bf16_ties_away", "u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000", "u = (u + 0x8000) & 0xFFFF0000"),
    ("no_rounding", "P = rnd(W[j1:, j0:j1]).astype(acc)", "P = W[j1:, j0:j1].astype(np.float64)"),
    ("update_sign", "W[j1:, j1:] = W[j1:, j1:] - np.tril(prod)", "W[j1:, j1:] = W[j1:, j1:] + np.tril(prod)"),
    ("trsm_transposed", "solve_triangular(Ljj, W[j1:, j0:j1].T, lower=True).T",
     "solve_triangular(Ljj.T, W[j1:, j0:j1].T, lower=False).T"),
    ("scale_one_side", "W = np.tril(W / (d[:, None] * d[None, :]))", "W = np.tril(W / (d[:, None] * d[:, None]))"),
    ("no_unscale", "L = d[:, None] * L", "L = L"),
    ("unscale_columns", "L = d[:, None] * L", "L = d[None, :] * L"),
    ("shift_ignored", "W[np.arange(n), np.arange(n)] += shift", "pass"),
    ("eta_no_b", "den = anorm * np.abs(X).max(axis=0) + np.abs(B).max(axis=0)",
     "den = anorm * np.abs(X).max(axis=0)"),
    ("ir_wrong_sign", "X = X + _plain.solve(L, R)", "X = X - _plain.solve(L, R)"),
    ("pcg_wrong_beta", "beta = np.where(restart | done, 0.0, rz_new / np.where(rz != 0, rz, 1.0))",
     "beta = np.where(restart | done, 0.0, rz / np.where(rz_new != 0, rz_new, 1.0))"),
    ("pcg_alpha_sign", "R = R - alpha[None, :] * Q", "R = R + alpha[None, :] * Q"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    pkg = tmp_path / "oracle_mut"
    pkg.mkdir()
    # the copy imports the plain oracle from the real package
    mutated = src.replace(old, new, 1).replace("from . import oracle as _plain", "from oracle import oracle as _plain")
    (pkg / "mixed_mut.py").write_text(mutated)
    spec = importlib.util.spec_from_file_location(f"mixed_mut_{name}", str(pkg / "mixed_mut.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = []
    for pin in mixed_pins.ALL_PINS:
        try:
            pin(mod)
        except AssertionError:
            caught.append(pin.__name__)
        except Exception as e:  # a crash of the mutant also counts as caught
            caught.append(f"{pin.__name__}:{type(e).__name__}")
        if caught:
            break
    assert caught, f"no pin caught mutant {name}"
