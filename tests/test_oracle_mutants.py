"""Plant plausible mistakes in copies of the oracle source and check that the
pins catch every one of them.  Everything here runs on the CPU: the mutants
are compiled with gcc into a temporary directory and never touch the HIP
library."""
import ctypes
import os

import pytest

import oracle
import oracle_pins
from oracle import oracle as _oracle_mod

SRC = os.path.join(os.path.dirname(oracle.lib_path), "oracle.c")

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("sign_update", "ai[k] = ai[k] - lij * AT(a, k, j, lda)", "ai[k] = ai[k] + lij * AT(a, k, j, lda)"),
    ("transposed_operand", "ai[k] = ai[k] - lij * AT(a, k, j, lda)", "ai[k] = ai[k] - lij * AT(a, j, k, lda)"),
    ("dropped_diag_update", "for (int64_t k = j + 1; k <= i; ++k)", "for (int64_t k = j + 1; k < i; ++k)"),
    ("shifted_update_start", "for (int64_t k = j + 1; k <= i; ++k)", "for (int64_t k = j + 2; k <= i; ++k)"),
    ("multiply_not_divide", "AT(a, i, j, lda) = AT(a, i, j, lda) / ljj;", "AT(a, i, j, lda) = AT(a, i, j, lda) * ljj;"),
    ("missing_sqrt", "double ljj = sqrt(d);", "double ljj = d;"),
    ("info_off_by_one", "if (!(d > 0.0)) { *info = j + 1; return 0; }\n    double ljj",
     "if (!(d > 0.0)) { *info = j; return 0; }\n    double ljj"),
    ("accepts_zero_pivot", "if (!(d > 0.0)) { *info = j + 1; return 0; }\n    double ljj",
     "if (d < 0.0) { *info = j + 1; return 0; }\n    double ljj"),
    ("crout_dropped_term", "for (int64_t k = 0; k < j; ++k) s = s - li[k] * lj[k];",
     "for (int64_t k = 1; k < j; ++k) s = s - li[k] * lj[k];"),
    ("crout_wrong_index", "for (int64_t k = 0; k < j; ++k) s = s - li[k] * lj[k];",
     "for (int64_t k = 0; k < j; ++k) s = s - li[k] * li[k];"),
    ("solve_forward_transposed", "s = s - AT(l, i, k, lda) * AT(b, k, c, ldb);", "s = s - AT(l, k, i, lda) * AT(b, k, c, ldb);"),
    ("solve_backward_transposed", "s = s - AT(l, k, i, lda) * AT(b, k, c, ldb);\n      AT(b, i, c, ldb) = s / AT(l, i, i, lda);\n    }\n  }",
     "s = s - AT(l, i, k, lda) * AT(b, k, c, ldb);\n      AT(b, i, c, ldb) = s / AT(l, i, i, lda);\n    }\n  }"),
    ("solve_sign", "s = s - AT(l, i, k, lda) * AT(b, k, c, ldb);", "s = s + AT(l, i, k, lda) * AT(b, k, c, ldb);"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    csrc = tmp_path / "oracle_mut.c"
    csrc.write_text(mutated)
    so = str(tmp_path / "liboracle_mut.so")
    oracle.build(str(csrc), so)
    lib = _oracle_mod._load(so)
    caught = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(lib)
        except AssertionError:
            caught.append(pin.__name__)
        except Exception as e:  # a crash of the mutant also counts as caught
            caught.append(f"{pin.__name__}:{type(e).__name__}")
    assert caught, f"no pin caught mutant {name}"


# Mistakes planted in the acceptance measures of oracle/oracle.py
# (name, text in oracle.py, replacement); the measure pins must catch each.
PY_SRC = _oracle_mod.__file__
PY_MUTANTS = [
    ("erow_no_sqrt", "d = np.sqrt(np.diag(np.asarray(A, dtype=np.float64)))",
     "d = np.diag(np.asarray(A, dtype=np.float64))"),
    ("erow_column_scaled", "(np.abs(Lt - Lr) / d[:, None])", "(np.abs(Lt - Lr) / d[None, :])"),
    ("erow_signed", "(np.abs(Lt - Lr) / d[:, None])", "((Lt - Lr) / d[:, None])"),
    ("erow_reads_upper", "Lt = np.tril(np.asarray(L_test, dtype=np.float64))",
     "Lt = np.asarray(L_test, dtype=np.float64)"),
    ("rho_no_n", "(n * U64 * np.linalg.norm(As))", "(U64 * np.linalg.norm(As))"),
    ("rho_no_u", "(n * U64 * np.linalg.norm(As))", "(n * np.linalg.norm(As))"),
    ("rho_dbl_epsilon", "U64 = 2.0 ** -53", "U64 = 2.0 ** -52"),
    ("rho_max_norm", "return float(np.linalg.norm(R) / (n * U64", "return float(np.abs(R).max() / (n * U64"),
    ("rho_no_completion", "As = _sym_from_lower(np.asarray(A, dtype=np.float64))\n    Lt = np.tril",
     "As = np.asarray(A, dtype=np.float64)\n    Lt = np.tril"),
    ("rho_reads_upper_L", "Lt = np.tril(np.asarray(L, dtype=np.float64))", "Lt = np.asarray(L, dtype=np.float64)"),
    ("completion_doubles_diag", "return low + np.tril(A, -1).T", "return low + np.tril(A).T"),
    ("eta_no_b", "den = anorm * np.abs(X2[:, c]).max() + np.abs(B2[:, c]).max()",
     "den = anorm * np.abs(X2[:, c]).max()"),
    ("eta_one_norms", "den = anorm * np.abs(X2[:, c]).max() + np.abs(B2[:, c]).max()",
     "den = anorm * np.abs(X2[:, c]).sum() + np.abs(B2[:, c]).sum()"),
    ("eta_global_x", "den = anorm * np.abs(X2[:, c]).max()", "den = anorm * np.abs(X2).max()"),
    ("eta_entry_norm", "anorm = np.abs(As).sum(axis=1).max()", "anorm = np.abs(As).max()"),
    ("eta_first_column", "worst = max(worst, float(", "worst = worst if c else (0.0 + float("),
]


@pytest.mark.parametrize("name,old,new", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_measure_pins_catch_mutant(name, old, new, tmp_path):
    import importlib.util

    import measure_pins

    src = open(PY_SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = tmp_path / "oracle_py_mut.py"
    path.write_text(src.replace(old, new, 1))
    spec = importlib.util.spec_from_file_location(f"oracle_py_mut_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = []
    for pin in measure_pins.ALL_PINS:
        try:
            pin(mod)
        except AssertionError:
            caught.append(pin.__name__)
        except Exception as e:  # a crash of the mutant also counts as caught
            caught.append(f"{pin.__name__}:{type(e).__name__}")
    assert caught, f"no pin caught mutant {name}"
