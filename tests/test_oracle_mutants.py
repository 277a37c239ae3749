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
