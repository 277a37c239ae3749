"""ctypes binding of the plain C FP64 oracle (test infrastructure only).

Nothing on the product path imports this module.  Every routine copies its
input, so callers keep their arrays.

Routines
  potrf(A)        right-looking unblocked Cholesky of the lower triangle
                  (Methods, POTRF definition with tile size 1).
  potrf_crout(A)  row-oriented form, same subtraction sequence (bitwise equal).
  solve(L, B)     forward then backward substitution, A X = B with A = L L^T.
  scaled_residual, backward_error, row_scaled_error
                  the acceptance measures used by the parity tests.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
lib_path = os.path.join(_HERE, "liboracle.so")

# No fused multiply-add and no fast-math: the rounding sequence is the plain
# IEEE one written in the source.
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c99"]


def build(src: str = _SRC, out: str = lib_path) -> str:
    """Compile the oracle with gcc into a shared library and return its path."""
    cmd = ["gcc", *CFLAGS, src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def _load(path: str | None = None):
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(lib_path):
            build()
        _lib = _bind(ctypes.CDLL(lib_path))
    return _lib


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    i64 = ctypes.c_int64
    lib.oracle_potrf.argtypes = [dp, i64, i64, ctypes.POINTER(i64)]
    lib.oracle_potrf.restype = ctypes.c_int
    lib.oracle_potrf_crout.argtypes = [dp, i64, i64, ctypes.POINTER(i64)]
    lib.oracle_potrf_crout.restype = ctypes.c_int
    lib.oracle_solve.argtypes = [dp, i64, i64, dp, i64, i64]
    lib.oracle_solve.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _factor(fn_name: str, A: np.ndarray, lib=None):
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    n = A.shape[0]
    info = ctypes.c_int64(0)
    lib = lib or _load()
    getattr(lib, fn_name)(_ptr(A), n, max(n, 1), ctypes.byref(info))
    return A, int(info.value)


def potrf(A: np.ndarray, lib=None):
    """Return (L_inplace, info).  Lower triangle holds L; strict upper is A's."""
    return _factor("oracle_potrf", A, lib)


def potrf_crout(A: np.ndarray, lib=None):
    return _factor("oracle_potrf_crout", A, lib)


def solve(L: np.ndarray, B: np.ndarray, lib=None) -> np.ndarray:
    """Return X with (L L^T) X = B, reading L from the lower triangle."""
    L = np.ascontiguousarray(L, dtype=np.float64)
    B = np.array(B, dtype=np.float64, order="C", copy=True)
    vec = B.ndim == 1
    if vec:
        B = B.reshape(-1, 1).copy()
    n, nrhs = B.shape
    lib = lib or _load()
    lib.oracle_solve(_ptr(L), n, L.shape[1], _ptr(B), nrhs, nrhs)
    return B.reshape(-1) if vec else B


def num_threads(lib=None) -> int:
    return int((lib or _load()).oracle_num_threads())


# ---------------------------------------------------------------- measures
U64 = 2.0 ** -53  # unit roundoff of IEEE binary64 (round to nearest)


def _sym_from_lower(A: np.ndarray) -> np.ndarray:
    low = np.tril(A)
    return low + np.tril(A, -1).T


def scaled_residual(A: np.ndarray, L: np.ndarray) -> float:
    """||A - L L^T||_F / (n u ||A||_F) with A the symmetric completion of its
    lower triangle and u = 2^-53."""
    n = A.shape[0]
    As = _sym_from_lower(np.asarray(A, dtype=np.float64))
    Lt = np.tril(np.asarray(L, dtype=np.float64))
    R = As - Lt @ Lt.T
    return float(np.linalg.norm(R) / (n * U64 * np.linalg.norm(As)))


def backward_error(A: np.ndarray, X: np.ndarray, B: np.ndarray) -> float:
    """max over right-hand sides of ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)."""
    As = _sym_from_lower(np.asarray(A, dtype=np.float64))
    X2 = np.asarray(X, dtype=np.float64).reshape(As.shape[0], -1)
    B2 = np.asarray(B, dtype=np.float64).reshape(As.shape[0], -1)
    R = B2 - As @ X2
    anorm = np.abs(As).sum(axis=1).max()
    worst = 0.0
    for c in range(X2.shape[1]):
        den = anorm * np.abs(X2[:, c]).max() + np.abs(B2[:, c]).max()
        worst = max(worst, float(np.abs(R[:, c]).max() / den) if den > 0 else 0.0)
    return worst


def row_scaled_error(L_test: np.ndarray, L_ref: np.ndarray, A: np.ndarray) -> float:
    """max_{i>=j} |L~_ij - L_ij| / sqrt(A_ii).  sqrt(A_ii) is the 2-norm of row
    i of L, so it bounds every |L_ij| in that row."""
    Lt = np.tril(np.asarray(L_test, dtype=np.float64))
    Lr = np.tril(np.asarray(L_ref, dtype=np.float64))
    d = np.sqrt(np.diag(np.asarray(A, dtype=np.float64)))
    return float((np.abs(Lt - Lr) / d[:, None]).max()) if Lt.size else 0.0
