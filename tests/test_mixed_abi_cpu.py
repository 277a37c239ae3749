"""Host-side checks of the mixed-precision entry points (no GPU needed):
argument validation happens before anything is enqueued, workspace sizes
follow the documented layout, and the empty problem is a no-op."""
from __future__ import annotations

import ctypes
import math

import pytest

FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
BIG = 1 << 40


@pytest.fixture(scope="module")
def tc():
    from paper_2606_11937_amd import tilechol
    return tilechol


def _factor(tc, A=FAKE, n=64, lda=64, T=16, prec=1, flags=1, shift=0.0, work=FAKE, wb=BIG):
    info = ctypes.c_int64(-7)
    st = tc.lib.chol_factor_mixed(A, n, lda, T, prec, flags, shift, work, wb, None, ctypes.byref(info))
    return st, info.value


@pytest.mark.parametrize("kw,bad_arg,code", [
    (dict(n=-1), 2, -1),
    (dict(lda=63), 3, -1),
    (dict(T=0), 4, -1),
    (dict(A=None), 1, -1),
    (dict(prec=3), 5, -1),
    (dict(prec=-1), 5, -1),
    (dict(flags=2), 6, -1),
    (dict(shift=-1e-3), 7, -1),
    (dict(shift=math.nan), 7, -1),
    (dict(shift=math.inf), 7, -1),
    (dict(work=None), 8, -1),
    (dict(wb=1000), 9, -3),
])
def test_factor_mixed_argument_checks(tc, kw, bad_arg, code):
    st, _ = _factor(tc, **kw)
    assert st == code
    assert tc.last_bad_arg() == bad_arg


def test_factor_mixed_empty_is_ok(tc):
    st, info = _factor(tc, A=None, n=0, lda=1, work=None, wb=0)
    assert st == tc.CHOL_OK and info == 0


def test_mixed_workspace_sizes(tc):
    n, T = 4096, 512
    plain = tc.chol_factor_workspace_size(n, T, 0)
    f64 = tc.chol_factor_mixed_workspace_size(n, T, "fp64")
    f32 = tc.chol_factor_mixed_workspace_size(n, T, "fp32")
    b16 = tc.chol_factor_mixed_workspace_size(n, T, "bf16")
    assert plain < f64 < b16 < f32
    # two rounded panel copies (the lookahead schedule rounds the next panel
    # while the bulk still reads the current one): n rows of
    # ceil(T / 64) * 64 elements each
    assert f32 - b16 == 2 * n * 512 * 2
    assert tc.chol_factor_mixed_workspace_size(100, 100, "fp32") - tc.chol_factor_mixed_workspace_size(
        100, 100, "bf16") >= 2 * 100 * 128 * 2
    assert tc.chol_factor_mixed_workspace_size(-1, 4, 1) == tc.CHOL_EINVAL
    assert tc.chol_factor_mixed_workspace_size(4, 0, 1) == tc.CHOL_EINVAL
    assert tc.chol_factor_mixed_workspace_size(4, 4, 9) == tc.CHOL_EINVAL
    r = tc.chol_refine_workspace_size(1000, 128, 16)
    assert r >= 4 * 1000 * 16 * 8
    assert tc.chol_refine_workspace_size(1000, 128, -1) == tc.CHOL_EINVAL
    assert tc.chol_refine_workspace_size(1000, 0, 1) == tc.CHOL_EINVAL


def _refine(tc, A=FAKE, lda=64, L=FAKE, ldl=64, n=64, T=16, B=FAKE, ldb=4, X=FAKE, ldx=4, nrhs=4, method=0,
            tol=1e-12, max_iter=10, work=FAKE, wb=BIG):
    it = ctypes.c_int64(-5)
    return tc.lib.chol_solve_refine(A, lda, L, ldl, n, T, B, ldb, X, ldx, nrhs, method, tol, max_iter, work, wb,
                                    None, ctypes.byref(it), None), it.value


@pytest.mark.parametrize("kw,bad_arg,code", [
    (dict(A=None), 1, -1),
    (dict(lda=63), 2, -1),
    (dict(L=None), 3, -1),
    (dict(ldl=10), 4, -1),
    (dict(n=-2), 5, -1),
    (dict(T=0), 6, -1),
    (dict(B=None), 7, -1),
    (dict(ldb=3), 8, -1),
    (dict(X=None), 9, -1),
    (dict(ldx=2), 10, -1),
    (dict(nrhs=-1), 11, -1),
    (dict(method=2), 12, -1),
    (dict(tol=0.0), 13, -1),
    (dict(tol=math.nan), 13, -1),
    (dict(max_iter=-1), 14, -1),
    (dict(work=None), 15, -1),
    (dict(wb=100), 16, -3),
])
def test_refine_argument_checks(tc, kw, bad_arg, code):
    st, _ = _refine(tc, **kw)
    assert st == code
    assert tc.last_bad_arg() == bad_arg


def test_refine_empty_is_ok(tc):
    st, it = _refine(tc, A=None, L=None, B=None, X=None, n=0, lda=1, ldl=1, work=None, wb=0)
    assert st == tc.CHOL_OK and it == 0
    st, it = _refine(tc, nrhs=0, work=None, wb=0)
    assert st == tc.CHOL_OK and it == 0


def test_not_converged_status_string(tc):
    assert "tolerance" in tc.status_str(tc.CHOL_NOT_CONVERGED)


# ------------------------------------------------------------------ batched
def test_batched_argument_checks(tc):
    n = (ctypes.c_int64 * 2)(64, 100)
    lda = (ctypes.c_int64 * 2)(64, 99)
    ptrs = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    st = tc.lib.chol_factor_batched(ptrs, n, lda, 2, None, FAKE, BIG, None, None)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == 3
    lda[1] = 100
    st = tc.lib.chol_factor_batched(ptrs, n, lda, -1, None, FAKE, BIG, None, None)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == 4
    st = tc.lib.chol_factor_batched(ptrs, n, lda, 2, None, None, BIG, None, None)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == 6
    st = tc.lib.chol_factor_batched(ptrs, n, lda, 2, None, FAKE, 10, None, None)
    assert st == tc.CHOL_EWORKSPACE and tc.last_bad_arg() == 7
    bad_t = (ctypes.c_int64 * 2)(0, 8)
    st = tc.lib.chol_factor_batched(ptrs, n, lda, 2, bad_t, FAKE, BIG, None, None)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == 5
    st = tc.lib.chol_factor_solve_batched(ptrs, None, n, lda, 2, None, FAKE, BIG, None, None)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == 2
    bptrs = (ctypes.c_void_p * 2)(0x3000, None)
    st = tc.lib.chol_factor_solve_batched(ptrs, bptrs, n, lda, 2, None, FAKE, BIG, None, None)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == 2


def test_batched_workspace_and_tiles(tc):
    ns = [0, 1, 100, 129, 2048, 5000]
    a = tc.chol_factor_batched_workspace_size(ns)
    b = tc.chol_factor_solve_batched_workspace_size(ns)
    assert 0 < a <= b
    assert tc.chol_factor_batched_workspace_size([]) > 0
    assert tc.chol_factor_batched_workspace_size([-1]) == tc.CHOL_EINVAL
    # the tuned table: one tile up to its first bucket, then at least 64
    assert tc.chol_batched_tile(1) == 1 and tc.chol_batched_tile(100) == 100
    prev = 0
    for n in (200, 500, 1000, 2048, 4096, 32768):
        t = tc.chol_batched_tile(n)
        assert t >= 64 and t >= prev
        prev = t
    assert tc.chol_batched_tile(100, "fp32") > 0 and tc.chol_batched_tile(100, "bf16") < 0
    # deterministic in n
    assert [tc.chol_batched_tile(n) for n in range(1, 3000, 37)] == [tc.chol_batched_tile(n) for n in range(1, 3000, 37)]


# ------------------------------------------------------------------ serving
def test_server_argument_checks(tc):
    out = ctypes.c_void_p()
    assert tc.lib.chol_server_create(None, 1 << 30, 1 << 20, 0, 16, ctypes.byref(out)) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 1
    assert tc.lib.chol_server_create(FAKE, 100, 1 << 20, 0, 16, ctypes.byref(out)) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 2
    assert tc.lib.chol_server_create(FAKE, 1 << 30, 10, 0, 16, ctypes.byref(out)) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 3
    assert tc.lib.chol_server_create(FAKE, 1 << 30, 1 << 20, 2, 16, ctypes.byref(out)) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 4
    assert tc.lib.chol_server_create(FAKE, 1 << 30, 1 << 20, 0, 0, ctypes.byref(out)) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 5
    assert tc.lib.chol_server_create(FAKE, 1 << 30, 1 << 20, 0, 16, None) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 6
    rid = ctypes.c_int64()
    assert tc.lib.chol_server_submit(None, FAKE, 10, 0.1, 0.01, FAKE, 1, 1e-12, 0, ctypes.byref(rid)) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 1
    assert tc.lib.chol_server_submit_solve(None, 0, FAKE, 10, 1, 1e-12, ctypes.byref(rid)) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 1
    assert tc.lib.chol_server_request_info(None, 0, None, None, None, None) == tc.CHOL_EINVAL
    assert tc.lib.chol_server_release_factor(None, 0) == tc.CHOL_EINVAL
    assert tc.lib.chol_server_evictions(None) == tc.CHOL_EINVAL
    assert tc.lib.chol_server_wait(None, 0, 1.0, None, None, None, None) == tc.CHOL_EINVAL
    assert tc.lib.chol_server_destroy(None) == tc.CHOL_OK
