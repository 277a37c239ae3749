"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every symbol its header declares, validates arguments before touching the
device, and its tile DAG (counts, roles, dispatch order) matches the
independent model in dag_model.py."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import dag_model as dm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tilechol.h")


@pytest.fixture(scope="module")
def tc():
    from paper_2606_11937_amd import tilechol
    return tilechol


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(chol_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("chol_factor", "chol_solve", "chol_factor_batched", "chol_factor_workspace_size",
                     "chol_solve_workspace_size", "chol_factor_batched_workspace_size"):
        assert required in names


def test_library_exports_every_declared_symbol(tc):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(tc.lib, name), name
    bound = {s[0] for s in tc.SIGNATURES}
    assert bound == set(names), (bound ^ set(names))


def test_status_strings(tc):
    for s in (0, 1, -1, -2, -3, -4):
        assert tc.status_str(s) and tc.status_str(s) != "unknown status"
    assert tc.status_str(99) == "unknown status"


def _factor_raw(tc, A, n, lda, T, sched, work, wbytes, info=True):
    inf = ctypes.c_int64(-7)
    st = tc.lib.chol_factor(A, n, lda, T, sched, work, wbytes, None, ctypes.byref(inf) if info else None)
    return st, inf.value


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("args,bad_arg,code", [
    ((FAKE, -1, 4, 2, 0), 2, -1),     # n < 0
    ((FAKE, 8, 7, 2, 0), 3, -1),      # lda < n
    ((FAKE, 8, 8, 0, 0), 4, -1),      # T < 1
    ((FAKE, 8, 8, 4, 6), 5, -1),      # unknown schedule
    ((FAKE, 8, 8, 4, 0x200), 5, -1),  # unknown schedule flag
    ((FAKE, 8, 8, 4, -1), 5, -1),     # negative schedule
    ((None, 8, 8, 4, 0), 1, -1),      # NULL matrix
    ((FAKE, 1 << 20, 1 << 20, 1, 1), 4, -1),  # too many tiles for the async schedule
    ((FAKE, 8, (1 << 20) + 1, 4, 0), 3, -1),  # lda beyond CHOL_MAX_N
    ((FAKE, (1 << 20) + 1, (1 << 20) + 1, 4, 0), 2, -1),  # n beyond CHOL_MAX_N
])
def test_factor_argument_checks(tc, args, bad_arg, code):
    A, n, lda, T, sched = args
    st, _ = _factor_raw(tc, A, n, lda, T, sched, FAKE, 1 << 40)
    assert st == code
    assert tc.last_bad_arg() == bad_arg


def test_factor_workspace_checks(tc):
    need = tc.chol_factor_workspace_size(64, 16, 0)
    assert need > 0
    st, _ = _factor_raw(tc, FAKE, 64, 64, 16, 0, None, need)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == 6
    st, _ = _factor_raw(tc, FAKE, 64, 64, 16, 0, FAKE, need - 1)
    assert st == tc.CHOL_EWORKSPACE and tc.last_bad_arg() == 7


def test_factor_empty_matrix_is_ok(tc):
    st, info = _factor_raw(tc, None, 0, 1, 4, 1, None, 0)
    assert st == tc.CHOL_OK and info == 0


def test_workspace_sizes(tc):
    assert tc.chol_factor_workspace_size(-1, 4, 0) == tc.CHOL_EINVAL
    assert tc.chol_factor_workspace_size(4, 0, 0) == tc.CHOL_EINVAL
    assert tc.chol_factor_workspace_size(4, 4, 7) == tc.CHOL_EINVAL
    a = tc.chol_factor_workspace_size(1024, 128, 0)
    b = tc.chol_factor_workspace_size(1024, 128, 1)
    assert a == b > 0
    # counters grow with the number of row blocks
    assert tc.chol_factor_workspace_size(32768, 128, 1) > tc.chol_factor_workspace_size(8192, 128, 1)
    # a 256-byte header, then the forward and backward payloads: 64-row
    # blocks of 2 columns (one or two right-hand sides) or 4 columns per
    # pass of four (up to 16 passes share a launch pair and its payloads)
    r256 = lambda x: (x + 255) // 256 * 256
    for n, nrhs in ((100, 3), (100, 1), (100, 2), (100, 8), (100, 9), (64, 16), (65, 40), (65, 64),
                    (65, 65), (65, 200), (32768, 1)):
        pw = 2 if nrhs <= 2 else 4
        npass = min(16, (nrhs + 3) // 4) if pw == 4 else 1
        want = 256 + 2 * r256(8 * ((n + 63) // 64) * 64 * pw * npass)
        assert tc.chol_solve_workspace_size(n, 16, nrhs) == want
    assert tc.chol_solve_workspace_size(100, 0, 3) == tc.CHOL_EINVAL


@pytest.mark.parametrize("args,bad_arg", [
    ((FAKE, -1, 4, 4, FAKE, 1, 1), 2),
    ((FAKE, 8, 4, 4, FAKE, 1, 1), 3),
    ((FAKE, 8, 8, 0, FAKE, 1, 1), 4),
    ((FAKE, 8, 8, 4, FAKE, -1, 1), 6),
    ((FAKE, 8, 8, 4, FAKE, 3, 2), 7),
    ((None, 8, 8, 4, FAKE, 1, 1), 1),
    ((FAKE, 8, 8, 4, None, 1, 1), 5),
])
def test_solve_argument_checks(tc, args, bad_arg):
    L, n, lda, T, B, nrhs, ldb = args
    st = tc.lib.chol_solve(L, n, lda, T, B, nrhs, ldb, FAKE, 1 << 20, None)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == bad_arg


def test_solve_workspace_checks(tc):
    need = tc.chol_solve_workspace_size(8, 4, 1)
    st = tc.lib.chol_solve(FAKE, 8, 8, 4, FAKE, 1, 1, None, need, None)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == 8
    st = tc.lib.chol_solve(FAKE, 8, 8, 4, FAKE, 1, 1, FAKE, need - 1, None)
    assert st == tc.CHOL_EWORKSPACE and tc.last_bad_arg() == 9
    # nothing to solve: OK without touching anything
    assert tc.lib.chol_solve(None, 0, 1, 4, None, 3, 3, None, 0, None) == tc.CHOL_OK


def test_batched_argument_checks(tc):
    n = (ctypes.c_int64 * 2)(4, 8)
    lda = (ctypes.c_int64 * 2)(4, 7)
    ptrs = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    st = tc.lib.chol_factor_batched(ptrs, n, lda, 2, None, FAKE, 1 << 30, None, None)
    assert st == tc.CHOL_EINVAL and tc.last_bad_arg() == 3
    assert tc.lib.chol_factor_batched(ptrs, n, lda, -1, None, FAKE, 1, None, None) == tc.CHOL_EINVAL
    assert tc.lib.chol_factor_batched(None, n, lda, 0, None, None, 0, None, None) == tc.CHOL_OK
    assert tc.chol_factor_batched_workspace_size([4, 8], None) > 0


def test_wait_limit_setter(tc):
    prev = tc.chol_set_wait_limit(3.0)
    assert tc.chol_set_wait_limit(prev) == 3.0
    assert tc.chol_set_wait_limit(-1.0) == -1.0


def test_default_tile_is_deterministic(tc):
    for n in (1, 100, 1024, 8192, 32768):
        T = tc.chol_default_tile(n)
        assert T >= 1 and T == tc.chol_default_tile(n)


# ------------------------------------------------------------------- DAG
@pytest.mark.parametrize("M", [1, 2, 3, 4, 8, 16, 64, 256])
def test_task_counts_match_paper(tc, M):
    # Results, problem-size scaling: M POTRF, M(M-1)/2 TRSM and SYRK, M(M-1)(M-2)/6 GEMM
    c = tc.chol_dag_counts(M * 128, 128)
    assert c["potrf"] == M
    assert c["trsm"] == c["syrk"] == M * (M - 1) // 2
    assert c["gemm"] == M * (M - 1) * (M - 2) // 6
    assert c["potrf"] + c["trsm"] + c["syrk"] + c["gemm"] == M * (M + 1) * (M + 2) // 6
    # the model's program-order task list agrees
    kinds = [t[0] for t in dm.tile_tasks(M)]
    assert kinds.count("GEMM") == c["gemm"] and kinds.count("TRSM") == c["trsm"]


@pytest.mark.parametrize("M", [1, 2, 4, 8, 12])
def test_critical_path_is_3M_minus_2(M):
    tasks = dm.tile_tasks(M)
    assert dm.critical_path(tasks, dm.dependency_edges(tasks)) == 3 * M - 2


def test_first_step_roles_match_fig2(tc):
    # 4 x 4 tiles, J = 0: P at (0,0); T at (1..3,0); S at (1,1),(2,2),(3,3);
    # G at (2,1),(3,1),(3,2)
    units = tc.chol_dag_enumerate(4 * 128, 128, grid=8)
    roles = {}
    for kind, J, I, a, K, b in units:
        if J != 0:
            continue
        if kind == dm.POTRF:
            roles[(I, I)] = "P"
        elif kind == dm.TRSM:
            roles[(I, 0)] = "T"
        else:
            roles[(I, K)] = "S" if I == K else "G"
    assert roles == {(0, 0): "P", (1, 0): "T", (2, 0): "T", (3, 0): "T", (1, 1): "S", (2, 2): "S",
                     (3, 3): "S", (2, 1): "G", (3, 1): "G", (3, 2): "G"}


CASES = [(1, 1), (5, 3), (128, 128), (300, 128), (1024, 128), (1000, 96), (777, 256), (2048, 512),
         (1536, 200), (640, 1024), (4096, 256)]


@pytest.mark.parametrize("n,T", CASES)
@pytest.mark.parametrize("grid", [1, 7, 256])
def test_ticket_order_is_topological(tc, n, T, grid):
    g = dm.Geom(n, T)
    units = tc.chol_dag_enumerate(n, T, grid=grid)
    assert len(units) == tc.chol_dag_counts(n, T)["units"]
    assert dm.check_ticket_order(g, units) == []


@pytest.mark.parametrize("n,T", CASES)
def test_units_cover_every_block_update_once(tc, n, T):
    """Each diagonal block is factored once, each block below it solved once
    per sub-column, each later panel block updated once per earlier
    sub-column of its panel, and each lower trailing block updated once per
    earlier step: the decomposition covers Fig. 1 exactly."""
    g = dm.Geom(n, T)
    units = tc.chol_dag_enumerate(n, T, grid=16)
    seen = set()
    for u in units:
        key = tuple(int(x) for x in u)
        assert key not in seen
        seen.add(key)
    expect = set(dm.program_order_units(g))
    assert seen == expect
    # hand count of the panel part for the first step
    G = g.NRB
    n_panel = sum(1 + (G - s - 1) + sum(G - t for t in range(s + 1, g.sb(0))) for s in range(g.sb(0)))
    assert sum(1 for u in seen if u[1] == 0 and u[0] != dm.UPDATE) == n_panel


def test_dropped_dependency_is_detected():
    """The order checker itself: moving a GEMM unit ahead of the TRSM it
    reads must be reported."""
    g = dm.Geom(512, 128)
    units = [list(u) for u in _program_order_units(g)]
    i_trsm = next(i for i, u in enumerate(units) if u[0] == dm.TRSM and u[2] == 2)
    assert units[i_trsm][1] == 0
    i_gemm = next(i for i, u in enumerate(units) if u[0] == dm.UPDATE and u[2] == 2 and u[4] == 1)
    assert dm.check_ticket_order(g, units) == []
    units.insert(i_trsm, units.pop(i_gemm))
    assert dm.check_ticket_order(g, units) != []


def _program_order_units(g):
    return np.array(dm.program_order_units(g), dtype=np.int32)


@pytest.mark.parametrize("n,T", CASES)
def test_forkjoin_update_launch_covers_each_step(tc, n, T):
    """The launch order of each fork-join trailing update visits every lower
    output block of the step's trailing matrix exactly once."""
    g = dm.Geom(n, T)
    for J in range(g.M):
        got = tc.chol_dag_forkjoin_update(n, T, J)
        keys = [tuple(int(x) for x in u) for u in got]
        assert len(keys) == len(set(keys))
        expect = set()
        for I in range(J + 1, g.M):
            for K in range(J + 1, I + 1):
                for a in range(g.sb(I)):
                    for b in range(g.sb(K)):
                        if I == K and b > a:
                            continue
                        expect.add((dm.UPDATE, J, I, a, K, b))
        assert set(keys) == expect, J


def test_timing_read_rejects_null_outputs(tc):
    import ctypes
    ms = (ctypes.c_double * 5)()
    assert tc.lib.chol_timing_read(None, None, None) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 2
    assert tc.lib.chol_timing_read(None, ms, None) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 3


@pytest.mark.parametrize("look", [0, 1, 7, 10 ** 9])
@pytest.mark.parametrize("n,T", [(1000, 96), (2048, 512), (1536, 200)])
def test_lookahead_setting_keeps_the_order_topological(tc, look, n, T):
    """Every dispatch-order setting (chain first, bulk first, in between)
    is still a topological order covering the same units."""
    prev = tc.chol_set_lookahead(look)
    try:
        g = dm.Geom(n, T)
        units = tc.chol_dag_enumerate(n, T, grid=16)
        assert dm.check_ticket_order(g, units) == []
        assert set(tuple(int(x) for x in u) for u in units) == set(dm.program_order_units(g))
    finally:
        tc.chol_set_lookahead(prev)
    assert tc.chol_set_lookahead(-5) == prev  # negative restores the default
    assert tc.chol_set_lookahead(prev) == -1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus above 1 exits with a message before
    touching a device."""
    import subprocess
    import sys as _sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([_sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_batched_mixed_argument_checks(tc):
    """chol_factor_solve_batched_mixed validates everything before touching
    the device: the factor must not overwrite the original, precisions and
    tile sides must be usable, and the workspace must be large enough."""
    vp = lambda *p: (ctypes.c_void_p * len(p))(*p)
    i64 = lambda *v: (ctypes.c_int64 * len(v))(*v)
    A, L, B, X = vp(FAKE.value), vp(0x2000), vp(0x3000), vp(0x4000)
    n, ld = i64(300), i64(300)
    call = lambda A_, L_, T_, p_, tol, it, wb: tc.lib.chol_factor_solve_batched_mixed(
        A_, L_, B, X, n, ld, ld, 1, T_, p_, tol, it, FAKE, wb, None, None, None, None)
    assert call(A, vp(FAKE.value), None, None, 1e-12, 5, 1 << 40) == tc.CHOL_EINVAL and tc.last_bad_arg() == 2
    assert call(A, L, None, None, 0.0, 5, 1 << 40) == tc.CHOL_EINVAL and tc.last_bad_arg() == 11
    assert call(A, L, None, None, 1e-12, -1, 1 << 40) == tc.CHOL_EINVAL and tc.last_bad_arg() == 12
    assert call(A, L, None, (ctypes.c_int32 * 1)(2), 1e-12, 5, 1 << 40) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 10  # BF16 is not offered in the batched launch
    assert call(A, L, i64(126), (ctypes.c_int32 * 1)(1), 1e-12, 5, 1 << 40) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 9  # FP32 products read the panel copy in 4-float pieces
    need = tc.chol_factor_solve_batched_mixed_workspace_size([300], [128], ["fp32"])
    assert need > tc.chol_factor_solve_batched_mixed_workspace_size([300], [128], ["fp64"]) > 0
    assert call(A, L, i64(128), (ctypes.c_int32 * 1)(1), 1e-12, 5, need - 1) == tc.CHOL_EWORKSPACE
    assert tc.last_bad_arg() == 14
    assert tc.chol_batched_tile(1000, "fp32") > 0 and tc.chol_batched_tile(1000, "bf16") == tc.CHOL_EINVAL
