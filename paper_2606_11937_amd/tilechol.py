"""Thin ctypes binding of libtilechol.so (the C ABI in include/tilechol.h).

Every function here only marshals arguments: tensors become device pointers
and sizes, the current torch stream becomes the HIP stream, and workspaces
are allocated with torch (the library itself never allocates).  All
computation happens in the HIP kernels of the library.  If the library is
missing this module raises on import instead of falling back to anything.

Names follow the C ABI: chol_factor, chol_solve, chol_factor_batched, ...
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtilechol.so")

CHOL_OK = 0
CHOL_NOT_SPD = 1
CHOL_EINVAL = -1
CHOL_EDEVICE = -2
CHOL_EWORKSPACE = -3
CHOL_ETIMEOUT = -4
CHOL_ESTALLED = -5
CHOL_ENOFACTOR = -6
CHOL_SERVE_KEEP = 1
CHOL_SCHED_FORK_JOIN = 0
CHOL_SCHED_ASYNC_DAG = 1
CHOL_SCHED_FORK_JOIN_NAIVE = 2
CHOL_SCHED_TASK_SYNC = 3
CHOL_SCHED_FORK_JOIN_LOOKAHEAD = 4
CHOL_SCHED_GRAPH_DAG = 5
CHOL_SCHED_NOOP = 0x100
CHOL_BLOCK = 128
CHOL_NOT_CONVERGED = 2
CHOL_PREC_FP64 = 0
CHOL_PREC_FP32 = 1
CHOL_PREC_BF16 = 2
CHOL_MIXED_SCALE = 1
CHOL_REFINE_IR = 0
CHOL_REFINE_PCG = 1
PRECISIONS = {"fp64": CHOL_PREC_FP64, "fp32": CHOL_PREC_FP32, "bf16": CHOL_PREC_BF16}
REFINE_METHODS = {"ir": CHOL_REFINE_IR, "pcg": CHOL_REFINE_PCG}
CHOL_SERVE_CONTINUOUS = 0
CHOL_SERVE_FIFO = 1
CHOL_SERVE_MAX_RHS = 8
CHOL_ASYNC_MAX_TILES = 1024
SCHEDULES = {"fork_join": CHOL_SCHED_FORK_JOIN, "async_dag": CHOL_SCHED_ASYNC_DAG,
             "fork_join_naive": CHOL_SCHED_FORK_JOIN_NAIVE, "task_sync": CHOL_SCHED_TASK_SYNC,
             "fork_join_lookahead": CHOL_SCHED_FORK_JOIN_LOOKAHEAD, "graph_dag": CHOL_SCHED_GRAPH_DAG}

# (name, restype, argtypes) for every symbol of include/tilechol.h
_i64, _int, _dbl, _vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
_pi64, _pi32 = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)
SIGNATURES = [
    ("chol_factor_workspace_size", _i64, [_i64, _i64, _int]),
    ("chol_factor", _int, [_vp, _i64, _i64, _i64, _int, _vp, _i64, _vp, _pi64]),
    ("chol_factor_info", _int, [_vp, _vp, _pi64]),
    ("chol_factor_noalloc", _int, [_vp, _i64, _i64, _i64, _int, _vp, _pi64]),
    ("chol_solve_workspace_size", _i64, [_i64, _i64, _i64]),
    ("chol_solve", _int, [_vp, _i64, _i64, _i64, _vp, _i64, _i64, _vp, _i64, _vp]),
    ("chol_solve_info", _int, [_vp, _vp]),
    ("chol_factor_batched_workspace_size", _i64, [_i64, _pi64, _pi64]),
    ("chol_factor_batched", _int, [ctypes.POINTER(_vp), _pi64, _pi64, _i64, _pi64, _vp, _i64, _vp, _pi64]),
    ("chol_factor_solve_batched_workspace_size", _i64, [_i64, _pi64, _pi64]),
    ("chol_factor_solve_batched", _int, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _pi64, _pi64, _i64, _pi64, _vp,
                                         _i64, _vp, _pi64]),
    ("chol_factor_solve_batched_mixed_workspace_size", _i64, [_i64, _pi64, _pi64, _pi32]),
    ("chol_factor_solve_batched_mixed", _int, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                               ctypes.POINTER(_vp), _pi64, _pi64, _pi64, _i64, _pi64, _pi32, _dbl,
                                               _i64, _vp, _i64, _vp, _pi64, _pi64, ctypes.POINTER(_dbl)]),
    ("chol_batched_tile", _i64, [_i64, _int]),
    ("chol_factor_mixed_workspace_size", _i64, [_i64, _i64, _int]),
    ("chol_factor_mixed", _int, [_vp, _i64, _i64, _i64, _int, _int, _dbl, _vp, _i64, _vp, _pi64]),
    ("chol_refine_workspace_size", _i64, [_i64, _i64, _i64]),
    ("chol_solve_refine", _int, [_vp, _i64, _vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _i64, _int, _dbl, _i64,
                                 _vp, _i64, _vp, _pi64, ctypes.POINTER(_dbl)]),
    ("chol_server_create", _int, [_vp, _i64, _i64, _int, _i64, ctypes.POINTER(_vp)]),
    ("chol_server_submit", _int, [_vp, _vp, _i64, _dbl, _dbl, _vp, _i64, _dbl, _int, _pi64]),
    ("chol_server_submit_solve", _int, [_vp, _i64, _vp, _i64, _i64, _dbl, _pi64]),
    ("chol_server_request_info", _int, [_vp, _i64, _pi64, ctypes.POINTER(_int), ctypes.POINTER(_int),
                                        ctypes.POINTER(_int)]),
    ("chol_server_release_factor", _int, [_vp, _i64]),
    ("chol_server_set_plan", _int, [_vp, _i64, _i64]),
    ("chol_server_evictions", _i64, [_vp]),
    ("chol_server_wait", _int, [_vp, _i64, _dbl, _vp, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), _pi64]),
    ("chol_server_ticks", _i64, [_vp]),
    ("chol_server_destroy", _int, [_vp]),
    ("chol_default_tile", _i64, [_i64]),
    ("chol_dag_counts", _int, [_i64, _i64, _pi64]),
    ("chol_dag_enumerate", _i64, [_i64, _i64, _i64, _pi32, _i64]),
    ("chol_dag_forkjoin_update", _i64, [_i64, _i64, _i64, _pi32, _i64]),
    ("chol_timing_enable", _int, [_int]),
    ("chol_timing_read", _int, [_vp, ctypes.POINTER(_dbl), _pi64]),
    ("chol_async_grid", _i64, []),
    ("chol_set_wait_limit", _dbl, [_dbl]),
    ("chol_set_lookahead", _i64, [_i64]),
    ("chol_last_bad_arg", _int, []),
    ("chol_status_str", ctypes.c_char_p, [_int]),
]


class TileCholError(RuntimeError):
    def __init__(self, status: int, where: str, bad_arg: int = 0):
        msg = f"{where}: {status_str(status)} (status {status}"
        if bad_arg:
            msg += f", argument {bad_arg}"
        super().__init__(msg + ")")
        self.status = status
        self.bad_arg = bad_arg


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2606_11937_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def status_str(status: int) -> str:
    return lib.chol_status_str(int(status)).decode()


def last_bad_arg() -> int:
    return int(lib.chol_last_bad_arg())


def _sched(s) -> int:
    return SCHEDULES[s] if isinstance(s, str) else int(s)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_matrix(A, name="A"):
    import torch
    if not isinstance(A, torch.Tensor) or A.dtype != torch.float64 or A.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float64 torch tensor")
    if not A.is_cuda:
        raise TypeError(f"{name} must live on the GPU")
    if A.shape[1] > 0 and A.stride(1) != 1:
        raise TypeError(f"{name} must be row-major (stride(1) == 1)")


# ----------------------------------------------------------------- factor
def chol_factor_workspace_size(n: int, T: int, sched="fork_join") -> int:
    return int(lib.chol_factor_workspace_size(n, T, _sched(sched)))


def factor_workspace(n: int, T: int, sched="fork_join", device="cuda"):
    import torch
    nb = chol_factor_workspace_size(n, T, sched)
    if nb < 0:
        raise TileCholError(int(nb), "chol_factor_workspace_size", last_bad_arg())
    return torch.empty(max(nb, 8), dtype=torch.uint8, device=device)


def chol_factor(A, T: int, sched="fork_join", n: int | None = None, work=None, stream=None,
                sync: bool = True, noop: bool = False) -> int:
    """Factor A (n x n view of a row-major float64 GPU tensor) in place.
    Returns info (0, or k > 0 for a non-positive-definite leading minor of
    order k) when sync, else None.  Raises TileCholError on errors.
    noop=True runs the schedule with empty unit bodies (measurement only;
    A is left unchanged)."""
    _check_matrix(A)
    n = A.shape[0] if n is None else n
    lda = A.stride(0) if A.shape[0] > 1 else max(1, A.shape[1])
    if work is None:
        work = factor_workspace(n, T, sched, A.device)
    info = ctypes.c_int64(0)
    code = _sched(sched) | (CHOL_SCHED_NOOP if noop else 0)
    st = lib.chol_factor(ctypes.c_void_p(A.data_ptr()), n, lda, T, code,
                         ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(stream),
                         ctypes.byref(info) if sync else None)
    if st not in (CHOL_OK, CHOL_NOT_SPD):
        raise TileCholError(st, "chol_factor", last_bad_arg())
    return int(info.value) if sync else None


def chol_factor_noalloc(A, T: int, sched="fork_join", n: int | None = None, stream=None, sync: bool = True) -> int:
    """chol_factor with the library's fixed device workspace (no allocation by
    the library or here).  Returns info when sync."""
    _check_matrix(A)
    n = A.shape[0] if n is None else n
    lda = A.stride(0) if A.shape[0] > 1 else max(1, A.shape[1])
    info = ctypes.c_int64(0)
    st = lib.chol_factor_noalloc(ctypes.c_void_p(A.data_ptr()), n, lda, T, _sched(sched), _stream(stream),
                                 ctypes.byref(info) if sync else None)
    if st not in (CHOL_OK, CHOL_NOT_SPD):
        raise TileCholError(st, "chol_factor_noalloc", last_bad_arg())
    return int(info.value) if sync else None


def chol_factor_info(work, stream=None) -> int:
    info = ctypes.c_int64(0)
    st = lib.chol_factor_info(ctypes.c_void_p(work.data_ptr()), _stream(stream), ctypes.byref(info))
    if st not in (CHOL_OK, CHOL_NOT_SPD):
        raise TileCholError(st, "chol_factor_info", last_bad_arg())
    return int(info.value)


# ------------------------------------------------------------------ solve
def chol_solve_workspace_size(n: int, T: int, nrhs: int) -> int:
    return int(lib.chol_solve_workspace_size(n, T, nrhs))


def chol_solve(L, B, T: int, n: int | None = None, work=None, stream=None) -> None:
    """Overwrite B (n x nrhs row-major float64 GPU tensor) with (L L^T)^{-1} B."""
    _check_matrix(L, "L")
    _check_matrix(B, "B")
    n = L.shape[0] if n is None else n
    lda = L.stride(0) if L.shape[0] > 1 else max(1, L.shape[1])
    nrhs = B.shape[1]
    ldb = B.stride(0) if B.shape[0] > 1 else max(1, nrhs)
    if work is None:
        import torch
        nb = chol_solve_workspace_size(n, T, nrhs)
        if nb < 0:
            raise TileCholError(nb, "chol_solve_workspace_size", last_bad_arg())
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=B.device)
    wptr, wbytes = work.data_ptr(), work.numel()
    st = lib.chol_solve(ctypes.c_void_p(L.data_ptr()), n, lda, T, ctypes.c_void_p(B.data_ptr()), nrhs, ldb,
                        ctypes.c_void_p(wptr), wbytes, _stream(stream))
    if st != CHOL_OK:
        raise TileCholError(st, "chol_solve", last_bad_arg())


def chol_solve_info(work, stream=None) -> int:
    """Status of the last chol_solve with this workspace: CHOL_OK or
    CHOL_ETIMEOUT (synchronises the stream)."""
    st = lib.chol_solve_info(ctypes.c_void_p(work.data_ptr()), _stream(stream))
    if st not in (CHOL_OK, CHOL_ETIMEOUT):
        raise TileCholError(st, "chol_solve_info", last_bad_arg())
    return st


# -------------------------------------------------------- mixed precision
def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def chol_factor_mixed_workspace_size(n: int, T: int, prec="fp32") -> int:
    return int(lib.chol_factor_mixed_workspace_size(n, T, _prec(prec)))


def chol_factor_mixed(A, T: int, prec="fp32", scale: bool = True, shift: float = 0.0, n: int | None = None,
                      work=None, stream=None, sync: bool = True):
    """Factor A in place with low-precision trailing products (FP32 or BF16
    panel operands, FP32 sums, FP64 storage; FP64 POTRF and TRSM), with
    optional diagonal scaling and shift.  Returns info when sync."""
    import torch
    _check_matrix(A)
    n = A.shape[0] if n is None else n
    lda = A.stride(0) if A.shape[0] > 1 else max(1, A.shape[1])
    if work is None:
        nb = chol_factor_mixed_workspace_size(n, T, prec)
        if nb < 0:
            raise TileCholError(nb, "chol_factor_mixed_workspace_size", last_bad_arg())
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=A.device)
    info = ctypes.c_int64(0)
    st = lib.chol_factor_mixed(ctypes.c_void_p(A.data_ptr()), n, lda, T, _prec(prec),
                               CHOL_MIXED_SCALE if scale else 0, float(shift), ctypes.c_void_p(work.data_ptr()),
                               work.numel(), _stream(stream), ctypes.byref(info) if sync else None)
    if st not in (CHOL_OK, CHOL_NOT_SPD):
        raise TileCholError(st, "chol_factor_mixed", last_bad_arg())
    return int(info.value) if sync else None


def chol_refine_workspace_size(n: int, T: int, nrhs: int) -> int:
    return int(lib.chol_refine_workspace_size(n, T, nrhs))


def chol_solve_refine(A, L, B, X, T: int, method="ir", tol: float = 1e-12, max_iter: int = 30,
                      n: int | None = None, work=None, stream=None):
    """Solve A X = B (FP64) with the factor L (of A or of a shifted A) by
    iterative refinement or PCG.  Returns (converged, iterations, eta per
    column as a list)."""
    import torch
    for t, nm in ((A, "A"), (L, "L"), (B, "B"), (X, "X")):
        _check_matrix(t, nm)
    n = A.shape[0] if n is None else n
    nrhs = B.shape[1]
    ld = lambda t: t.stride(0) if t.shape[0] > 1 else max(1, t.shape[1])
    if work is None:
        nb = chol_refine_workspace_size(n, T, nrhs)
        if nb < 0:
            raise TileCholError(nb, "chol_refine_workspace_size", last_bad_arg())
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=A.device)
    it = ctypes.c_int64(0)
    eta = (ctypes.c_double * max(nrhs, 1))()
    m = REFINE_METHODS[method] if isinstance(method, str) else int(method)
    st = lib.chol_solve_refine(ctypes.c_void_p(A.data_ptr()), ld(A), ctypes.c_void_p(L.data_ptr()), ld(L), n, T,
                               ctypes.c_void_p(B.data_ptr()), ld(B), ctypes.c_void_p(X.data_ptr()), ld(X), nrhs, m,
                               float(tol), int(max_iter), ctypes.c_void_p(work.data_ptr()), work.numel(),
                               _stream(stream), ctypes.byref(it), eta)
    if st not in (CHOL_OK, CHOL_NOT_CONVERGED):
        raise TileCholError(st, "chol_solve_refine", last_bad_arg())
    return st == CHOL_OK, int(it.value), [float(eta[c]) for c in range(nrhs)]


# ---------------------------------------------------------------- batched
def chol_factor_batched_workspace_size(ns, Ts=None) -> int:
    b = len(ns)
    n_arr = (ctypes.c_int64 * max(b, 1))(*ns)
    t_arr = (ctypes.c_int64 * b)(*Ts) if Ts is not None else None
    return int(lib.chol_factor_batched_workspace_size(b, n_arr, t_arr))


def chol_factor_solve_batched_workspace_size(ns, Ts=None) -> int:
    b = len(ns)
    n_arr = (ctypes.c_int64 * max(b, 1))(*ns)
    t_arr = (ctypes.c_int64 * b)(*Ts) if Ts is not None else None
    return int(lib.chol_factor_solve_batched_workspace_size(b, n_arr, t_arr))


def chol_batched_tile(n: int, prec="fp64") -> int:
    return int(lib.chol_batched_tile(n, _prec(prec)))


def _batch_args(As):
    """Checks every matrix as _check_matrix does and returns the batch's
    count, orders, device pointers, orders and leading dimensions; one pass,
    with as few tensor attribute reads per matrix as the checks allow (a
    batch has thousands of them)."""
    import torch
    f64, Tensor = torch.float64, torch.Tensor
    ns, ldas, ps = [], [], []
    for A in As:
        if not isinstance(A, Tensor):
            raise TypeError("A must be a 2-D float64 torch tensor")
        sh, st = A.shape, A.stride()
        if A.dtype is not f64 or len(sh) != 2:
            raise TypeError("A must be a 2-D float64 torch tensor")
        if not A.is_cuda:
            raise TypeError("A must live on the GPU")
        if sh[1] > 0 and st[1] != 1:
            raise TypeError("A must be row-major (stride(1) == 1)")
        n = sh[0]
        ns.append(n)
        ldas.append(st[0] if n > 1 else max(1, sh[1]))
        ps.append(A.data_ptr())
    b = len(As)
    ptrs = (ctypes.c_void_p * max(b, 1))(*ps)
    return b, ns, ptrs, (ctypes.c_int64 * max(b, 1))(*ns), (ctypes.c_int64 * max(b, 1))(*ldas)


def chol_factor_batched(As, Ts=None, work=None, stream=None, sync: bool = True):
    """Factor a list of square row-major float64 GPU tensors in place, in one
    persistent launch.  Returns the list of infos when sync."""
    import torch
    b, ns, ptrs, n_arr, l_arr = _batch_args(As)
    if work is None:
        nb = chol_factor_batched_workspace_size(ns, Ts)
        if nb < 0:
            raise TileCholError(nb, "chol_factor_batched_workspace_size", last_bad_arg())
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=As[0].device if b else "cuda")
    t_arr = (ctypes.c_int64 * b)(*Ts) if Ts is not None else None
    infos = (ctypes.c_int64 * max(b, 1))()
    st = lib.chol_factor_batched(ptrs, n_arr, l_arr, b, t_arr, ctypes.c_void_p(work.data_ptr()), work.numel(),
                                 _stream(stream), infos if sync else None)
    if st not in (CHOL_OK, CHOL_NOT_SPD):
        raise TileCholError(st, "chol_factor_batched", last_bad_arg())
    return [int(infos[i]) for i in range(b)] if sync else None


def chol_factor_solve_batched(As, Bs, Ts=None, work=None, stream=None, sync: bool = True):
    """Factor each A_i in place and overwrite each b_i (contiguous float64 GPU
    vector of n_i entries) with A_i^{-1} b_i, all in one persistent launch.
    Returns the list of infos when sync."""
    import torch
    b, ns, ptrs, n_arr, l_arr = _batch_args(As)
    if len(Bs) != b:
        raise ValueError("one right-hand side per matrix")
    f64 = torch.float64
    for B, n in zip(Bs, ns):
        if B.dtype is not f64 or not B.is_cuda or B.numel() != n or not B.is_contiguous():
            raise TypeError("each right-hand side must be a contiguous float64 GPU vector of n entries")
    if work is None:
        nb = chol_factor_solve_batched_workspace_size(ns, Ts)
        if nb < 0:
            raise TileCholError(nb, "chol_factor_solve_batched_workspace_size", last_bad_arg())
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=As[0].device if b else "cuda")
    bptrs = (ctypes.c_void_p * max(b, 1))(*[B.data_ptr() for B in Bs])
    t_arr = (ctypes.c_int64 * b)(*Ts) if Ts is not None else None
    infos = (ctypes.c_int64 * max(b, 1))()
    st = lib.chol_factor_solve_batched(ptrs, bptrs, n_arr, l_arr, b, t_arr, ctypes.c_void_p(work.data_ptr()),
                                       work.numel(), _stream(stream), infos if sync else None)
    if st not in (CHOL_OK, CHOL_NOT_SPD):
        raise TileCholError(st, "chol_factor_solve_batched", last_bad_arg())
    return [int(infos[i]) for i in range(b)] if sync else None


def chol_factor_solve_batched_mixed_workspace_size(ns, Ts=None, precs=None) -> int:
    b = len(ns)
    n_arr = (ctypes.c_int64 * max(b, 1))(*ns)
    t_arr = (ctypes.c_int64 * b)(*Ts) if Ts is not None else None
    p_arr = (ctypes.c_int32 * b)(*[_prec(p) for p in precs]) if precs is not None else None
    return int(lib.chol_factor_solve_batched_mixed_workspace_size(b, n_arr, t_arr, p_arr))


def chol_factor_solve_batched_mixed(As, Ls, Bs, Xs, Ts=None, precs=None, tol: float = 1e-12, max_iter: int = 10,
                                    work=None, stream=None, sync: bool = True):
    """Factor each original A_i (left untouched) into L_i with FP32 or FP64
    trailing products (precs: list of "fp32"/"fp64", None = FP64), then solve
    A_i x_i = b_i into X_i with FP64 refinement to tol, all in one persistent
    launch.  Returns (infos, corrections, etas) when sync."""
    import torch
    b, ns, a_ptrs, n_arr, la_arr = _batch_args(As)
    bl, nls, l_ptrs, _, ll_arr = _batch_args(Ls)
    if bl != b or len(Bs) != b or len(Xs) != b:
        raise ValueError("As, Ls, Bs and Xs must have one entry per matrix")
    if nls != ns:
        raise ValueError("each L must have the order of its A")
    f64 = torch.float64
    for n, B, X in zip(ns, Bs, Xs):
        for v in (B, X):
            if v.dtype is not f64 or not v.is_cuda or v.numel() != n or not v.is_contiguous():
                raise TypeError("right-hand sides and solutions must be contiguous float64 GPU vectors of n entries")
    if work is None:
        nb = chol_factor_solve_batched_mixed_workspace_size(ns, Ts, precs)
        if nb < 0:
            raise TileCholError(nb, "chol_factor_solve_batched_mixed_workspace_size", last_bad_arg())
        work = torch.empty(max(nb, 8), dtype=torch.uint8, device=As[0].device if b else "cuda")
    vp = lambda ts: (ctypes.c_void_p * max(b, 1))(*[t.data_ptr() for t in ts])
    t_arr = (ctypes.c_int64 * b)(*Ts) if Ts is not None else None
    p_arr = (ctypes.c_int32 * b)(*[_prec(p) for p in precs]) if precs is not None else None
    infos, its = (ctypes.c_int64 * max(b, 1))(), (ctypes.c_int64 * max(b, 1))()
    etas = (ctypes.c_double * max(b, 1))()
    st = lib.chol_factor_solve_batched_mixed(a_ptrs, l_ptrs, vp(Bs), vp(Xs), n_arr, la_arr, ll_arr, b, t_arr, p_arr,
                                             float(tol), int(max_iter),
                                             ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(stream),
                                             infos if sync else None, its if sync else None,
                                             etas if sync else None)
    if st not in (CHOL_OK, CHOL_NOT_SPD, CHOL_NOT_CONVERGED):
        raise TileCholError(st, "chol_factor_solve_batched_mixed", last_bad_arg())
    if not sync:
        return None
    return [int(infos[i]) for i in range(b)], [int(its[i]) for i in range(b)], [float(etas[i]) for i in range(b)]


# ---------------------------------------------------------------- serving
class Server:
    """Factor + solve server with continuous batching (chol_server_*).

    The device arena (a torch uint8 GPU tensor, the HBM budget) is held for
    the server's lifetime.  submit() takes numpy inputs and returns a request
    id; wait() returns (status, X, eta, latency_s, info)."""

    def __init__(self, arena, pinned_bytes: int = 1 << 30, mode: str = "continuous", max_per_tick: int = 4096):
        import numpy as np  # noqa: F401
        self.arena = arena
        self.h = ctypes.c_void_p()
        m = CHOL_SERVE_CONTINUOUS if mode == "continuous" else CHOL_SERVE_FIFO
        st = lib.chol_server_create(ctypes.c_void_p(arena.data_ptr()), arena.numel(), pinned_bytes, m, max_per_tick,
                                    ctypes.byref(self.h))
        if st != CHOL_OK:
            raise TileCholError(st, "chol_server_create", last_bad_arg())
        self.shapes = {}

    def submit(self, points, B, lengthscale: float, nugget: float, tol: float, keep: bool = False) -> int:
        import numpy as np
        P = np.ascontiguousarray(points, dtype=np.float64)
        Bm = np.ascontiguousarray(B, dtype=np.float64)
        if Bm.ndim == 1:
            Bm = Bm.reshape(-1, 1)
        n, nrhs = Bm.shape
        rid = ctypes.c_int64(-1)
        st = lib.chol_server_submit(self.h, P.ctypes.data_as(ctypes.c_void_p), n, float(lengthscale), float(nugget),
                                    Bm.ctypes.data_as(ctypes.c_void_p), nrhs, float(tol),
                                    CHOL_SERVE_KEEP if keep else 0, ctypes.byref(rid))
        if st != CHOL_OK:
            raise TileCholError(st, "chol_server_submit", last_bad_arg())
        self.shapes[rid.value] = (n, nrhs)
        return rid.value

    def submit_solve(self, factor: int, B, tol: float) -> int:
        """A solve with a resident factor; raises TileCholError with status
        CHOL_ENOFACTOR if it is no longer resident."""
        import numpy as np
        Bm = np.ascontiguousarray(B, dtype=np.float64)
        if Bm.ndim == 1:
            Bm = Bm.reshape(-1, 1)
        n, nrhs = Bm.shape
        rid = ctypes.c_int64(-1)
        st = lib.chol_server_submit_solve(self.h, int(factor), Bm.ctypes.data_as(ctypes.c_void_p), n, nrhs,
                                          float(tol), ctypes.byref(rid))
        if st != CHOL_OK:
            raise TileCholError(st, "chol_server_submit_solve", last_bad_arg())
        self.shapes[rid.value] = (n, nrhs)
        return rid.value

    def request_info(self, rid: int):
        """(factor handle or -1, precision, corrections, refactors) of a request."""
        f, p, c, r = ctypes.c_int64(-1), ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        st = lib.chol_server_request_info(self.h, rid, ctypes.byref(f), ctypes.byref(p), ctypes.byref(c),
                                          ctypes.byref(r))
        if st != CHOL_OK:
            raise TileCholError(st, "chol_server_request_info", last_bad_arg())
        return f.value, p.value, c.value, r.value

    def release_factor(self, factor: int) -> bool:
        return lib.chol_server_release_factor(self.h, int(factor)) == CHOL_OK

    def set_plan(self, fp32_min_n_loose: int, fp32_min_n_strict: int) -> None:
        """FP32 trailing products from these orders on (per tolerance class)
        for requests submitted from now on."""
        st = lib.chol_server_set_plan(self.h, int(fp32_min_n_loose), int(fp32_min_n_strict))
        if st != CHOL_OK:
            raise TileCholError(st, "chol_server_set_plan", last_bad_arg())

    def evictions(self) -> int:
        return int(lib.chol_server_evictions(self.h))

    def wait(self, rid: int, timeout: float = 60.0, want_x: bool = True):
        import numpy as np
        n, nrhs = self.shapes[rid]
        X = np.empty((n, nrhs)) if want_x else None
        eta, lat, info = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_int64(0)
        st = lib.chol_server_wait(self.h, rid, float(timeout), X.ctypes.data_as(ctypes.c_void_p) if want_x else None,
                                  ctypes.byref(eta), ctypes.byref(lat), ctypes.byref(info))
        if st < 0 and st not in (CHOL_EWORKSPACE, CHOL_ETIMEOUT, CHOL_ESTALLED):
            raise TileCholError(st, "chol_server_wait", last_bad_arg())
        return st, X, eta.value, lat.value, info.value

    def ticks(self) -> int:
        return int(lib.chol_server_ticks(self.h))

    def close(self):
        if self.h:
            st = lib.chol_server_destroy(self.h)
            self.h = ctypes.c_void_p()
            if st != CHOL_OK:
                raise TileCholError(st, "chol_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ----------------------------------------------------------- introspection
def chol_default_tile(n: int) -> int:
    return int(lib.chol_default_tile(n))


def chol_dag_counts(n: int, T: int):
    c = (ctypes.c_int64 * 5)()
    st = lib.chol_dag_counts(n, T, c)
    if st != CHOL_OK:
        raise TileCholError(st, "chol_dag_counts", last_bad_arg())
    return {"potrf": c[0], "trsm": c[1], "syrk": c[2], "gemm": c[3], "units": c[4]}


def chol_dag_enumerate(n: int, T: int, grid: int = 256):
    """Work units of the asynchronous schedule in ticket order as an
    (N, 6) int32 numpy array of {kind, J, I, a, K, b}."""
    import numpy as np
    total = int(lib.chol_dag_enumerate(n, T, grid, None, 0))
    if total < 0:
        raise TileCholError(total, "chol_dag_enumerate", last_bad_arg())
    out = np.zeros((total, 6), dtype=np.int32)
    got = lib.chol_dag_enumerate(n, T, grid, out.ctypes.data_as(_pi32), total)
    assert got == total
    return out


def chol_dag_forkjoin_update(n: int, T: int, J: int):
    """Units of the fork-join trailing-update launch of step J, launch order."""
    import numpy as np
    total = int(lib.chol_dag_forkjoin_update(n, T, J, None, 0))
    if total < 0:
        raise TileCholError(total, "chol_dag_forkjoin_update", last_bad_arg())
    out = np.zeros((total, 6), dtype=np.int32)
    lib.chol_dag_forkjoin_update(n, T, J, out.ctypes.data_as(_pi32), total)
    return out


TIMING_KINDS = {"potrf": 1, "trsm": 2, "update": 4, "panel": 8, "persistent": 16, "update_rest": 32}
_TIMING_NAMES = ("potrf", "trsm", "update", "panel", "persistent", "update_rest")


def chol_timing_enable(kinds) -> int:
    """Time the chol_factor launches of the given kinds on this thread
    (an iterable of names from TIMING_KINDS, or an int mask; empty / 0
    turns timing off).  Returns the previous mask."""
    mask = kinds if isinstance(kinds, int) else sum(TIMING_KINDS[k] for k in kinds)
    return int(lib.chol_timing_enable(mask))


def chol_timing_read(stream=None):
    """Summed device milliseconds and launch counts per kernel kind recorded
    since the last read: {"potrf": (ms, n), "trsm": ..., "update": ...,
    "panel": ..., "persistent": ..., "update_rest": ...}.  Synchronises the
    stream."""
    k = len(_TIMING_NAMES)
    ms = (ctypes.c_double * k)()
    cnt = (ctypes.c_int64 * k)()
    st = lib.chol_timing_read(_stream(stream), ms, cnt)
    if st != CHOL_OK:
        raise TileCholError(st, "chol_timing_read", last_bad_arg())
    return {_TIMING_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(k)}


def chol_async_grid() -> int:
    g = int(lib.chol_async_grid())
    if g < 0:
        raise TileCholError(g, "chol_async_grid")
    return g


def chol_set_wait_limit(seconds: float) -> float:
    return float(lib.chol_set_wait_limit(seconds))


def chol_set_lookahead(units: int) -> int:
    """Bulk units after each panel-chain link in the asynchronous ticket
    order (-1 default, 0 chain first, large = no lookahead)."""
    return int(lib.chol_set_lookahead(units))
