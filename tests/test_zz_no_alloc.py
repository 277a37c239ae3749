"""chol_factor_noalloc (the factorization with the library's fixed device
workspace, for callers that cannot allocate) against chol_factor with a
caller workspace, through the C ABI: bit-identical factors and infos on two
calls in a row, the second with a smaller input, for both schedules it
offers; and the size limit rejected before anything is enqueued."""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

from paper_2606_11937_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_11937_amd import tilechol
    return tilechol


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.mark.parametrize("sched", ["fork_join", "async_dag"])
def test_noalloc_matches_workspace_entry_point(tc, sched):
    import torch
    for n, T, seed in ((1000, 128, 81), (300, 64, 82)):  # the second call is smaller
        say(f"[noalloc] {sched} n={n} T={T}")
        A = inputs.gg_plus_identity(n, seed=seed)
        ref = torch.from_numpy(A).cuda()
        assert tc.chol_factor(ref, T, sched) == 0
        got = torch.from_numpy(A).cuda()
        assert tc.chol_factor_noalloc(got, T, sched) == 0
        torch.cuda.synchronize()
        assert torch.equal(torch.tril(got), torch.tril(ref)), (sched, n)


def test_noalloc_reports_not_spd_like_the_workspace_entry_point(tc):
    import torch
    A, L0 = inputs.integer_factor(400, seed=83)
    A[250, 250] = float(np.sum(L0[250, :250] ** 2)) - 1.0
    for sched in ("fork_join", "async_dag"):
        a = torch.from_numpy(A).cuda()
        b = torch.from_numpy(A).cuda()
        assert tc.chol_factor(a, 128, sched) == tc.chol_factor_noalloc(b, 128, sched) == 251


def test_noalloc_rejects_oversized_problems(tc):
    n = 1 << 18  # its workspace exceeds CHOL_NOALLOC_WORKSPACE; nothing is read
    st = tc.lib.chol_factor_noalloc(ctypes.c_void_p(0x1000), n, n, 128, 0, None, None)
    assert st == tc.CHOL_EWORKSPACE and tc.last_bad_arg() == 2
    assert tc.lib.chol_factor_noalloc(ctypes.c_void_p(0x1000), 100, 100, 128, 4, None, None) == tc.CHOL_EINVAL
    assert tc.last_bad_arg() == 5
