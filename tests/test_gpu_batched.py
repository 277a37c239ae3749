"""The one-launch batched factorization and solve against the CPU oracle and
against the single-matrix schedules, through the C ABI.

The batched kernel runs the asynchronous schedule's units with the same
bodies and the same per-block update order, so with the same tile side its
factor is bit-identical to chol_factor's; the oracle checks the numbers
(e_row <= 1e-10, solve backward error <= 1e-12, integer-exact inputs bit for
bit).  The solve unit (one workgroup, substitution over 64-row blocks) is
checked by its backward error and on integer-exact systems.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from paper_2606_11937_amd import inputs

pytestmark = pytest.mark.gpu

E_ROW_TOL = 1e-10
ETA_TOL = 1e-12


@pytest.fixture(scope="module")
def tc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_11937_amd import tilechol
    return tilechol


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def _dev(A):
    import torch
    return torch.from_numpy(np.ascontiguousarray(A)).cuda()


def lower_equal(X, Y):
    return np.array_equal(np.tril(X), np.tril(Y))


EDGE = [1, 2, 31, 64, 65, 127, 128, 129, 200, 255, 256, 257, 383, 640, 1000]


@pytest.mark.parametrize("tiles", ["tuned", "fixed"])
def test_batched_factor_solve_uneven(tc, tiles):
    import torch
    sizes = EDGE + inputs.batch_sizes(25, seed=7, lo=32, hi=700)
    As = [inputs.gg_plus_identity(n, seed=100 + i) for i, n in enumerate(sizes)]
    rng = np.random.default_rng(5)
    Bs = [rng.standard_normal(n) for n in sizes]
    Ts = None if tiles == "tuned" else [128 if n > 128 else max(n, 1) for n in sizes]
    dA = [_dev(A) for A in As]
    dB = [_dev(b) for b in Bs]
    say(f"batched factor+solve {len(sizes)} matrices, tiles={tiles}")
    infos = tc.chol_factor_solve_batched(dA, dB, Ts)
    torch.cuda.synchronize()
    assert infos == [0] * len(sizes)
    for i, (n, A, b) in enumerate(zip(sizes, As, Bs)):
        L = dA[i].cpu().numpy()
        Lref, info = oracle.potrf(A)
        assert info == 0
        e = oracle.row_scaled_error(L, Lref, A)
        assert e <= E_ROW_TOL, (n, e)
        x = dB[i].cpu().numpy()
        eta = oracle.backward_error(A, x, b)
        assert eta <= ETA_TOL, (n, eta)
        # same tile side, same units, same bodies: the single-matrix factor
        T = Ts[i] if Ts else tc.chol_batched_tile(n)
        d1 = _dev(A)
        assert tc.chol_factor(d1, T, "async_dag") == 0
        assert np.array_equal(np.tril(L), np.tril(d1.cpu().numpy())), n


def test_batched_integer_exact(tc):
    import torch
    sizes = [1, 7, 128, 129, 300, 513]
    As, L0s, Bs, Xs = [], [], [], []
    for i, n in enumerate(sizes):
        A, L0 = inputs.integer_factor(n, seed=20 + i, band=6)
        x = np.random.default_rng(30 + i).integers(-3, 4, n).astype(np.float64)
        As.append(A); L0s.append(L0); Xs.append(x); Bs.append(A @ x)
    dA = [_dev(A) for A in As]
    dB = [_dev(b) for b in Bs]
    infos = tc.chol_factor_solve_batched(dA, dB, [128] * len(sizes))
    torch.cuda.synchronize()
    assert infos == [0] * len(sizes)
    for i in range(len(sizes)):
        assert np.array_equal(np.tril(dA[i].cpu().numpy()), L0s[i])
        assert np.array_equal(dB[i].cpu().numpy(), Xs[i])


def test_batched_failure_is_isolated(tc):
    import torch
    sizes = [300, 500, 200, 64]
    As = [inputs.gg_plus_identity(n, seed=40 + i) for i, n in enumerate(sizes)]
    As[1][333, 333] = -5.0
    As[3][0, 0] = 0.0
    dA = [_dev(A) for A in As]
    infos = tc.chol_factor_batched(dA, [128] * 4)
    torch.cuda.synchronize()
    assert infos[1] == 334 and infos[3] == 1
    for i in (0, 2):
        assert infos[i] == 0
        Lref, _ = oracle.potrf(As[i])
        assert oracle.row_scaled_error(dA[i].cpu().numpy(), Lref, As[i]) <= E_ROW_TOL


def test_batched_skips_empty_and_strided(tc):
    import torch
    n, lda = 333, 400
    A = inputs.gg_plus_identity(n, seed=50)
    buf = torch.full((n, lda), float("nan"), dtype=torch.float64, device="cuda")
    buf[:, :n] = _dev(A)
    empty = torch.zeros((0, 1), dtype=torch.float64, device="cuda")
    infos = tc.chol_factor_batched([empty, buf[:, :n], empty], [1, 128, 1])
    torch.cuda.synchronize()
    assert infos == [0, 0, 0]
    out = buf.cpu().numpy()
    assert np.isnan(out[:, n:]).all()
    Lref, _ = oracle.potrf(A)
    assert oracle.row_scaled_error(out[:, :n], Lref, A) <= E_ROW_TOL


def test_batched_full_workload_sampled(tc):
    """The benchmark's workload: 4096 orders log-uniform in [32, 2048]
    (seed 3), A_i = G_i G_i^T / n_i + I built on the device, one right-hand
    side each, in one launch.  Every solve's backward error is recomputed
    with torch's FP64 products; eight matrices (the largest and the
    smallest among them) are checked against the oracle."""
    import torch
    sizes = inputs.batch_sizes(4096, seed=3)
    As = inputs.gg_batch_device(sizes, seed=3)
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    Bs = [torch.randn(n, generator=g, dtype=torch.float64, device="cuda") for n in sizes]
    order = np.argsort(sizes)
    pick = [int(order[-1]), int(order[-2]), int(order[0]), int(order[1])] + [int(order[k]) for k in (500, 1500, 2500, 3500)]
    keepA = {i: As[i].cpu().numpy() for i in pick}
    keepB = [b.clone() for b in Bs]
    Ls = [A.clone() for A in As]
    say("batched full workload: 4096 matrices")
    infos = tc.chol_factor_solve_batched(Ls, Bs)
    torch.cuda.synchronize()
    assert infos == [0] * len(sizes)
    worst = 0.0
    for A, L, x, b in zip(As, Ls, Bs, keepB):
        r = b - A @ x
        den = A.abs().sum(dim=1).max() * x.abs().max() + b.abs().max()
        worst = max(worst, (r.abs().max() / den).item())
    say(f"  worst backward error over the batch {worst:.2e}")
    assert worst <= ETA_TOL
    for i in pick:
        Lref, info = oracle.potrf(keepA[i])
        assert info == 0
        assert oracle.row_scaled_error(Ls[i].cpu().numpy(), Lref, keepA[i]) <= E_ROW_TOL, sizes[i]


# ------------------------------------------------ FP32 products + refinement
def _mixed_batch(tc, As, precs, Ts, tol=1e-12, max_iter=10, seed=0):
    import torch
    dA = [torch.from_numpy(A).cuda() for A in As]
    dL = [torch.full_like(a, float("nan")) for a in dA]
    rng = np.random.default_rng(seed)
    Bs = [rng.standard_normal(A.shape[0]) for A in As]
    dB = [torch.from_numpy(b).cuda() for b in Bs]
    dX = [torch.zeros_like(b) for b in dB]
    infos, its, etas = tc.chol_factor_solve_batched_mixed(dA, dL, dB, dX, Ts=Ts, precs=precs, tol=tol,
                                                          max_iter=max_iter)
    torch.cuda.synchronize()
    # the originals are read only
    for A, a, b, B in zip(As, dA, dB, Bs):
        assert np.array_equal(a.cpu().numpy(), A) and np.array_equal(b.cpu().numpy(), B)
    return infos, its, etas, [l.cpu().numpy() for l in dL], [x.cpu().numpy() for x in dX], Bs


@pytest.mark.parametrize("T", [128, 256])
def test_batched_fp32_matches_single_matrix_mixed(tc, T):
    """FP32 trailing products in the batched launch: each factor equals, bit
    for bit, the single-matrix mixed factorization with FP32 products (same
    tile bodies, same panel rounding, no scaling, no shift); every refined
    solution meets eta <= 1e-12 (checked by the oracle's measure) and agrees
    with the oracle's FP64 solve."""
    import torch
    ns = [1, 17, 100, 128, 129, 300, 513, 700, 1000]
    rng = np.random.default_rng(91)
    As = [inputs.gg_plus_identity(n, seed=int(rng.integers(1 << 30))) for n in ns]
    say(f"[batched fp32] T={T} sizes={ns}")
    infos, its, etas, Ls, Xs, Bs = _mixed_batch(tc, As, ["fp32"] * len(ns), [T] * len(ns), seed=92)
    assert infos == [0] * len(ns)
    for A, L, X, b, it, eta in zip(As, Ls, Xs, Bs, its, etas):
        n = A.shape[0]
        d = torch.from_numpy(A).cuda()
        assert tc.chol_factor_mixed(d, T, "fp32", scale=False) == 0
        assert lower_equal(L, d.cpu().numpy()), n
        e = oracle.backward_error(A, X, b)
        Lref, _ = oracle.potrf(A)
        xr = oracle.solve(Lref, b)
        say(f"  n={n} corrections={it} eta={eta:.2e} (oracle {e:.2e})")
        assert e <= ETA_TOL and eta <= ETA_TOL
        # the two residuals sum in different orders: they agree to about
        # n u relative to ||A|| ||x||, the denominator of eta
        assert abs(e - eta) <= 2.0 * n * 2.0 ** -53 + 1e-3 * e
        assert np.abs(X - xr).max() <= 1e-10 * max(1.0, np.abs(xr).max())
        if n > T:
            assert it >= 1  # the FP32 factor alone does not reach 1e-12


def test_batched_mixed_fp64_members_equal_the_fp64_launch(tc):
    import torch
    ns = [64, 300, 777]
    As = [inputs.gg_plus_identity(n, seed=93 + n) for n in ns]
    infos, its, etas, Ls, Xs, Bs = _mixed_batch(tc, As, ["fp64", "fp32", "fp64"], [128, 128, 256], seed=94)
    assert infos == [0, 0, 0]
    ref = [torch.from_numpy(A).cuda() for A in As]
    assert tc.chol_factor_batched(ref, Ts=[128, 128, 256]) == [0, 0, 0]
    for k in (0, 2):
        assert lower_equal(Ls[k], ref[k].cpu().numpy())
        assert its[k] == 0 and etas[k] <= ETA_TOL


def test_batched_fp32_integer_exact(tc):
    """Rows of norm 4: every panel entry is exact in FP32 and so is every
    product sum, so the FP32 batched factor is L0 bit for bit."""
    mats = [inputs.integer_factor_norm4(n, seed=95 + n) for n in (200, 333, 700)]
    infos, its, etas, Ls, Xs, Bs = _mixed_batch(tc, [A for A, _ in mats], ["fp32"] * 3, [128, 100, 256], seed=96)
    assert infos == [0, 0, 0]
    for (A, L0), L in zip(mats, Ls):
        assert lower_equal(L, L0)


def test_batched_fp32_failure_is_isolated(tc):
    good = inputs.gg_plus_identity(400, seed=97)
    bad = inputs.gg_plus_identity(400, seed=98)
    bad[250, 250] = -1.0
    infos, its, etas, Ls, Xs, Bs = _mixed_batch(tc, [good, bad, good], ["fp32"] * 3, [128] * 3, seed=99)
    assert infos[0] == 0 and infos[2] == 0 and infos[1] == oracle.potrf(bad)[1]
    assert oracle.backward_error(good, Xs[0], Bs[0]) <= ETA_TOL
