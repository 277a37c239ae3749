"""Parity of the mixed-precision factorization and of the refined solves
against the CPU references (oracle.potrf for FP64, oracle.mixed for the
low-precision algorithm), through the C ABI.

What is compared, and why that way:
  * integer-exact inputs (rows of L0 of norm 4): every rounding is exact,
    so every precision must return L0 bit for bit, for ragged tiles and
    tile widths that leave a partial k chunk;
  * prec FP64 without scaling or shift is chol_factor, bit for bit;
  * SE matrices: the factor values of a low-precision factorization have no
    reference rounding sequence (the FP32 sums run in a different order on
    the matrix cores), so the GPU factor is compared with the reference
    mixed factor (same algorithm, same rounding of the panel) and both with
    the FP64 factor: the GPU must be as close to FP64 as the reference is,
    and much closer to the reference than either is to FP64 when a shift
    dominates the difference;
  * refined solves: backward error <= 1e-12 computed on the host by the
    oracle from the returned X, forward error against the FP64 oracle
    solution, and iteration counts close to the reference's.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from oracle import mixed
from paper_2606_11937_amd import inputs

pytestmark = pytest.mark.gpu

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


def gpu_mixed(tc, A, T, prec, scale=True, shift=0.0, lda=None):
    import torch
    n = A.shape[0]
    lda = lda or n
    buf = torch.full((n, lda), float("nan"), dtype=torch.float64, device="cuda")
    buf[:, :n] = torch.from_numpy(A)
    info = tc.chol_factor_mixed(buf, T, prec, scale=scale, shift=shift)
    torch.cuda.synchronize()
    out = buf.cpu().numpy()
    return out, info


@pytest.fixture(scope="module")
def se2000():
    n = 2000
    A = inputs.se_kernel(n, seed=1)
    L64, info = oracle.potrf(A)
    assert info == 0
    B = np.random.default_rng(2).standard_normal((n, 16))
    return A, np.tril(L64), B, oracle.solve(np.tril(L64), B)


# ----------------------------------------------------------- exact cases
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("T", [128, 100, 256])
@pytest.mark.parametrize("scale", [True, False])
def test_integer_exact_every_precision(tc, prec, T, scale):
    A, L0 = inputs.integer_factor_norm4(700, seed=3)
    say(f"mixed integer-exact prec={prec} T={T} scale={scale}")
    L, info = gpu_mixed(tc, A, T, prec, scale, lda=712)
    assert info == 0
    assert np.array_equal(np.tril(L[:, :700]), L0)
    # strict upper triangle and padding untouched
    assert np.array_equal(np.triu(L[:, :700], 1), np.triu(A, 1))
    assert np.isnan(L[:, 700:]).all()


def test_fp64_precision_is_chol_factor(tc, se2000):
    import torch
    A = se2000[0]
    say("mixed fp64 == chol_factor")
    L1, i1 = gpu_mixed(tc, A, 256, "fp64", scale=False)
    d = torch.from_numpy(A).cuda()
    i2 = tc.chol_factor(d, 256, "fork_join")
    assert i1 == i2 == 0
    assert np.array_equal(np.tril(L1), np.tril(d.cpu().numpy()))


def test_nonpositive_diagonal_reported(tc):
    A = inputs.gg_plus_identity(300, seed=5)
    A[137, 137] = -1.0
    say("mixed not-SPD diagonal")
    for scale in (True, False):
        _, info = gpu_mixed(tc, A, 128, "fp32", scale)
        assert info == 138, (scale, info)


# ------------------------------------------------------ SE matrix factors
@pytest.mark.parametrize("prec,shift", [("fp32", 0.0), ("bf16", 0.064)])
def test_se_factor_against_references(tc, se2000, prec, shift):
    A, L64, _, _ = se2000
    say(f"mixed SE n=2000 prec={prec} shift={shift}")
    L, info = gpu_mixed(tc, A, 256, prec, shift=shift)
    Lo, io = mixed.potrf_mixed(A, 256, prec, shift=shift)
    assert info == io == 0
    e_gpu = oracle.row_scaled_error(L, L64, A)
    e_ref = oracle.row_scaled_error(Lo, L64, A)
    e_pair = oracle.row_scaled_error(L, Lo, A)
    say(f"  e_row gpu-fp64 {e_gpu:.3e} ref-fp64 {e_ref:.3e} gpu-ref {e_pair:.3e}")
    assert 0.5 * e_ref <= e_gpu <= 2.0 * e_ref
    if shift == 0.0:
        assert e_pair <= 2.0 * e_ref
    else:
        # the shift's deterministic change cancels between the two
        assert e_pair <= 0.05 * e_ref


def test_bf16_without_shift_breaks_down(tc, se2000):
    A = se2000[0]
    _, info = gpu_mixed(tc, A, 256, "bf16")
    _, io = mixed.potrf_mixed(A, 256, "bf16")
    say(f"bf16 unshifted: gpu info {info}, reference info {io}")
    assert io > 0 and info > 0


# -------------------------------------------------------- refined solves
def _refine(tc, A, L, B, T, method, max_iter=100):
    import torch
    dA = torch.from_numpy(A).cuda()
    dL = torch.from_numpy(np.ascontiguousarray(L)).cuda()
    dB = torch.from_numpy(B).cuda()
    X = torch.zeros_like(dB)
    ok, it, eta = tc.chol_solve_refine(dA, dL, dB, X, T, method, ETA_TOL, max_iter)
    torch.cuda.synchronize()
    assert np.array_equal(dB.cpu().numpy(), B)  # B is read only
    return ok, it, eta, X.cpu().numpy()


@pytest.mark.parametrize("prec,shift,method", [("fp32", 0.0, "ir"), ("fp32", 0.0, "pcg"), ("bf16", 0.064, "pcg")])
def test_refined_solve(tc, se2000, prec, shift, method):
    A, L64, B, Xr = se2000
    say(f"refine n=2000 prec={prec} shift={shift} method={method}")
    L, info = gpu_mixed(tc, A, 256, prec, shift=shift)
    assert info == 0
    ok, it, eta, X = _refine(tc, A, L, B, 256, method)
    Lo, _ = mixed.potrf_mixed(A, 256, prec, shift=shift)
    _, it_ref, _ = (mixed.refine_ir if method == "ir" else mixed.pcg)(A, Lo, B, max_iter=100)
    eta_host = oracle.backward_error(A, X, B)
    fe = np.abs(X - Xr).max() / np.abs(Xr).max()
    say(f"  converged={ok} it={it} (reference {it_ref}) eta={max(eta):.2e} host eta={eta_host:.2e} fe={fe:.2e}")
    assert ok and max(eta) <= ETA_TOL
    assert eta_host <= ETA_TOL
    assert fe <= 1e-8
    assert abs(it - it_ref) <= max(2, it_ref // 5)


def test_refine_with_exact_factor_needs_no_correction(tc, se2000):
    A, L64, B, Xr = se2000
    for method in ("ir", "pcg"):
        ok, it, eta, X = _refine(tc, A, L64, B, 256, method)
        assert ok and it == 0
        assert oracle.backward_error(A, X, B) <= 1e-14


def test_refine_reports_not_converged(tc, se2000):
    A, _, B, _ = se2000
    L, info = gpu_mixed(tc, A, 256, "bf16", shift=0.064)
    assert info == 0
    ok, it, eta, X = _refine(tc, A, L, B, 256, "ir", max_iter=3)
    assert not ok and it == 3 and max(eta) > ETA_TOL


def test_refine_ragged_rhs_and_strides(tc):
    """nrhs not a multiple of 16, leading dimensions above the widths."""
    import torch
    n = 777
    A = inputs.se_kernel(n, seed=4)
    B = np.random.default_rng(5).standard_normal((n, 19))
    L, info = gpu_mixed(tc, A, 128, "fp32")
    assert info == 0
    dA = torch.zeros((n, n + 5), dtype=torch.float64, device="cuda")
    dA[:, :n] = torch.from_numpy(A)
    dL = torch.zeros((n, n + 3), dtype=torch.float64, device="cuda")
    dL[:, :n] = torch.from_numpy(L)
    dB = torch.zeros((n, 24), dtype=torch.float64, device="cuda")
    dB[:, :19] = torch.from_numpy(B)
    X = torch.full((n, 21), 7.0, dtype=torch.float64, device="cuda")
    ok, it, eta = tc.chol_solve_refine(dA[:, :n], dL[:, :n], dB[:, :19], X[:, :19], 128, "ir", ETA_TOL, 10)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    assert ok and (Xh[:, 19:] == 7.0).all()
    assert oracle.backward_error(A, Xh[:, :19], B) <= ETA_TOL


# ------------------------------------------------- the full-size workload
@pytest.fixture(scope="module")
def se32k_fp32(tc):
    """n = 32768, T = 512, FP32 products: the mixed-precision workload in
    the launch configuration the benchmark times."""
    import torch
    n, T = 32768, 512
    A = inputs.se_kernel_device(n)
    L = A.clone()
    say("mixed n=32768 T=512 fp32 factor")
    info = tc.chol_factor_mixed(L, T, "fp32")
    torch.cuda.synchronize()
    assert info == 0
    yield A, L, T
    del A, L
    torch.cuda.empty_cache()


def test_full_size_leading_block(tc, se32k_fp32):
    """The leading m x m block of the factor depends only on the leading
    block of A (same tiles, same units, same scaling rows): bit-equal to the
    GPU factor of A[:m, :m], and close to the reference mixed factor."""
    A, L, T = se32k_fp32
    m = 2048
    Am = A[:m, :m].cpu().numpy()
    Lm, info = gpu_mixed(tc, Am, T, "fp32")
    assert info == 0
    got = np.tril(L[:m, :m].cpu().numpy())
    assert np.array_equal(got, np.tril(Lm))
    Lo, _ = mixed.potrf_mixed(Am, T, "fp32")
    L64 = np.tril(oracle.potrf(Am)[0])
    e_ref = oracle.row_scaled_error(Lo, L64, Am)
    e_gpu = oracle.row_scaled_error(got, L64, Am)
    say(f"  leading 2048: e_row gpu-fp64 {e_gpu:.3e} ref-fp64 {e_ref:.3e}")
    assert 0.5 * e_ref <= e_gpu <= 2.0 * e_ref


def test_full_size_refined_solve(tc, se32k_fp32):
    """16 right-hand sides refined to backward error <= 1e-12; the residual
    is recomputed independently with torch's FP64 matrix product."""
    import torch
    A, L, T = se32k_fp32
    n = A.shape[0]
    g = torch.Generator().manual_seed(2)
    B = torch.randn(n, 16, generator=g, dtype=torch.float64).cuda()
    X = torch.zeros_like(B)
    ok, it, eta = tc.chol_solve_refine(A, L, B, X, T, "ir", ETA_TOL, 10)
    say(f"  n=32768 refine: ok={ok} it={it} eta={max(eta):.2e}")
    assert ok and it <= 4
    As = torch.tril(A) + torch.tril(A, -1).T
    R = B - As @ X
    anorm = As.abs().sum(dim=1).max()
    eta_t = (R.abs().amax(dim=0) / (anorm * X.abs().amax(dim=0) + B.abs().amax(dim=0))).max().item()
    say(f"  torch eta {eta_t:.2e}")
    assert eta_t <= ETA_TOL
