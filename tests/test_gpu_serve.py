"""The factor + solve server (continuous batching and the FIFO baseline)
against the CPU oracle, through the C ABI.

Each request's matrix is assembled on the device from its points; the
oracle builds the same kernel matrix on the host (same formula, FP64) and
measures the backward error of the returned X.  A request's result must be
bit-identical alone and in a mix (tile side and precision depend only on
the request), admission must respect the arena (a request that can never
fit is rejected, the others proceed), and requests that do not fit at once
must wait for memory and still complete.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle

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


def make_request(rng, n):
    pts = rng.random((n, 2))
    ell = float(rng.uniform(0.05, 0.5))
    nrhs = int(rng.integers(1, 9))
    B = rng.standard_normal((n, nrhs))
    tol = 1e-6 if rng.random() < 0.5 else 1e-12
    return pts, B, ell, 1e-2, tol


def host_matrix(pts, ell, nugget):
    d0 = pts[:, 0:1] - pts[None, :, 0]
    d1 = pts[:, 1:2] - pts[None, :, 1]
    A = np.exp(-(d0 * d0 + d1 * d1) * (1.0 / (2.0 * ell * ell)))
    A[np.arange(len(pts)), np.arange(len(pts))] += nugget
    return A


def arena(nbytes):
    import torch
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("mode", ["continuous", "fifo"])
def test_server_results_against_oracle(tc, mode):
    rng = np.random.default_rng(60)
    sizes = [64, 65, 127, 128, 200, 333, 512, 700] + [int(v) for v in np.rint(np.exp(rng.uniform(np.log(64), np.log(800), 16)))]
    reqs = [make_request(rng, n) for n in sizes]
    say(f"server {mode}: {len(reqs)} requests")
    with tc.Server(arena(8 << 30), 256 << 20, mode) as srv:
        ids = [srv.submit(p, B, ell, nug, tol) for (p, B, ell, nug, tol) in reqs]
        for rid, (p, B, ell, nug, tol) in zip(ids, reqs):
            st, X, eta, lat, info = srv.wait(rid)
            assert st == tc.CHOL_OK, (st, len(p))
            A = host_matrix(p, ell, nug)
            eh = oracle.backward_error(A, X, B)
            assert eh <= tol and eta <= tol, (len(p), eh, eta)
            assert lat > 0
        if mode == "continuous":
            assert srv.ticks() >= 1
        else:
            assert srv.ticks() == len(reqs)


def test_server_right_hand_side_counts(tc):
    """Requests with every right-hand-side count the server takes (1 to 8)
    in one tick: the tick's solves run as one launch pair in which each item
    owns its own ticket range and takes its passes of four (one or two);
    results against the oracle."""
    rng = np.random.default_rng(64)
    reqs = []
    for n, k in ((100, 1), (333, 5), (640, 8), (257, 3), (700, 7), (65, 2), (129, 4), (512, 6)):
        pts = rng.random((n, 2))
        reqs.append((pts, rng.standard_normal((n, k)), float(rng.uniform(0.05, 0.5)), 1e-2, 1e-12))
    with tc.Server(arena(4 << 30), 256 << 20, "continuous") as srv:
        ids = [srv.submit(p, B, ell, nug, tol) for (p, B, ell, nug, tol) in reqs]
        for rid, (p, B, ell, nug, tol) in zip(ids, reqs):
            st, X, eta, lat, info = srv.wait(rid)
            assert st == tc.CHOL_OK, (st, len(p), B.shape[1])
            eh = oracle.backward_error(host_matrix(p, ell, nug), X, B)
            say(f"server n={len(p)} nrhs={B.shape[1]}: eta {eh:.2e}")
            assert eh <= tol and eta <= tol, (len(p), B.shape[1], eh, eta)


def test_server_result_independent_of_the_mix(tc):
    rng = np.random.default_rng(61)
    probe = [make_request(rng, n) for n in (100, 450, 999)]
    others = [make_request(rng, int(n)) for n in rng.integers(64, 900, 20)]
    alone = []
    with tc.Server(arena(8 << 30), 256 << 20, "continuous") as srv:
        for p, B, ell, nug, tol in probe:
            rid = srv.submit(p, B, ell, nug, tol)
            st, X, eta, lat, info = srv.wait(rid)
            assert st == tc.CHOL_OK
            alone.append((X, eta))
    with tc.Server(arena(8 << 30), 256 << 20, "continuous") as srv:
        ids = []
        for k, r in enumerate(others):
            ids.append(srv.submit(*r[:2], *r[2:]))
            if k % 7 == 3:
                ids.append(("probe", k // 7, srv.submit(*probe[k // 7][:2], *probe[k // 7][2:])))
        mixed = {}
        for rid in ids:
            if isinstance(rid, tuple):
                st, X, eta, lat, info = srv.wait(rid[2])
                assert st == tc.CHOL_OK
                mixed[rid[1]] = (X, eta)
            else:
                assert srv.wait(rid, want_x=False)[0] == tc.CHOL_OK
        assert srv.ticks() < len(ids)  # requests did share ticks
    for k in range(3):
        assert np.array_equal(alone[k][0], mixed[k][0]), k
        assert alone[k][1] == mixed[k][1]


def test_server_admission_by_footprint(tc):
    rng = np.random.default_rng(62)
    # about 40 MB of arena: a 2000-order request (32 MB matrix + workspace)
    # never fits alongside... and a 3000-order one never fits at all
    with tc.Server(arena(40 << 20), 64 << 20, "continuous") as srv:
        big = make_request(rng, 3000)
        small = [make_request(rng, 1200) for _ in range(8)]  # ~12 MB each: a few at a time
        rb = srv.submit(*big[:2], *big[2:])
        ids = [srv.submit(*r[:2], *r[2:]) for r in small]
        st, X, eta, lat, info = srv.wait(rb, want_x=False)
        assert st == tc.CHOL_EWORKSPACE
        for rid, (p, B, ell, nug, tol) in zip(ids, small):
            st, X, eta, lat, info = srv.wait(rid)
            assert st == tc.CHOL_OK
            assert oracle.backward_error(host_matrix(p, ell, nug), X, B) <= tol


# ------------------------------------------------- precision tiers, large n
def _plan(prec_code, tc):
    return {tc.CHOL_PREC_FP64: "fp64", tc.CHOL_PREC_FP32: "fp32"}[prec_code]


def _check_against_oracle(p, B, ell, nug, X, tol):
    A = host_matrix(p, ell, nug)
    eh = oracle.backward_error(A, X, B)
    assert eh <= tol, eh
    return eh


@pytest.mark.parametrize("n,tol", [(1500, 1e-6), (2600, 1e-12), (5000, 1e-12), (8192, 1e-6)])
def test_server_tiers_alone_and_in_a_mix(tc, n, tol):
    """Orders up to 8192 (multi-tile tiles of 512 and 1024 inside the
    batched launch): the request's result meets its tolerance by the
    oracle's measure, and is bit-identical served alone and in a mix of
    other requests of both tolerance classes."""
    rng = np.random.default_rng(70 + n)
    probe = (rng.random((n, 2)), rng.standard_normal((n, 3)), 0.25, 1e-2, tol)
    with tc.Server(arena(24 << 30), 1 << 30, "continuous") as srv:
        rid = srv.submit(*probe[:2], *probe[2:])
        st, X1, eta1, lat, info = srv.wait(rid, timeout=300)
        f, prec, corr, refac = srv.request_info(rid)
    say(f"server n={n} tol={tol}: status {st} prec {_plan(prec, tc)} corrections {corr} refactor {refac} "
        f"eta {eta1:.2e}")
    assert st == tc.CHOL_OK
    _check_against_oracle(*probe[:4], X1, tol)
    others = [make_request(rng, int(m)) for m in np.rint(np.exp(rng.uniform(np.log(64), np.log(4000), 12)))]
    with tc.Server(arena(24 << 30), 1 << 30, "continuous") as srv:
        ids = [srv.submit(*r[:2], *r[2:]) for r in others[:6]]
        rid = srv.submit(*probe[:2], *probe[2:])
        ids += [srv.submit(*r[:2], *r[2:]) for r in others[6:]]
        st, X2, eta2, lat, info = srv.wait(rid, timeout=300)
        for i in ids:
            assert srv.wait(i, timeout=300, want_x=False)[0] == tc.CHOL_OK
    assert st == tc.CHOL_OK
    assert np.array_equal(X1, X2) and eta1 == eta2


def test_server_precision_plan_and_refinement(tc):
    """The plan depends on (n, tol) only: FP32 trailing products for large
    orders, refined to the request's tolerance (strict requests take FP64
    corrections), FP64 below; all against the oracle."""
    rng = np.random.default_rng(75)
    reqs = [(rng.random((n, 2)), rng.standard_normal((n, 2)), 0.3, 1e-2, tol)
            for n, tol in ((600, 1e-6), (600, 1e-12), (3000, 1e-6), (3000, 1e-12), (6000, 1e-12))]
    with tc.Server(arena(24 << 30), 1 << 30, "continuous") as srv:
        ids = [srv.submit(*r[:2], *r[2:]) for r in reqs]
        seen = []
        for rid, r in zip(ids, reqs):
            st, X, eta, lat, info = srv.wait(rid, timeout=300)
            f, prec, corr, refac = srv.request_info(rid)
            say(f"  n={len(r[0])} tol={r[4]}: prec {_plan(prec, tc)} corrections {corr} refactor {refac} "
                f"eta {eta:.2e}")
            assert st == tc.CHOL_OK
            _check_against_oracle(*r[:4], X, r[4])
            seen.append((len(r[0]), r[4], prec))
    assert (600, 1e-12, tc.CHOL_PREC_FP64) in seen
    assert any(p == tc.CHOL_PREC_FP32 for _, _, p in seen)


def test_server_resident_factors(tc):
    """A request kept resident answers later solves without refactoring;
    the results meet their tolerance by the oracle's measure and equal a
    plain solve with the same factor; a released factor is gone."""
    rng = np.random.default_rng(76)
    n = 1800
    p, B, ell, nug = rng.random((n, 2)), rng.standard_normal((n, 2)), 0.2, 1e-2
    with tc.Server(arena(8 << 30), 256 << 20, "continuous") as srv:
        rid = srv.submit(p, B, ell, nug, 1e-12, keep=True)
        st, X, eta, lat, info = srv.wait(rid, timeout=120)
        assert st == tc.CHOL_OK
        f, prec, corr, refac = srv.request_info(rid)
        assert f >= 0
        ticks = srv.ticks()
        B2 = rng.standard_normal((n, 3))
        sid = srv.submit_solve(f, B2, 1e-12)
        st2, X2, eta2, lat2, info2 = srv.wait(sid, timeout=120)
        assert st2 == tc.CHOL_OK
        _check_against_oracle(p, B2, ell, nug, X2, 1e-12)
        assert srv.request_info(sid)[0] == f
        say(f"resident factor {f}: solve eta {eta2:.2e} latency {lat2 * 1e3:.2f} ms (factor + solve "
            f"{lat * 1e3:.2f} ms), ticks {srv.ticks() - ticks}")
        # the same right-hand sides give the same solution as the first request
        sid = srv.submit_solve(f, B, 1e-12)
        st3, X3, eta3, _, _ = srv.wait(sid, timeout=120)
        assert st3 == tc.CHOL_OK and np.array_equal(X3, X)
        assert srv.release_factor(f)
        with pytest.raises(tc.TileCholError) as e:
            srv.submit_solve(f, B2, 1e-12)
        assert e.value.status == tc.CHOL_ENOFACTOR


def test_server_evicts_least_recently_used_factors(tc):
    """Resident factors are evicted, least recently used first, when a new
    request needs their memory; solves against an evicted factor are
    refused, those against a surviving one still answer."""
    rng = np.random.default_rng(77)
    n = 1500  # about 18 MB resident per factor
    with tc.Server(arena(96 << 20), 64 << 20, "continuous") as srv:
        fs = []
        for k in range(4):
            r = (rng.random((n, 2)), rng.standard_normal((n, 1)), 0.2, 1e-2, 1e-12)
            rid = srv.submit(*r[:2], *r[2:], keep=True)
            assert srv.wait(rid, timeout=120)[0] == tc.CHOL_OK
            fs.append((srv.request_info(rid)[0], r))
        # a request that needs the memory of several of them
        big = make_request(rng, 2500)
        rid = srv.submit(*big[:2], *big[2:])
        assert srv.wait(rid, timeout=120)[0] == tc.CHOL_OK
        assert srv.evictions() >= 1
        gone = []
        for f, r in fs:
            try:
                sid = srv.submit_solve(f, r[1], 1e-12)
            except tc.TileCholError as e:
                assert e.status == tc.CHOL_ENOFACTOR
                gone.append(f)
                continue
            st, X, eta, _, _ = srv.wait(sid, timeout=120)
            assert st == tc.CHOL_OK
            _check_against_oracle(*r[:4], X, 1e-12)
        say(f"evicted {srv.evictions()} factors: {gone} of {[f for f, _ in fs]}")
        assert gone and gone == sorted(gone) and gone[0] == fs[0][0]  # oldest first


def test_server_stalled_request_restarts_once(tc):
    """A dependency wait that runs out restarts its request once; when the
    restart runs out too, the request is reported as stalled (X unspecified).
    The condition is forced from the host: the server is created with a
    wait limit of one microsecond, so every wait that is not satisfied at
    once ends (no kernel can hang).  A server with the normal limit then
    serves the same request to its tolerance."""
    rng = np.random.default_rng(81)
    n = 3000
    p, B, ell, nug = rng.random((n, 2)), rng.standard_normal((n, 2)), 0.2, 1e-2
    prev = tc.chol_set_wait_limit(1e-6)
    try:
        srv = tc.Server(arena(4 << 30), 256 << 20, "continuous")
    finally:
        tc.chol_set_wait_limit(prev)
    with srv:
        rid = srv.submit(p, B, ell, nug, 1e-12)
        st, X, eta, lat, info = srv.wait(rid, timeout=120)
        say(f"server with a 1 us wait limit: status {st} info {info} ticks {srv.ticks()}")
        assert st == tc.CHOL_ESTALLED
        assert srv.ticks() >= 2  # the first run and its restart
    with tc.Server(arena(4 << 30), 256 << 20, "continuous") as srv:
        rid = srv.submit(p, B, ell, nug, 1e-12)
        st, X, eta, lat, info = srv.wait(rid, timeout=120)
        assert st == tc.CHOL_OK
        _check_against_oracle(p, B, ell, nug, X, 1e-12)
