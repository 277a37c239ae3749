// kernels.hip -- gfx950 kernels and host launchers of the factorization
// schedules, the mixed-precision factor and the batched launch.
//
//   fork-join  (Methods, "fork-join collapsed"): per step J one launch for
//              POTRF(J), one for the TRSM panel of column J, one for the
//              collapsed SYRK+GEMM trailing update; kernel boundaries on the
//              stream are the barriers.
//   async DAG  (Methods, "task asynchronous" with explicit dependencies):
//              one persistent launch; workgroups take units in ticket order
//              (a topological order, see dag.h), wait until the per-block
//              counters say the unit's inputs are final, run it, and publish
//              its completion.  No global barrier.
//   the paper's naive fork-join and synchronous tasking variants, fork-join
//   with a one-step lookahead on two streams, and the fork-join launches as
//   a HIP graph with explicit dependency edges.
//
// Every schedule calls the same tile bodies from tile_ops.h with the same
// work-unit decomposition, so their factors are bit-identical.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "batch_plan.h"
#include "dag.h"
#include "gptr.h"
#include "launch.h"
#include "tile_ops.h"
#include "tile_ops_lp.h"

// ---------------------------------------------------------------- workspace
// [0, 256)              TcWsHeader (batch_plan.h)
// [256, +8*(M+1))       phase offsets (async only), rounded to 256 bytes
// then int32 pdone[NRB] (panel columns finalised per row block)
// then int32 ver[NRB*NRB] (updates applied per output block)
int64_t tc_ws_bytes(int64_t n, int64_t T) {
  TcGeom g = tc_geom(n, T, 0);
  int64_t b = 256;
  b += tc_round256(8 * ((int64_t)g.M + 1));
  b += tc_round256(4 * (int64_t)g.NRB);
  b += tc_round256(4 * (int64_t)g.NRB * g.NRB);
  return b;
}

static TcWs tc_ws_map(void* base, const TcGeom& g) {
  TcWs w;
  char* p = (char*)base;
  w.hdr = (TcWsHeader*)p;
  p += 256;
  w.offs = (int64_t*)p;
  p += tc_round256(8 * ((int64_t)g.M + 1));
  w.pdone = (int32_t*)p;
  p += tc_round256(4 * (int64_t)g.NRB);
  w.ver = (int32_t*)p;
  w.noop = 0;
  return w;
}

// ------------------------------------------------------------ small kernels
__global__ void tc_fill_zero(int32_t* p, int64_t count) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = 0;
}

// Phase offsets of the ticket space: offs[P] = first ticket of phase P.
__global__ void tc_phase_offsets(TcGeom g, int64_t* offs) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t acc = 0;
  for (int32_t P = 0; P < g.M; ++P) {
    offs[P] = acc;
    acc += tc_phase_size(g, P);
  }
  offs[g.M] = acc;
}

__device__ __forceinline__ bool tc_err_set(const TcWsHeader* h) {
  return __hip_atomic_load(&h->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__device__ __forceinline__ void tc_report_fail(TcWsHeader* h, int32_t code, int64_t info) {
  int32_t expected = 0;
  if (__hip_atomic_compare_exchange_strong(&h->error, &expected, code, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT)) {
    __hip_atomic_store(&h->info, info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------ unit runners
union alignas(512) TcSmem {
  TcTrsmSmem trsm;
  TcPotrfSmem potrf;
  TcUpdSmem upd;
};

// POTRF(J, s): the diagonal block gid(J, s).
__device__ __forceinline__ void tc_run_potrf(double* A, int64_t lda, const TcGeom& g, int32_t J, int32_t s,
                                             TcWsHeader* h, TcPotrfSmem& sm) {
  const int64_t d0 = tc_row0(g, J, s);
  const int bad = tc_potrf_tile(A + d0 * lda + d0, lda, tc_rows(g, J, s), sm);
  if (bad >= 0 && tc_tid() == 0) tc_report_fail(h, 1, d0 + bad + 1);
}

// TRSM(J, s, (I, a)): block (I, a) of sub-column gid(J, s).
__device__ __forceinline__ void tc_run_trsm(double* A, int64_t lda, const TcGeom& g, int32_t J, int32_t s, int32_t I,
                                            int32_t a, TcTrsmSmem& sm) {
  const int64_t r0 = tc_row0(g, I, a);
  const int64_t c0 = tc_row0(g, J, s);
  tc_trsm_block(A + r0 * lda + c0, A + c0 * lda + c0, lda, tc_rows(g, I, a), tc_rows(g, J, s), sm);
}

// Rows [64 h, 64 h + 64) of the same unit (h = 0, 1), for launches that give
// each half a workgroup of its own.
__device__ __forceinline__ void tc_run_trsm_half(double* A, int64_t lda, const TcGeom& g, int32_t J, int32_t s,
                                                 int32_t I, int32_t a, int h, TcTrsmSmem& sm) {
  const int mr = (int)tc_rows(g, I, a) - 64 * h;
  if (mr <= 0) return;
  const int64_t r0 = tc_row0(g, I, a) + 64 * h;
  const int64_t c0 = tc_row0(g, J, s);
  tc_trsm_rows(A + r0 * lda + c0, A + c0 * lda + c0, lda, mr < 64 ? mr : 64, tc_rows(g, J, s), sm);
}

// UPDATE(J, (I, a), (K, b)): K-depth the whole tile column J.
__device__ __forceinline__ void tc_run_update(double* A, int64_t lda, const TcGeom& g, const TcUnit& u, TcUpdSmem& sm) {
  const int64_t ri = tc_row0(g, u.I, u.a);
  const int64_t rk = tc_row0(g, u.K, u.b);
  const int64_t cj = (int64_t)u.J * g.T;
  tc_update_block(A + ri * lda + rk, A + ri * lda + cj, A + rk * lda + cj, lda, tc_rows(g, u.I, u.a),
                  tc_rows(g, u.K, u.b), (int)tc_tdim(g, u.J), ri == rk, sm);
}

// PANEL(J, s, (I, a), s'): block ((I, a), gid(J, s')) minus the product of
// the finished sub-column s in rows (I, a) and gid(J, s'); K-depth one block.
__device__ __forceinline__ void tc_run_panel(double* A, int64_t lda, const TcGeom& g, const TcUnit& u, TcUpdSmem& sm) {
  const int64_t ri = tc_row0(g, u.I, u.a);
  const int64_t rt = tc_row0(g, u.J, u.b);
  const int64_t cs = tc_row0(g, u.J, u.K);
  tc_update_block(A + ri * lda + rt, A + ri * lda + cs, A + rt * lda + cs, lda, tc_rows(g, u.I, u.a),
                  tc_rows(g, u.J, u.b), tc_rows(g, u.J, u.K), ri == rt, sm);
}

// UPDATE and PANEL units through one call of the block product, so that the
// persistent kernels, which run both kinds, hold one copy of its code.
__device__ __forceinline__ void tc_run_product(double* A, int64_t lda, const TcGeom& g, const TcUnit& u,
                                               TcUpdSmem& sm) {
  const bool up = u.kind == TC_UNIT_UPDATE;
  const int64_t ri = tc_row0(g, u.I, u.a);
  const int64_t rk = up ? tc_row0(g, u.K, u.b) : tc_row0(g, u.J, u.b);
  const int64_t ck = up ? (int64_t)u.J * g.T : tc_row0(g, u.J, u.K);
  const int mc = up ? tc_rows(g, u.K, u.b) : tc_rows(g, u.J, u.b);
  const int kd = up ? (int)tc_tdim(g, u.J) : tc_rows(g, u.J, u.K);
  tc_update_block(A + ri * lda + rk, A + ri * lda + ck, A + rk * lda + ck, lda, tc_rows(g, u.I, u.a), mc, kd,
                  ri == rk, sm);
}

// ---------------------------------------------------------- fork-join kernels
// The fork-join kernels declare only the shared memory their body uses (the
// persistent kernel needs the union of all of them).
__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_potrf(double* A, int64_t lda, TcGeom g, int32_t J, int32_t s,
                                                          TcWs ws) {
  __shared__ TcPotrfSmem sm;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  tc_run_potrf(A, lda, g, J, s, ws.hdr, sm);
}

__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_trsm(double* A, int64_t lda, TcGeom g, int32_t J, int32_t s,
                                                         TcWs ws) {
  __shared__ TcTrsmSmem sm;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  const TcUnit u = tc_decode_trsm(g, J, s, blockIdx.x >> 1);  // two workgroups per unit
  tc_run_trsm_half(A, lda, g, J, s, u.I, u.a, (int)(blockIdx.x & 1), sm);
}

// The panel-update and trailing-update launches each carry the next POTRF:
// launch index 0 is the update of the next diagonal block (sub-column s+1 of
// the panel, or sub-column 0 of the next tile column), which is its POTRF's
// only remaining input, so that workgroup factors the block right after
// updating it.  The POTRF then overlaps the rest of the launch instead of
// waiting for all of it plus a launch of its own; the operations and their
// order per block are unchanged.
union alignas(512) TcUpdPotrfSmem {
  TcUpdSmem upd;
  TcPotrfSmem potrf;
};

__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_panel(double* A, int64_t lda, TcGeom g, int32_t J, int32_t s,
                                                             TcWs ws) {
  __shared__ TcUpdPotrfSmem sm;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  const TcUnit u = tc_decode_panel(g, J, s, blockIdx.x);
  tc_run_panel(A, lda, g, u, sm.upd);
  if (blockIdx.x == 0) {  // the update of diagonal block gid(J, s+1)
    __syncthreads();
    tc_run_potrf(A, lda, g, J, s + 1, ws.hdr, sm.potrf);
  }
}

// Panel update without the fused POTRF (the naive variant launches every
// POTRF on its own).
__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_panel_only(double* A, int64_t lda, TcGeom g, int32_t J,
                                                                  int32_t s, TcWs ws) {
  __shared__ TcUpdSmem sm;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  const TcUnit u = tc_decode_panel(g, J, s, blockIdx.x);
  tc_run_panel(A, lda, g, u, sm);
}

__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_update(double* A, int64_t lda, TcGeom g, int32_t J, TcWs ws) {
  __shared__ TcUpdPotrfSmem sm;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  const TcUnit u = tc_decode_trailing(g, J, J, blockIdx.x);
  tc_run_update(A, lda, g, u, sm.upd);
  if (blockIdx.x == 0) {  // the last update of diagonal block gid(J+1, 0)
    __syncthreads();
    tc_run_potrf(A, lda, g, J + 1, 0, ws.hdr, sm.potrf);
  }
}

// Naive fork-join (the paper's first variant): the trailing update is
// parallel over tile rows I only; one workgroup walks the whole row, SYRK
// block (a, b <= a) then the GEMM tiles K = J+1 .. I-1, one block at a time.
// Same blocks, same arithmetic, far less parallelism.
__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_update_naive(double* A, int64_t lda, TcGeom g, int32_t J,
                                                                    TcWs ws) {
  __shared__ TcUpdSmem sm;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  const int32_t I = J + 1 + (int32_t)blockIdx.x;
  for (int32_t K = J + 1; K <= I; ++K)
    for (int32_t a = 0; a < tc_sb(g, I); ++a)
      for (int32_t b = 0; b < tc_sb(g, K); ++b) {
        if (I == K && b > a) continue;
        const TcUnit u = {TC_UNIT_UPDATE, J, I, a, K, b};
        tc_run_update(A, lda, g, u, sm);
        __syncthreads();
      }
}

// ------------------------------------------------- fork-join with lookahead
// The trailing update of step J split by tile column: units [first, first +
// gridDim.x) of the launch order (column-major over K).  The first range,
// column J+1 alone, carries the fused POTRF(J+1, 0) like the whole-update
// launch; the rest (columns > J+1) runs on a second stream while the panel
// of step J+1 is factored.
__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_update_range(double* A, int64_t lda, TcGeom g, int32_t J,
                                                                    TcWs ws, int64_t first) {
  __shared__ TcUpdPotrfSmem sm;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  const TcUnit u = tc_decode_trailing(g, J, J, first + blockIdx.x);
  tc_run_update(A, lda, g, u, sm.upd);
  if (first == 0 && blockIdx.x == 0) {  // the last update of diagonal block gid(J+1, 0)
    __syncthreads();
    tc_run_potrf(A, lda, g, J + 1, 0, ws.hdr, sm.potrf);
  }
}

// The bulk of step J's update (units [first, first + count) of the launch
// order above) by workgroups that take units from a counter until none is
// left.  The lookahead schedule launches it twice per step on one counter:
// first with fewer workgroups than fit on the chip, so that the panel chain
// of step J+1 finds free workgroup slots at once instead of queueing behind
// the bulk, then, behind that chain, into the slots the chain frees.  Each
// unit's body, and the order of the updates each block receives, are those
// of the one-unit-per-workgroup launch.
__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_update_pool(double* A, int64_t lda, TcGeom g, int32_t J,
                                                                   TcWs ws, int64_t first, int64_t count,
                                                                   unsigned long long* ctr) {
  __shared__ TcUpdSmem sm;
  __shared__ int64_t s_u;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  for (;;) {
    if (threadIdx.x == 0) s_u = (int64_t)atomicAdd(ctr, 1ull);
    __syncthreads();  // also: every thread is done with the previous unit's LDS
    const int64_t u = s_u;
    if (u >= count) break;
    tc_run_update(A, lda, g, tc_decode_trailing(g, J, J, first + u), sm);
    __syncthreads();  // s_u is rewritten next
  }
}

// ----------------------------------------------- low-precision trailing update
// Mixed precision: after the FP64 panel of step J is final, its
// rows below the diagonal tile are rounded once into the panel copy P (row r
// of A at row r of P, column J*T + k at column k); the trailing update then
// forms its products from P on the FP32 or BF16 matrix cores and subtracts
// them from the FP64 trailing matrix.  The unit decomposition, the fused
// POTRF(J+1, 0) and the per-block order of operations are those of the FP64
// fork-join kernels.
template <int PREC>
__global__ __launch_bounds__(TC_THREADS) void tc_round_panel(const double* A, int64_t lda, TcGeom g, int32_t J,
                                                             typename TcLp<PREC>::elem* P, int64_t ldp, TcWs ws) {
  if (tc_err_set(ws.hdr) || ws.noop) return;
  const int64_t kd = tc_tdim(g, J);
  const int64_t r0 = (int64_t)(J + 1) * g.T + (int64_t)blockIdx.x * 16;
  const int64_t c0 = (int64_t)J * g.T;
  for (int64_t idx = threadIdx.x; idx < 16 * kd; idx += TC_THREADS) {
    const int64_t rr = idx / kd, k = idx - rr * kd;
    const int64_t r = r0 + rr;
    if (r < g.n) P[r * ldp + k] = tc_round_lp<PREC>(A[r * lda + c0 + k]);
  }
}

// Trailing-update unit u of step J from the rounded panel copy P.
template <int PREC>
__device__ __forceinline__ void tc_run_update_lp(double* A, int64_t lda, const TcGeom& g, int32_t J, const TcUnit& u,
                                                 const typename TcLp<PREC>::elem* P, int64_t ldp, TcUpdSmem& sm) {
  const int64_t ri = tc_row0(g, u.I, u.a);
  const int64_t rk = tc_row0(g, u.K, u.b);
  tc_update_block_lp<PREC>(A + ri * lda + rk, P + ri * ldp, P + rk * ldp, lda, ldp, tc_rows(g, u.I, u.a),
                           tc_rows(g, u.K, u.b), (int)tc_tdim(g, J), ri == rk, sm);
}

// The low-precision factorization runs the lookahead schedule, with
// kernels as for FP64 (tc_fj_update_range, tc_fj_update_pool): units
// [first, first + gridDim.x) with the fused POTRF(J+1, 0) when first == 0,
// and the pool on a unit counter.  The unit bodies and the per-block update
// order are those of one launch per step, so the factor is too.
template <int PREC>
__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_update_lp_range(double* A, int64_t lda, TcGeom g, int32_t J,
                                                                       TcWs ws, const typename TcLp<PREC>::elem* P,
                                                                       int64_t ldp, int64_t first) {
  __shared__ TcUpdPotrfSmem sm;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  tc_run_update_lp<PREC>(A, lda, g, J, tc_decode_trailing(g, J, J, first + blockIdx.x), P, ldp, sm.upd);
  if (first == 0 && blockIdx.x == 0) {
    __syncthreads();
    tc_run_potrf(A, lda, g, J + 1, 0, ws.hdr, sm.potrf);
  }
}

template <int PREC>
__global__ __launch_bounds__(TC_THREADS, 2) void tc_fj_update_lp_pool(double* A, int64_t lda, TcGeom g, int32_t J,
                                                                      TcWs ws, const typename TcLp<PREC>::elem* P,
                                                                      int64_t ldp, int64_t first, int64_t count,
                                                                      unsigned long long* ctr) {
  __shared__ TcUpdSmem sm;
  __shared__ int64_t s_u;
  if (tc_err_set(ws.hdr) || ws.noop) return;
  for (;;) {
    if (threadIdx.x == 0) s_u = (int64_t)atomicAdd(ctr, 1ull);
    __syncthreads();  // also: every thread is done with the previous unit's LDS
    const int64_t u = s_u;
    if (u >= count) break;
    tc_run_update_lp<PREC>(A, lda, g, J, tc_decode_trailing(g, J, J, first + u), P, ldp, sm);
    __syncthreads();  // s_u is rewritten next
  }
}

// ---------------------------------------------------------- diagonal scaling
// d_i = sqrt(A_ii) by one workgroup; the first non-positive (or NaN)
// diagonal entry is reported as a failed pivot at that column.
__global__ __launch_bounds__(TC_THREADS) void tc_diag_scale(const double* A, int64_t lda, int64_t n, double* d,
                                                            TcWsHeader* h) {
  __shared__ int64_t first;
  if (threadIdx.x == 0) first = n;
  __syncthreads();
  int64_t mine = n;
  for (int64_t i = threadIdx.x; i < n; i += TC_THREADS) {
    const double a = A[i * lda + i];
    if (a > 0.0) {
      d[i] = sqrt(a);
    } else {
      d[i] = 1.0;
      if (i < mine) mine = i;
    }
  }
  if (mine < n) atomicMin((unsigned long long*)&first, (unsigned long long)mine);
  __syncthreads();
  if (threadIdx.x == 0 && first < n) tc_report_fail(h, 1, first + 1);
}

// Row i of the lower triangle: A_ij <- A_ij / (d_i d_j) (when d is given),
// then A_ii <- A_ii + shift.  One workgroup per row.
__global__ __launch_bounds__(TC_THREADS) void tc_scale_lower(double* A, int64_t lda, int64_t n, const double* d,
                                                             double shift, const TcWsHeader* h) {
  if (tc_err_set(h)) return;
  const int64_t i = blockIdx.x;
  double* row = A + i * lda;
  if (d != nullptr) {
    const double di = d[i];
    for (int64_t j = threadIdx.x; j <= i; j += TC_THREADS) row[j] = row[j] / (di * d[j]);
  }
  if (shift != 0.0) {
    __syncthreads();
    if (threadIdx.x == 0) row[i] = row[i] + shift;
  }
}

// Row i of the lower triangle: L_ij <- d_i L_ij (skipped after a failure).
__global__ __launch_bounds__(TC_THREADS) void tc_unscale_lower(double* A, int64_t lda, int64_t n, const double* d,
                                                               const TcWsHeader* h) {
  if (tc_err_set(h)) return;
  const int64_t i = blockIdx.x;
  double* row = A + i * lda;
  const double di = d[i];
  for (int64_t j = threadIdx.x; j <= i; j += TC_THREADS) row[j] = di * row[j];
}

// ------------------------------------------------------- persistent kernel
#define TC_MAX_PHASES 1024

// Dependency test and completion of unit u (the counter rules are in dag.h):
// the counters are read with relaxed agent-scope atomic loads (the caller
// issues the acquire fence once the unit is ready) and incremented with
// relaxed agent-scope atomic adds (after the workgroup's release fence).
__device__ __forceinline__ bool tc_unit_ready(const TcGeom& g, const TcWs& ws, const TcUnit& u) {
  return tc_unit_ready_with(g, ws.pdone, ws.ver, u, [](const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  });
}

__device__ __forceinline__ void tc_unit_publish(const TcGeom& g, const TcWs& ws, const TcUnit& u) {
  tc_unit_publish_with(g, ws.pdone, ws.ver, u, [](int32_t* p) {
    __hip_atomic_fetch_add(p, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  });
}

// Loop-invariant launch state of the persistent kernel that is not a pointer.
// It lives in LDS and is re-read on every pass (after a compiler-only memory
// barrier) instead of being held in scalar registers across the unit bodies:
// the update body alone needs nearly the whole register file, and state
// carried around the loop would otherwise be spilled inside its inner loop.
// The pointers stay kernel arguments so that the compiler still knows they
// address global memory (a pointer read back from LDS would turn every access
// into a flat instruction, which also counts against the LDS wait counter).
struct TcCtx {
  TcGeom g;
  int64_t wait_ticks;
  int64_t total;
};

__device__ __forceinline__ int64_t tc_ctx64(const int64_t& v) { return tc_uniform(v); }
__device__ __forceinline__ int32_t tc_ctx32(const int32_t& v) { return tc_uniform(v); }

__device__ __forceinline__ TcGeom tc_ctx_geom(const TcGeom& s) {
  TcGeom g;
  g.n = tc_ctx64(s.n);
  g.T = tc_ctx64(s.T);
  g.M = tc_ctx32(s.M);
  g.SB = tc_ctx32(s.SB);
  g.SBL = tc_ctx32(s.SBL);
  g.NRB = tc_ctx32(s.NRB);
  g.Q = tc_ctx64(s.Q);
  return g;
}

__global__ __launch_bounds__(TC_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void tc_async(
    double* A, int64_t lda, TcGeom g, TcWs ws, int64_t wait_ticks) {
  __shared__ TcSmem sm;
  // 32-bit copies of the phase offsets (the launcher checks that the ticket
  // count fits); 4 KB instead of 8 keeps two workgroups per CU
  __shared__ int32_t offs[TC_MAX_PHASES + 1];
  __shared__ TcCtx s_ctx;
  __shared__ TcUnit s_unit;
  __shared__ int32_t s_go;
  for (int i = threadIdx.x; i <= g.M; i += TC_THREADS) offs[i] = (int32_t)ws.offs[i];
  if (threadIdx.x == 0) {
    s_ctx.g = g;
    s_ctx.wait_ticks = wait_ticks;
    s_unit.kind = -1;
  }
  __syncthreads();
  if (threadIdx.x == 0) s_ctx.total = offs[g.M];
  __syncthreads();
  for (;;) {
    // nothing read from LDS before this point is reused after it
    asm volatile("" ::: "memory");
    // Thread 0 alone publishes the previous unit, takes the next ticket,
    // decodes it and waits for its inputs, all in one branch between two
    // barriers.  One thread-0 region per pass leaves the compiler no pair of
    // identical thread-0 conditions to thread into a second, divergent inner
    // loop that would run barriers without thread 0.
    if (threadIdx.x == 0) {
      const TcGeom cg = s_ctx.g;
      const TcUnit prev = s_unit;
      if (prev.kind >= 0 && !tc_err_set(ws.hdr)) tc_unit_publish(cg, ws, prev);
      const int64_t t = __hip_atomic_fetch_add(&ws.hdr->ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int32_t go = 0;
      if (t < s_ctx.total) {
        // phase of ticket t: last P with offs[P] <= t
        int32_t lo = 0, hi = cg.M - 1;
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if (offs[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const TcUnit u = tc_decode_in_phase(cg, lo, t - offs[lo]);
        go = 1;
        const uint64_t t0 = wall_clock64();
        while (!tc_unit_ready(cg, ws, u)) {
          if (tc_err_set(ws.hdr)) { go = 0; break; }
          if (wall_clock64() - t0 > (uint64_t)s_ctx.wait_ticks) { tc_report_fail(ws.hdr, 2, t + 1); go = 0; break; }
          __builtin_amdgcn_s_sleep(1);
        }
        if (go) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_unit = u;
      }
      s_go = go;
    }
    __syncthreads();
    if (!tc_uniform(s_go)) break;
    const TcUnit u = {tc_ctx32(s_unit.kind), tc_ctx32(s_unit.J), tc_ctx32(s_unit.I),
                      tc_ctx32(s_unit.a), tc_ctx32(s_unit.K), tc_ctx32(s_unit.b)};
    const TcGeom cg = tc_ctx_geom(s_ctx.g);
    if (ws.noop) {
      // measurement mode: the schedule's own cost only
    } else if (u.kind == TC_UNIT_UPDATE || u.kind == TC_UNIT_PANEL) {
      tc_run_product(A, lda, cg, u, sm.upd);
    } else if (u.kind == TC_UNIT_TRSM) {
      tc_run_trsm(A, lda, cg, u.J, u.K, u.I, u.a, sm.trsm);
    } else {
      tc_run_potrf(A, lda, cg, u.J, u.a, ws.hdr, sm.potrf);
    }
    // every wave makes its stores visible device-wide before the unit is published
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
  }
}

// ------------------------------------------------------------------ batched
// Many independent SPD matrices in one persistent launch.  Every matrix keeps
// its own tile DAG (geometry, counters, status header) and its own ticket
// order (the asynchronous schedule's, cut into its segments: the column
// updates that open phase P, then for each panel sub-column the POTRF, the
// TRSM column and the panel updates, each followed by its lookahead chunk of
// bulk updates, then the rest of the bulk).  The global ticket order takes
// segment k of phase P of every matrix that has one, largest matrix first,
// for (P, k) in order, and places a matrix's solve unit right after its last
// segment.  Each unit therefore waits only for units of its own matrix with
// smaller tickets, so the co-resident grid cannot deadlock, and the units at
// the same depth of all matrices sit together: the grid finds ready work
// while every matrix's chain advances.  A matrix whose factorization fails is
// skipped from then on; the others are unaffected.
// (descriptor, unit and slot records: batch_plan.h)

__global__ __launch_bounds__(TC_THREADS) void tc_batch_units(const TcBatchMat* __restrict__ mats,
                                                             const TcBatchSlot* __restrict__ slots,
                                                             TcBatchUnit* __restrict__ table) {
  const TcBatchSlot sl = slots[blockIdx.x];
  const TcGeom g = mats[sl.m].g;
  for (int64_t r = threadIdx.x; r < sl.size; r += TC_THREADS) table[sl.start + r] = tc_batch_slot_unit(sl, g, r);
}

// ---- one-workgroup solve with one right-hand side, in place in b
// (forward then backward substitution over 64-row blocks).  The finished
// part of x is folded into a block with reads along the stored rows of L, a
// whole 512-byte row segment per wave instruction and up to 32 of them in
// flight: forward, wave w takes the block's rows 16w..16w+15 and lane l the
// columns l (mod 64), its 16 per-row partial sums then reduced across the
// wave by a halving exchange; backward, wave w takes the 64-row chunks w,
// w + 4, ... below the block and lane l column l of the block, the four
// wave partials then added in wave order.  The diagonal block, loaded into
// registers before the fold and parked in LDS after it, is solved by wave 0
// in registers, one row per lane.  Every sum has a fixed order.
struct TcSolveSmem {
  double Lbb[64][65];
  double part[4][64];
};

// Sums of 16 per-lane partials (acc[q] for row q) over the 64 lanes of a
// wave: halving exchanges over lane bits 5, 4, 3, 2 leave lane l holding a
// partial of row (l >> 2), the exchanges over bits 0, 1 complete it.
__device__ __forceinline__ double tc_wave_rowsum16(double acc[16], int lane) {
#pragma unroll
  for (int h = 8, bit = 32; h >= 1; h >>= 1, bit >>= 1) {
    const bool hi = (lane & bit) != 0;
#pragma unroll
    for (int q = 0; q < h; ++q) {
      const double send = hi ? acc[q] : acc[q + h];
      const double keep = hi ? acc[q + h] : acc[q];
      acc[q] = keep + __shfl_xor(send, bit);
    }
  }
  double s = acc[0];
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  return s;
}

// One column of the right-hand sides: entries b[k * ldb].
__device__ __forceinline__ void tc_wg_solve(const double* __restrict__ L, int64_t lda, int64_t n,
                                            double* __restrict__ b, int64_t ldb, TcSolveSmem& sm) {
  const int tid = tc_tid(), lane = tid & 63, w = tid >> 6;
  const int wu = tc_uniform((int32_t)w);
  const int64_t nb = (n + 63) / 64;
  double dv[16];
  // the diagonal block, rows w + 4q, column lane, staged in LDS while the
  // first loads of the fold are in flight.  A full block is read whole (the
  // entries above its diagonal are never used); the last block reads zeros
  // past its end, and its padding rows take a unit pivot in the substitution.
  // (The thread index is re-read so that nothing lane-dependent is hoisted
  // out of the block loop and kept live across it.)
  auto load_diag = [&](int64_t r0, int nr) {
    const int t = tc_tid(), wl = t >> 6, ll = t & 63;
    const int32_t wo = (int32_t)(wl * lda) + ll;
    if (nr == 64) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double* Bq = L + (r0 + 4 * q) * lda + r0;
        dv[q] = Bq[wo];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double* Bq = L + (r0 + 4 * q) * lda + r0;
        dv[q] = (wl + 4 * q < nr && ll < nr) ? Bq[wo] : 0.0;
      }
    }
  };
  auto put_diag = [&]() {
#pragma unroll
    for (int q = 0; q < 16; ++q) sm.Lbb[w + 4 * q][lane] = dv[q];
  };
  for (int64_t blk = 0; blk < nb; ++blk) {
    const int64_t r0 = blk * 64;
    const int nr = n - r0 < 64 ? (int)(n - r0) : 64;
    // part_i = sum_{k < r0} L_ik x_k; rows past the block's end read its
    // last row (their sums are never used).  The row addresses are uniform:
    // lane l reads element l of each 64-column segment.
    double acc[16];
    int32_t rq[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      acc[q] = 0.0;
      rq[q] = 16 * wu + q < nr ? 16 * wu + q : nr - 1;
    }
    // two register sets: the loads of the next 64 columns are issued before
    // the current ones are folded in (the scheduling barriers keep the
    // compiler from interleaving each load with its use)
    double va[16], vb[16], xa = 0.0, xb = 0.0;
    auto fetch = [&](double(&v)[16], double& x, int64_t c0) {
      x = b[(c0 + lane) * ldb];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double* Lr = L + (r0 + rq[q]) * lda + c0;
        v[q] = Lr[lane];
      }
    };
    auto fold = [&](const double(&v)[16], double x) {
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = __builtin_fma(v[q], x, acc[q]);
    };
    // the block's own entries of b (wave 0 uses them after the fold), read
    // now so that their round trip overlaps the fold
    const double bo = b[(r0 + (lane < nr ? lane : nr - 1)) * ldb];
    if (r0 > 0) fetch(va, xa, 0);
    load_diag(r0, nr);  // its wait overlaps the first fetch
    put_diag();
    for (int64_t c0 = 0; c0 < r0; c0 += 128) {
      if (c0 + 64 < r0) fetch(vb, xb, c0 + 64);
      __builtin_amdgcn_sched_barrier(0);
      fold(va, xa);
      if (c0 + 64 >= r0) break;
      if (c0 + 128 < r0) fetch(va, xa, c0 + 128);
      __builtin_amdgcn_sched_barrier(0);
      fold(vb, xb);
    }
    const double s = tc_wave_rowsum16(acc, lane);
    if ((lane & 3) == 0) sm.part[0][16 * w + (lane >> 2)] = s;
    __syncthreads();
    if (w == 0) {
      double v = lane < nr ? bo - sm.part[0][lane] : 0.0;
      const double dl = lane < nr ? sm.Lbb[lane][lane] : 1.0, rl = 1.0 / dl;
      // eight pivots per pass (a rolled loop keeps the kernel's code small)
#pragma unroll 1
      for (int i0 = 0; i0 < nr; i0 += 8) {
        double l8[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) l8[k] = sm.Lbb[lane][i0 + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = i0 + k;
          const double xi = tc_div_rcp(tc_readlane(v, i), tc_readlane(dl, i), tc_readlane(rl, i));
          if (lane == i) v = xi;
          else if (lane > i) v = v - l8[k] * xi;
        }
      }
      if (lane < nr) b[(r0 + lane) * ldb] = v;
    }
    __syncthreads();
  }
  for (int64_t blk = nb - 1; blk >= 0; --blk) {
    const int64_t r0 = blk * 64;
    const int nr = n - r0 < 64 ? (int)(n - r0) : 64;
    // part_j = sum_{k >= r0 + 64} L_kj x_k for column j = r0 + lane (every
    // block but the last, whose loop is empty, has 64 columns).  Wave w takes
    // the 64-row chunks w, w + 4, ... below the block, 16 rows at a time,
    // with the next 16 rows' loads in flight; rows past n read row n - 1
    // against a zero x.
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    double va[16], vb[16], xa = 0.0, xb = 0.0;
    auto fetch = [&](double(&v)[16], double& x, int64_t k) {
      const int64_t kx = k + (lane & 15);
      x = kx < n ? b[kx * ldb] : 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t kr = k + q < n ? k + q : n - 1;
        const double* Lr = L + kr * lda + r0;
        v[q] = Lr[lane];
      }
    };
    auto fold = [&](const double(&v)[16], double x) {
#pragma unroll
      for (int q = 0; q < 16; ++q) a4[q & 3] = __builtin_fma(v[q], tc_readlane(x, q), a4[q & 3]);
    };
    const int64_t kb = r0 + 64;
    auto gk = [&](int64_t j) { return kb + 64 * (wu + 4 * (j >> 2)) + 16 * (j & 3); };
    const double bo = b[(r0 + (lane < nr ? lane : nr - 1)) * ldb];  // as in the forward sweep
    if (gk(0) < n) fetch(va, xa, gk(0));
    load_diag(r0, nr);
    put_diag();
    for (int64_t j = 0; gk(j) < n; j += 2) {
      if (gk(j + 1) < n) fetch(vb, xb, gk(j + 1));
      __builtin_amdgcn_sched_barrier(0);
      fold(va, xa);
      if (gk(j + 1) >= n) break;
      if (gk(j + 2) < n) fetch(va, xa, gk(j + 2));
      __builtin_amdgcn_sched_barrier(0);
      fold(vb, xb);
    }
    sm.part[w][lane] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    __syncthreads();
    if (w == 0) {
      const double s = (sm.part[0][lane] + sm.part[1][lane]) + (sm.part[2][lane] + sm.part[3][lane]);
      double v = lane < nr ? bo - s : 0.0;
      const double dl = lane < nr ? sm.Lbb[lane][lane] : 1.0, rl = 1.0 / dl;
      // pivots from the last one down, eight per pass (padding rows give 0)
#pragma unroll 1
      for (int i0 = ((nr - 1) >> 3) << 3; i0 >= 0; i0 -= 8) {
        double l8[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) l8[k] = sm.Lbb[i0 + k][lane];
#pragma unroll
        for (int k = 7; k >= 0; --k) {
          const int i = i0 + k;
          const double xi = tc_div_rcp(tc_readlane(v, i), tc_readlane(dl, i), tc_readlane(rl, i));
          if (lane == i) v = xi;
          else if (lane < i) v = v - l8[k] * xi;
        }
      }
      if (lane < nr) b[(r0 + lane) * ldb] = v;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ TcWs tc_global_ws(const TcWs& w) {
  TcWs g = w;
  g.hdr = tc_global(w.hdr);
  g.offs = tc_global(w.offs);
  g.pdone = tc_global(w.pdone);
  g.ver = tc_global(w.ver);
  return g;
}

// ---- one-workgroup residual r = b0 - A0 x of one matrix (A0 symmetric, its
// lower triangle read), with the norms of the backward error.  Rows go in
// 64-row blocks; for each block the 64 x 64 tiles of the symmetric matrix
// are staged in LDS in column-block order (a tile above the diagonal is read
// transposed from the lower triangle), and thread (row r, part p) sums its
// 16 columns of every tile in order; the four parts are added in order
// p = 0..3.  Deterministic.  Returns, in red[0..3] (LDS, after a barrier),
// max |r_i|, max |x_i|, max |b0_i| and max_i sum_j |A0_ij|.
struct TcResSmem {
  double t[64][65];
  double xs[64];
  double part[4][64];
  double apart[4][64];
  double red[4][TC_THREADS];
};

__device__ __forceinline__ void tc_wg_residual(const double* __restrict__ A0, int64_t lda0, int64_t n,
                                               const double* __restrict__ x, const double* __restrict__ b0,
                                               double* __restrict__ r, TcResSmem& sm) {
  const int tid = tc_tid(), rr = tid >> 2, p = tid & 3;
  double rmax = 0.0, xmax = 0.0, bmax = 0.0, amax = 0.0;
  for (int64_t R0 = 0; R0 < n; R0 += 64) {
    double acc = 0.0, asum = 0.0;
    for (int64_t C0 = 0; C0 < n; C0 += 64) {
      if (tid < 64) sm.xs[tid] = C0 + tid < n ? x[C0 + tid] : 0.0;
      // coalesced: along the stored row of the lower triangle.  All 16 loads
      // of a thread are issued before the first is stored (from clamped,
      // in-range positions; entries past n are then replaced by zero).
      double tv[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = tid + q * TC_THREADS;
        const int i = C0 > R0 ? (e & 63) : (e >> 6), k = C0 > R0 ? (e >> 6) : (e & 63);
        const int64_t gi = R0 + i < n ? R0 + i : n - 1, gj = C0 + k < n ? C0 + k : n - 1;
        tv[q] = gj <= gi ? A0[gi * lda0 + gj] : A0[gj * lda0 + gi];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = tid + q * TC_THREADS;
        const int i = C0 > R0 ? (e & 63) : (e >> 6), k = C0 > R0 ? (e >> 6) : (e & 63);
        sm.t[i][k] = (R0 + i < n && C0 + k < n) ? tv[q] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < 16; ++kk) {
        const double v = sm.t[rr][16 * p + kk];
        acc += v * sm.xs[16 * p + kk];
        asum += fabs(v);
      }
      __syncthreads();
    }
    sm.part[p][rr] = acc;
    sm.apart[p][rr] = asum;
    __syncthreads();
    if (p == 0 && R0 + rr < n) {
      const int64_t i = R0 + rr;
      const double sum = sm.part[0][rr] + sm.part[1][rr] + sm.part[2][rr] + sm.part[3][rr];
      const double as = sm.apart[0][rr] + sm.apart[1][rr] + sm.apart[2][rr] + sm.apart[3][rr];
      const double bi = b0[i], ri = bi - sum;
      r[i] = ri;
      rmax = fmax(rmax, fabs(ri));
      xmax = fmax(xmax, fabs(x[i]));
      bmax = fmax(bmax, fabs(bi));
      amax = fmax(amax, as);
    }
    __syncthreads();
  }
  sm.red[0][tid] = rmax;
  sm.red[1][tid] = xmax;
  sm.red[2][tid] = bmax;
  sm.red[3][tid] = amax;
  __syncthreads();
  if (tid < 4) {
    double m = 0.0;
    for (int t = 0; t < TC_THREADS; ++t) m = fmax(m, sm.red[tid][t]);
    sm.red[tid][0] = m;
  }
  __syncthreads();
}

union alignas(512) TcBatchSmem {
  TcSmem f;
  TcSolveSmem s;
  TcResSmem r;
};

// The solve unit of one matrix.  Plain: each of the nrhs columns of B
// (leading dimension ldb) in turn, in place.  With refinement (one
// right-hand side, in place in x = B, which holds b0 on entry): x = (L L^T)^-1
// b0, then while the backward error ||b0 - A0 x||_inf / (||A0||_inf ||x||_inf
// + ||b0||_inf) exceeds tol and fewer than max_iter corrections were applied,
// x += (L L^T)^-1 (b0 - A0 x); {eta, corrections} go to stat.  Every pass
// goes through one call of the solve, which keeps the kernel's code small.
__device__ __forceinline__ void tc_wg_solve_unit(const double* __restrict__ L, int64_t lda, int64_t n, double* B,
                                                 int64_t nrhs, int64_t ldb, bool refine, const double* A0,
                                                 int64_t lda0, const double* b0, double* R, double tol,
                                                 int64_t max_iter, double* stat, TcBatchSmem& sm) {
  if (!refine && nrhs <= 0) return;
  double eta = 0.0;
  int64_t p = 0;
  for (;; ++p) {
    // refinement: the first pass solves in x, the later ones for the correction in R
    tc_wg_solve(L, lda, n, refine ? (p == 0 ? B : R) : B + p, refine ? 1 : ldb, sm.s);
    if (!refine) {
      if (p + 1 >= nrhs) break;
      continue;
    }
    if (p > 0) {
      for (int64_t i = tc_tid(); i < n; i += TC_THREADS) B[i] = B[i] + R[i];
      __syncthreads();
    }
    tc_wg_residual(A0, lda0, n, B, b0, R, sm.r);
    const double den = sm.r.red[3][0] * sm.r.red[1][0] + sm.r.red[2][0];
    eta = tc_uniform(den > 0.0 ? sm.r.red[0][0] / den : 0.0);
    __syncthreads();
    if (!(eta > tol) || p >= max_iter) break;
  }
  if (refine && tc_tid() == 0) {
    stat[0] = eta;
    stat[1] = (double)p;
  }
}

// Round row block (I, a)'s finished panel strip of tile column J to FP32 into
// P (same row and column indices, leading dimension ldp).  Called by the
// workgroup that just ran the strip's last TRSM, after a barrier.
__device__ __forceinline__ void tc_round_strip(const double* __restrict__ A, int64_t lda, const TcGeom& g,
                                               int32_t J, int32_t I, int32_t a, float* __restrict__ P, int64_t ldp) {
  const int64_t r0 = tc_row0(g, I, a), c0 = (int64_t)J * g.T;
  const int mr = tc_rows(g, I, a);
  const int64_t kd = tc_tdim(g, J);
  // eight rows at a time, their loads issued before the first store (rows
  // past the block's end re-read its last row and are not stored)
  for (int rb = 0; rb < mr; rb += 8)
    for (int64_t k = tc_tid(); k < kd; k += TC_THREADS) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int rr = rb + q < mr ? rb + q : mr - 1;
        v[q] = A[(r0 + rr) * lda + c0 + k];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (rb + q < mr) P[(r0 + rb + q) * ldp + c0 + k] = tc_round_lp<TC_PREC_FP32>(v[q]);
    }
}

__global__ __launch_bounds__(TC_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void tc_batched(
    const TcBatchMat* __restrict__ mats, const TcBatchUnit* __restrict__ table, int64_t total, int32_t* ticket,
    int64_t wait_ticks) {
  __shared__ TcBatchSmem sm;
  __shared__ TcBatchMat s_mat;
  __shared__ TcUnit s_unit;
  __shared__ int32_t s_go, s_run;
  if (threadIdx.x == 0) {
    s_unit.kind = -1;
    s_run = 0;
  }
  __syncthreads();
  for (;;) {
    asm volatile("" ::: "memory");
    // thread 0: publish the previous unit, take a ticket, wait for its inputs
    // (one thread-0 region per pass, as in the single-matrix kernel)
    if (threadIdx.x == 0) {
      if (s_unit.kind >= 0 && s_unit.kind != TC_UNIT_SOLVE && s_run) {
        const TcWs pws = tc_global_ws(s_mat.ws);
        if (!tc_err_set(pws.hdr)) {
          tc_unit_publish(s_mat.g, pws, s_unit);
          __hip_atomic_fetch_add(tc_global(s_mat.done), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      const int64_t t = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      int32_t go = 0, run = 0;
      if (t < total) {
        const TcBatchUnit e = table[t];
        s_mat = mats[e.m];
        const TcUnit u = {e.kind, e.J, e.I, e.a, e.K, e.b};
        go = 1;
        run = 1;
        const TcWs mws = tc_global_ws(s_mat.ws);
        const int32_t* mdone = tc_global(s_mat.done);
        const uint64_t t0 = wall_clock64();
        for (;;) {
          if (tc_err_set(mws.hdr)) { run = 0; break; }
          const bool ready = u.kind == TC_UNIT_SOLVE
                                 ? __hip_atomic_load(mdone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                                       s_mat.nunits
                                 : tc_unit_ready(s_mat.g, mws, u);
          if (ready) break;
          if (wall_clock64() - t0 > (uint64_t)wait_ticks) { tc_report_fail(mws.hdr, 2, t + 1); run = 0; break; }
          __builtin_amdgcn_s_sleep(1);
        }
        if (run) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_unit = u;
      }
      s_go = go;
      s_run = run;
    }
    __syncthreads();
    if (!tc_uniform(s_go)) break;
    if (tc_uniform(s_run)) {
      const TcUnit u = {tc_ctx32(s_unit.kind), tc_ctx32(s_unit.J), tc_ctx32(s_unit.I),
                        tc_ctx32(s_unit.a), tc_ctx32(s_unit.K), tc_ctx32(s_unit.b)};
      const TcGeom cg = tc_ctx_geom(s_mat.g);
      double* A = tc_global(s_mat.A);
      const int64_t lda = tc_ctx64(s_mat.lda);
      const int32_t prec = tc_ctx32(s_mat.prec);
      if (u.kind == TC_UNIT_UPDATE && prec == TC_PREC_FP32) {
        const float* P = tc_global(s_mat.P);
        const int64_t ldp = tc_ctx64(s_mat.ldp);
        const int64_t ri = tc_row0(cg, u.I, u.a), rk = tc_row0(cg, u.K, u.b), cj = (int64_t)u.J * cg.T;
        tc_update_block_lp<TC_PREC_FP32>(A + ri * lda + rk, P + ri * ldp + cj, P + rk * ldp + cj, lda, ldp,
                                         tc_rows(cg, u.I, u.a), tc_rows(cg, u.K, u.b), (int)tc_tdim(cg, u.J),
                                         ri == rk, sm.f.upd);
      } else if (u.kind == TC_UNIT_UPDATE || u.kind == TC_UNIT_PANEL) {
        tc_run_product(A, lda, cg, u, sm.f.upd);
      } else if (u.kind == TC_UNIT_TRSM) {
        tc_run_trsm(A, lda, cg, u.J, u.K, u.I, u.a, sm.f.trsm);
        if (prec == TC_PREC_FP32 && u.K == tc_sb(cg, u.J) - 1 && u.I > u.J) {
          __syncthreads();  // the strip's new block is visible to the whole workgroup
          tc_round_strip(A, lda, cg, u.J, u.I, u.a, tc_global(s_mat.P), tc_ctx64(s_mat.ldp));
        }
      } else if (u.kind == TC_UNIT_POTRF) {
        tc_run_potrf(A, lda, cg, u.J, u.a, tc_global(s_mat.ws.hdr), sm.f.potrf);
      } else {
        tc_wg_solve_unit(A, lda, cg.n, tc_global(s_mat.b), tc_ctx64(s_mat.nrhs), tc_ctx64(s_mat.ldb),
                         tc_ctx32(s_mat.refine) != 0, tc_global(s_mat.A0), tc_ctx64(s_mat.lda0), tc_global(s_mat.b0),
                         tc_global(s_mat.R), tc_uniform(s_mat.tol), tc_ctx64(s_mat.max_iter), tc_global(s_mat.stat),
                         sm);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
  }
}

// Synchronous tasking (the paper's task-synchronous variant, tasks with a
// taskwait after each phase): one persistent launch walks the phases of the
// blocked program order, for each step J and sub-column s the POTRF, the
// TRSM column and the panel update, then the trailing update; inside a phase
// workgroup w takes units w, w + grid, ...; a grid-wide barrier separates
// phases.  The units, and each block's update order, are those of the other
// schedules, so the factor is the same bits.  Every barrier wait is bounded
// by the wall-clock limit and by the error flag.
__device__ __forceinline__ int32_t tc_grid_barrier(const TcWs& ws, int64_t target, int64_t wait_ticks,
                                                   int32_t* s_go) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t go = 1;
    __hip_atomic_fetch_add(&ws.hdr->bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(&ws.hdr->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (tc_err_set(ws.hdr)) { go = 0; break; }
      if (wall_clock64() - t0 > (uint64_t)wait_ticks) { tc_report_fail(ws.hdr, 2, 0); go = 0; break; }
      __builtin_amdgcn_s_sleep(1);
    }
    if (go) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_go = go;
  }
  __syncthreads();
  return tc_uniform(*s_go);
}

__global__ __launch_bounds__(TC_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void tc_sync(
    double* A, int64_t lda, TcGeom g, TcWs ws, int64_t wait_ticks) {
  __shared__ TcSmem sm;
  __shared__ int32_t s_go;
  const int64_t grid = gridDim.x;
  int64_t phase = 0;
  for (int32_t J = 0; J < g.M; ++J) {
    const int32_t sbJ = tc_sb(g, J);
    for (int32_t sc = 0; sc < sbJ; ++sc) {
      for (int32_t link = 0; link < 3; ++link) {
        const int64_t cnt = link == 0 ? 1 : link == 1 ? tc_trsm_count(g, J, sc) : tc_panel_count(g, J, sc);
        for (int64_t i = blockIdx.x; i < cnt && !ws.noop; i += grid) {
          if (link == 0) {
            tc_run_potrf(A, lda, g, J, sc, ws.hdr, sm.potrf);
          } else if (link == 1) {
            const TcUnit u = tc_decode_trsm(g, J, sc, i);
            tc_run_trsm(A, lda, g, J, sc, u.I, u.a, sm.trsm);
          } else {
            const TcUnit u = tc_decode_panel(g, J, sc, i);
            tc_run_panel(A, lda, g, u, sm.upd);
          }
          __syncthreads();
        }
        if (cnt > 0) {
          ++phase;
          if (!tc_grid_barrier(ws, phase * grid, wait_ticks, &s_go)) return;
        }
      }
    }
    const int64_t nu = tc_trailing_units(g, J);
    for (int64_t i = blockIdx.x; i < nu && !ws.noop; i += grid) {
      const TcUnit u = tc_decode_trailing(g, J, J, i);
      tc_run_update(A, lda, g, u, sm.upd);
      __syncthreads();
    }
    if (nu > 0) {
      ++phase;
      if (!tc_grid_barrier(ws, phase * grid, wait_ticks, &s_go)) return;
    }
  }
}

// ------------------------------------------------------------ host launchers
static int tc_chk(hipError_t e) { return e == hipSuccess ? 0 : TC_LAUNCH_EDEVICE; }

// Per-launch timing (a measurement aid, off by default): when enabled on the
// calling thread, every tile-operation launch and the persistent launch are
// bracketed by a pair of HIP events on the launch stream.  Events are created
// on first use and reused; they are runtime objects, not device memory.
namespace {
struct TcTimer {
  int mask = 0;  // bit k: time launches of kind k
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int kind;
    hipEvent_t a, b;
    hipEvent_t b2;  // a second end event on another stream (or null): the interval ends at the later one
  };
  std::vector<Rec> recs;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};
thread_local TcTimer g_timer;

// Launch `fn` on `st`, timed under `kind` when the timer is on.
template <typename F>
void tc_timed(int kind, hipStream_t st, F fn) {
  if (!(g_timer.mask >> kind & 1)) {
    fn();
    return;
  }
  hipEvent_t a = g_timer.next(), b = g_timer.next();
  if (a == nullptr || b == nullptr) {
    fn();
    return;
  }
  (void)hipEventRecord(a, st);
  fn();
  (void)hipEventRecord(b, st);
  g_timer.recs.push_back({kind, a, b, nullptr});
}
}  // namespace

// Index of the last timed record (or -1 when `kind` is not timed), and
// ending that record also at an event recorded now on `st`.
static int tc_timed_last(int kind) { return (g_timer.mask >> kind & 1) ? (int)g_timer.recs.size() - 1 : -1; }
static void tc_timed_extend(int rec, hipStream_t st) {
  if (rec < 0 || rec >= (int)g_timer.recs.size()) return;
  hipEvent_t e = g_timer.next();
  if (e == nullptr || hipEventRecord(e, st) != hipSuccess) return;
  g_timer.recs[rec].b2 = e;
}

int tc_timing_enable(int mask) {
  const int prev = g_timer.mask;
  g_timer.mask = mask & ((1 << TC_TIMING_KINDS) - 1);
  return prev;
}

int tc_timing_read(hipStream_t st, double ms[TC_TIMING_KINDS], int64_t cnt[TC_TIMING_KINDS]) {
  for (int k = 0; k < TC_TIMING_KINDS; ++k) {
    ms[k] = 0.0;
    cnt[k] = 0;
  }
  int rc = 0;
  if (hipStreamSynchronize(st) != hipSuccess) rc = TC_LAUNCH_EDEVICE;
  for (const TcTimer::Rec& r : g_timer.recs) {
    float t = 0.0f, t2 = 0.0f;
    if (rc == 0 && hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) rc = TC_LAUNCH_EDEVICE;
    if (rc == 0 && r.b2 != nullptr && hipEventElapsedTime(&t2, r.a, r.b2) != hipSuccess) rc = TC_LAUNCH_EDEVICE;
    ms[r.kind] += t2 > t ? t2 : t;
    cnt[r.kind] += 1;
  }
  g_timer.recs.clear();
  g_timer.used = 0;
  return rc;
}

// A second stream and two events per host thread and device for the
// lookahead schedule (default priority; created on first use and kept).
namespace {
struct TcSide {
  int dev = -1;
  hipStream_t st = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
};
thread_local TcSide g_side[8];
TcSide* tc_side() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 8) return nullptr;
  TcSide& S = g_side[dev];
  if (S.st == nullptr) {
    if (hipStreamCreateWithFlags(&S.st, hipStreamNonBlocking) != hipSuccess) return nullptr;
    for (int k = 0; k < 2; ++k)
      if (hipEventCreateWithFlags(&S.ev[k], hipEventDisableTiming) != hipSuccess) return nullptr;
    S.dev = dev;
  }
  return &S;
}
}  // namespace

static hipStream_t tc_side_stream() {
  TcSide* S = tc_side();
  return S ? S->st : nullptr;
}
static hipEvent_t tc_side_event(int k) {
  TcSide* S = tc_side();
  return S ? S->ev[k] : nullptr;
}

// ------------------------------------------------- tile DAG as a HIP graph
// The fork-join launches become the nodes of one HIP graph whose edges are
// the dependencies between them, with the trailing update of step J split
// into one node per tile column K > J (units colsum(J, K-J-1) ..
// + colsize(K) of the step's column-major order):
//   - TRSM(J, s) and PANEL(J, s) form step J's chain, in sub-column order;
//   - step J+1's chain starts after the column-(J+1) update of step J, which
//     carries POTRF(J+1, 0);
//   - the column-K update of step J waits for step J's chain and for the
//     column-K update of step J-1.
// The HIP runtime starts a node when its predecessors have finished, so the
// updates of later columns overlap the following chains as far as the
// dependencies allow: a lookahead of any depth, managed by the runtime
// instead of a ticket order or stream events.  Every block still receives
// its updates in step order from the same bodies, so the factor is
// bit-identical to fork-join.  Instantiated graphs are cached per (matrix,
// workspace, geometry).
namespace {
struct TcGraphKey {
  const void* A;
  int64_t lda, n, T;
  const void* work;
  int noop, dev;
  bool operator<(const TcGraphKey& o) const {
    return std::tie(A, lda, n, T, work, noop, dev) < std::tie(o.A, o.lda, o.n, o.T, o.work, o.noop, o.dev);
  }
};
std::mutex g_graph_mu;
std::map<TcGraphKey, hipGraphExec_t> g_graphs;
std::deque<TcGraphKey> g_graph_order;  // insertion order, for eviction
constexpr size_t TC_GRAPH_CACHE = 16;
}  // namespace

static int tc_graph_node(hipGraph_t gr, hipGraphNode_t* out, const hipGraphNode_t* deps, size_t ndeps,
                         const void* fn, unsigned grid, void** args) {
  hipKernelNodeParams p{};
  p.func = (void*)fn;
  p.gridDim = dim3(grid);
  p.blockDim = dim3(TC_THREADS);
  p.sharedMemBytes = 0;
  p.kernelParams = args;  // the node copies the argument values
  p.extra = nullptr;
  return hipGraphAddKernelNode(out, gr, deps, ndeps, &p) == hipSuccess ? 0 : TC_LAUNCH_EDEVICE;
}

static int tc_build_factor_graph(double* A, int64_t lda, const TcGeom& g, const TcWs& ws, hipGraphExec_t* exec) {
  hipGraph_t gr = nullptr;
  if (hipGraphCreate(&gr, 0) != hipSuccess) return TC_LAUNCH_EDEVICE;
  TcGeom gv = g;
  TcWs wv = ws;
  int rc = 0;
  hipGraphNode_t prev = nullptr;
  {
    int32_t J = 0, sc = 0;
    void* args[] = {&A, &lda, &gv, &J, &sc, &wv};
    rc = tc_graph_node(gr, &prev, nullptr, 0, (const void*)tc_fj_potrf, 1, args);
  }
  std::vector<hipGraphNode_t> colprev(g.M, nullptr);  // latest update node of each tile column
  for (int32_t J = 0; J < g.M && rc == 0; ++J) {
    if (J > 0) prev = colprev[J];
    for (int32_t sc = 0; sc < tc_sb(g, J) && rc == 0; ++sc) {
      int32_t Jv = J, sv = sc;
      void* args[] = {&A, &lda, &gv, &Jv, &sv, &wv};
      const int64_t nt = tc_trsm_count(g, J, sc);
      if (nt > 0) {
        hipGraphNode_t nd = nullptr;
        rc = tc_graph_node(gr, &nd, &prev, 1, (const void*)tc_fj_trsm, (unsigned)(2 * nt), args);
        prev = nd;
      }
      const int64_t np = tc_panel_count(g, J, sc);
      if (np > 0 && rc == 0) {
        hipGraphNode_t nd = nullptr;
        rc = tc_graph_node(gr, &nd, &prev, 1, (const void*)tc_fj_panel, (unsigned)np, args);
        prev = nd;
      }
    }
    const hipGraphNode_t chain = prev;
    for (int32_t K = J + 1; K < g.M && rc == 0; ++K) {
      int32_t Jv = J;
      int64_t first = tc_colsum(g, J, K - J - 1);
      void* args[] = {&A, &lda, &gv, &Jv, &wv, &first};
      const hipGraphNode_t deps[2] = {chain, colprev[K]};
      hipGraphNode_t nd = nullptr;
      rc = tc_graph_node(gr, &nd, deps, colprev[K] ? 2 : 1, (const void*)tc_fj_update_range,
                         (unsigned)tc_colsize(g, K), args);
      colprev[K] = nd;
    }
  }
  if (rc == 0 && hipGraphInstantiate(exec, gr, nullptr, nullptr, 0) != hipSuccess) rc = TC_LAUNCH_EDEVICE;
  (void)hipGraphDestroy(gr);
  return rc;
}

static int tc_launch_factor_graph(double* A, int64_t n, int64_t lda, int64_t T, const TcGeom& g, const TcWs& ws,
                                  void* work, hipStream_t st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TC_LAUNCH_EDEVICE;
  const TcGraphKey key{A, lda, n, T, work, ws.noop, dev};
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto it = g_graphs.find(key);
  if (it == g_graphs.end()) {
    hipGraphExec_t ex = nullptr;
    if (int e = tc_build_factor_graph(A, lda, g, ws, &ex)) return e;
    if (g_graphs.size() >= TC_GRAPH_CACHE) {
      // the oldest graph may still be running on some stream: wait for the
      // device before releasing it (rare: only when the cache is full)
      if (hipDeviceSynchronize() != hipSuccess) return TC_LAUNCH_EDEVICE;
      const TcGraphKey old = g_graph_order.front();
      g_graph_order.pop_front();
      (void)hipGraphExecDestroy(g_graphs[old]);
      g_graphs.erase(old);
    }
    it = g_graphs.emplace(key, ex).first;
    g_graph_order.push_back(key);
  }
  if (hipGraphLaunch(it->second, st) != hipSuccess) return TC_LAUNCH_EDEVICE;
  return tc_chk(hipGetLastError());
}

static int64_t tc_pool_grid_size();

// Fork-join with a one-step lookahead on two streams, after POTRF(0, 0):
// stream A (the caller's) runs the panel chain and, for step J, the update
// of column J+1 only; stream B runs the update of the columns beyond J+1,
// which overlaps the panel chain of step J+1.  Each block still receives its
// updates in step order: the column-(J+1) update of step J waits for the
// bulk of step J-1, and the bulk of step J for A's panel J and column J+1
// (which ran after the bulk of step J-1).
// The bulk runs as a pool on a per-step unit counter: on B with `reserve`
// workgroup slots left free for A's panel chain, then on A behind the next
// step's chain, into the slots the chain frees.  Unit bodies and per-block
// update order are the fork-join ones, so the factor is bit-identical to
// every other schedule.
// before(J) runs on A once panel J is final, ahead of step J's updates
// (false: a launch failed); range(J, count) launches the column-(J+1)
// units [0, count) with the fused POTRF(J+1, 0); pool(J, stream, grid,
// first, count, ctr) launches a pool over units [first, first + count).
// The per-step unit counters live in the phase-offset words (zeroed by the
// caller; used by the persistent schedule only).
template <class Before, class Range, class Pool>
static int tc_lookahead_steps(double* A, int64_t lda, const TcGeom& g, TcWs ws, hipStream_t st, Before before,
                              Range range, Pool pool) {
  hipStream_t sb = tc_side_stream();
  hipEvent_t ea = tc_side_event(0), eb = tc_side_event(1);
  if (sb == nullptr || ea == nullptr || eb == nullptr) return TC_LAUNCH_EDEVICE;
  const int64_t cap = tc_pool_grid_size();
  if (cap <= 0) return TC_LAUNCH_EDEVICE;
  // slots left to the chain: 3/16 of the chip, measured best among 1/16 ..
  // 6/16 at n=32768, T=1024 (205.6 .. 204.4 .. 206.4 ms)
  const int64_t reserve = cap * 3 / 16 > 0 ? cap * 3 / 16 : 1;
  unsigned long long* cnt = (unsigned long long*)ws.offs;
  bool b_used = false;
  int32_t tail = -1;  // the step whose bulk still needs its second launch on A
  int64_t tail_first = 0, tail_count = 0;
  int tail_rec = -1;  // its timing record, ended by the tail too
  auto launch_tail = [&]() {
    if (tail < 0) return;
    pool(tail, st, reserve, tail_first, tail_count, cnt + tail);
    tc_timed_extend(tail_rec, st);
    tail = -1;
  };
  for (int32_t J = 0; J < g.M; ++J) {
    for (int32_t sc = 0; sc < tc_sb(g, J); ++sc) {
      const int64_t nt = tc_trsm_count(g, J, sc);
      if (nt > 0)
        tc_timed(TC_UNIT_TRSM, st, [&] {
          hipLaunchKernelGGL(tc_fj_trsm, dim3((unsigned)(2 * nt)), dim3(TC_THREADS), 0, st, A, lda, g, J, sc, ws);
        });
      const int64_t np = tc_panel_count(g, J, sc);
      if (np > 0)
        tc_timed(TC_UNIT_PANEL, st, [&] {
          hipLaunchKernelGGL(tc_fj_panel, dim3((unsigned)np), dim3(TC_THREADS), 0, st, A, lda, g, J, sc, ws);
        });
    }
    launch_tail();  // step J-1's bulk, into the slots panel J leaves
    const int64_t nu = tc_trailing_units(g, J);
    if (nu <= 0) continue;
    if (!before(J)) return TC_LAUNCH_EDEVICE;
    const int64_t ncol = tc_colsize(g, J + 1);  // units of tile column J+1 at step J
    if (b_used && hipStreamWaitEvent(st, eb, 0) != hipSuccess) return TC_LAUNCH_EDEVICE;  // B's bulk J-1
    // column J+1 first, on the whole chip: the chain of step J+1 waits
    // for it, while the bulk waits only for its own inputs
    tc_timed(TC_UNIT_UPDATE, st, [&] { range(J, ncol); });
    if (hipEventRecord(ea, st) != hipSuccess) return TC_LAUNCH_EDEVICE;  // panel J, bulk J-1, column J+1
    if (nu > ncol) {
      if (hipStreamWaitEvent(sb, ea, 0) != hipSuccess) return TC_LAUNCH_EDEVICE;
      tc_timed(TC_TIMING_REST, sb, [&] { pool(J, sb, cap - reserve, ncol, nu - ncol, cnt + J); });
      tail_rec = tc_timed_last(TC_TIMING_REST);
      if (hipEventRecord(eb, sb) != hipSuccess) return TC_LAUNCH_EDEVICE;
      b_used = true;
      tail = J;
      tail_first = ncol;
      tail_count = nu - ncol;
    }
  }
  launch_tail();
  // the caller's stream covers all of it
  if (b_used && hipStreamWaitEvent(st, eb, 0) != hipSuccess) return TC_LAUNCH_EDEVICE;
  return tc_chk(hipGetLastError());
}


int tc_launch_factor(double* A, int64_t n, int64_t lda, int64_t T, int sched_flags, void* work, hipStream_t st,
                     int64_t grid, int64_t wait_ticks, int64_t chunk) {
  const int sched = sched_flags & 0xff;
  TcGeom g = tc_geom(n, T, chunk);
  TcWs ws = tc_ws_map(work, g);
  ws.noop = (sched_flags & TC_SCHED_NOOP) ? 1 : 0;
  // clear header and counters with a fill kernel (graph-capture friendly)
  const int64_t words = (tc_ws_bytes(n, T)) / 4;
  hipLaunchKernelGGL(tc_fill_zero, dim3(256), dim3(256), 0, st, (int32_t*)work, words);
  if (int e = tc_chk(hipGetLastError())) return e;
  if (sched == 2) {
    // naive fork-join: a launch per POTRF, per TRSM column and per panel
    // update of each sub-column, then the row-parallel trailing update
    for (int32_t J = 0; J < g.M; ++J) {
      for (int32_t sc = 0; sc < tc_sb(g, J); ++sc) {
        tc_timed(TC_UNIT_POTRF, st, [&] {
          hipLaunchKernelGGL(tc_fj_potrf, dim3(1), dim3(TC_THREADS), 0, st, A, lda, g, J, sc, ws);
        });
        const int64_t nt = tc_trsm_count(g, J, sc);
        if (nt > 0)
          tc_timed(TC_UNIT_TRSM, st, [&] {
            hipLaunchKernelGGL(tc_fj_trsm, dim3((unsigned)(2 * nt)), dim3(TC_THREADS), 0, st, A, lda, g, J, sc, ws);
          });
        const int64_t np = tc_panel_count(g, J, sc);
        if (np > 0)
          tc_timed(TC_UNIT_PANEL, st, [&] {
            hipLaunchKernelGGL(tc_fj_panel_only, dim3((unsigned)np), dim3(TC_THREADS), 0, st, A, lda, g, J, sc, ws);
          });
      }
      if (J + 1 < g.M)
        tc_timed(TC_UNIT_UPDATE, st, [&] {
          hipLaunchKernelGGL(tc_fj_update_naive, dim3((unsigned)(g.M - 1 - J)), dim3(TC_THREADS), 0, st, A, lda, g, J,
                             ws);
        });
    }
    return tc_chk(hipGetLastError());
  }
  if (sched == 3) {
    tc_timed(TC_TIMING_PERSISTENT, st, [&] {
      hipLaunchKernelGGL(tc_sync, dim3((unsigned)grid), dim3(TC_THREADS), 0, st, A, lda, g, ws, wait_ticks);
    });
    return tc_chk(hipGetLastError());
  }
  if (sched == 4) {
    hipLaunchKernelGGL(tc_fill_zero, dim3(1), dim3(256), 0, st, (int32_t*)ws.offs, (int64_t)(2 * (g.M + 1)));
    tc_timed(TC_UNIT_POTRF, st, [&] {
      hipLaunchKernelGGL(tc_fj_potrf, dim3(1), dim3(TC_THREADS), 0, st, A, lda, g, 0, 0, ws);
    });
    return tc_lookahead_steps(
        A, lda, g, ws, st, [](int32_t) { return true; },
        [&](int32_t J, int64_t count) {
          hipLaunchKernelGGL(tc_fj_update_range, dim3((unsigned)count), dim3(TC_THREADS), 0, st, A, lda, g, J, ws,
                             (int64_t)0);
        },
        [&](int32_t J, hipStream_t s, int64_t grid, int64_t first, int64_t count, unsigned long long* ctr) {
          hipLaunchKernelGGL(tc_fj_update_pool, dim3((unsigned)grid), dim3(TC_THREADS), 0, s, A, lda, g, J, ws, first,
                             count, ctr);
        });
  }
  if (sched == 5) return tc_launch_factor_graph(A, n, lda, T, g, ws, work, st);
  if (sched == 0) {
    // POTRF(0, 0) is the only POTRF with a launch of its own; every other one
    // rides at the head of the launch that finishes its input (see above)
    tc_timed(TC_UNIT_POTRF, st, [&] {
      hipLaunchKernelGGL(tc_fj_potrf, dim3(1), dim3(TC_THREADS), 0, st, A, lda, g, 0, 0, ws);
    });
    for (int32_t J = 0; J < g.M; ++J) {
      for (int32_t sc = 0; sc < tc_sb(g, J); ++sc) {
        const int64_t nt = tc_trsm_count(g, J, sc);
        if (nt > 0)
          tc_timed(TC_UNIT_TRSM, st, [&] {
            hipLaunchKernelGGL(tc_fj_trsm, dim3((unsigned)(2 * nt)), dim3(TC_THREADS), 0, st, A, lda, g, J, sc, ws);
          });
        const int64_t np = tc_panel_count(g, J, sc);
        if (np > 0)
          tc_timed(TC_UNIT_PANEL, st, [&] {
            hipLaunchKernelGGL(tc_fj_panel, dim3((unsigned)np), dim3(TC_THREADS), 0, st, A, lda, g, J, sc, ws);
          });
      }
      const int64_t nu = tc_trailing_units(g, J);
      if (nu > 0)
        tc_timed(TC_UNIT_UPDATE, st, [&] {
          hipLaunchKernelGGL(tc_fj_update, dim3((unsigned)nu), dim3(TC_THREADS), 0, st, A, lda, g, J, ws);
        });
    }
    return tc_chk(hipGetLastError());
  }
  if (g.M > TC_MAX_PHASES) return TC_LAUNCH_EINVAL;
  {
    int64_t tickets = 0;
    for (int32_t P = 0; P < g.M; ++P) tickets += tc_phase_size(g, P);
    if (tickets > INT32_MAX) return TC_LAUNCH_EINVAL;
  }
  hipLaunchKernelGGL(tc_phase_offsets, dim3(1), dim3(64), 0, st, g, ws.offs);
  tc_timed(TC_TIMING_PERSISTENT, st, [&] {
    hipLaunchKernelGGL(tc_async, dim3((unsigned)grid), dim3(TC_THREADS), 0, st, A, lda, g, ws, wait_ticks);
  });
  return tc_chk(hipGetLastError());
}

// Mixed-precision workspace: the fork-join workspace, then d (n doubles),
// then the panel copy P (n rows of tc_lp_ld(T) elements).
int64_t tc_lp_ld(int64_t T) { return (T + 63) & ~(int64_t)63; }
static int64_t tc_lp_elem(int prec) { return prec == TC_PREC_FP32 ? 4 : prec == TC_PREC_BF16 ? 2 : 0; }

// the fork-join workspace, the diagonal scale factors, then two rounded
// panel copies (the lookahead schedule rounds panel J+1 while the bulk of
// step J still reads panel J)
int64_t tc_ws_mixed_bytes(int64_t n, int64_t T, int prec) {
  return tc_ws_bytes(n, T) + tc_round256(8 * n) + 2 * tc_round256(n * tc_lp_ld(T) * tc_lp_elem(prec));
}

// The low-precision factorization with the lookahead schedule: panel J is
// rounded into copy J mod 2, which the column-(J+1) launch and the bulk of
// step J read.
template <int PREC>
static int tc_lp_lookahead(double* A, int64_t lda, const TcGeom& g, TcWs ws, void* P0, void* P1, int64_t ldp,
                           hipStream_t st) {
  typedef typename TcLp<PREC>::elem E;
  auto pj = [&](int32_t J) { return (E*)((J & 1) ? P1 : P0); };
  return tc_lookahead_steps(
      A, lda, g, ws, st,
      [&](int32_t J) {
        const int64_t rows = g.n - (int64_t)(J + 1) * g.T;
        hipLaunchKernelGGL(tc_round_panel<PREC>, dim3((unsigned)((rows + 15) / 16)), dim3(TC_THREADS), 0, st, A, lda,
                           g, J, pj(J), ldp, ws);
        return true;
      },
      [&](int32_t J, int64_t count) {
        hipLaunchKernelGGL(tc_fj_update_lp_range<PREC>, dim3((unsigned)count), dim3(TC_THREADS), 0, st, A, lda, g, J,
                           ws, (const E*)pj(J), ldp, (int64_t)0);
      },
      [&](int32_t J, hipStream_t s, int64_t grid, int64_t first, int64_t count, unsigned long long* ctr) {
        hipLaunchKernelGGL(tc_fj_update_lp_pool<PREC>, dim3((unsigned)grid), dim3(TC_THREADS), 0, s, A, lda, g, J, ws,
                           (const E*)pj(J), ldp, first, count, ctr);
      });
}

int tc_launch_factor_mixed(double* A, int64_t n, int64_t lda, int64_t T, int prec, int scale, double shift,
                           void* work, hipStream_t st) {
  TcGeom g = tc_geom(n, T, 0);
  TcWs ws = tc_ws_map(work, g);
  char* tail = (char*)work + tc_ws_bytes(n, T);
  double* d = (double*)tail;
  void* P = tail + tc_round256(8 * n);
  const int64_t ldp = tc_lp_ld(T);
  hipLaunchKernelGGL(tc_fill_zero, dim3(256), dim3(256), 0, st, (int32_t*)work, tc_ws_bytes(n, T) / 4);
  if (scale) hipLaunchKernelGGL(tc_diag_scale, dim3(1), dim3(TC_THREADS), 0, st, A, lda, n, d, ws.hdr);
  if (scale || shift != 0.0)
    hipLaunchKernelGGL(tc_scale_lower, dim3((unsigned)n), dim3(TC_THREADS), 0, st, A, lda, n,
                       scale ? (const double*)d : nullptr, shift, ws.hdr);
  tc_timed(TC_UNIT_POTRF, st, [&] {
    hipLaunchKernelGGL(tc_fj_potrf, dim3(1), dim3(TC_THREADS), 0, st, A, lda, g, 0, 0, ws);
  });
  if (prec == TC_PREC_FP32 || prec == TC_PREC_BF16) {
    // the unit counters of the lookahead pool are zero: the whole
    // fork-join workspace was cleared above
    void* P1 = (char*)P + tc_round256(n * ldp * tc_lp_elem(prec));
    const int r = prec == TC_PREC_FP32 ? tc_lp_lookahead<TC_PREC_FP32>(A, lda, g, ws, P, P1, ldp, st)
                                       : tc_lp_lookahead<TC_PREC_BF16>(A, lda, g, ws, P, P1, ldp, st);
    if (r != 0) return r;
    if (scale)
      hipLaunchKernelGGL(tc_unscale_lower, dim3((unsigned)n), dim3(TC_THREADS), 0, st, A, lda, n, d, ws.hdr);
    return tc_chk(hipGetLastError());
  }
  for (int32_t J = 0; J < g.M; ++J) {
    for (int32_t sc = 0; sc < tc_sb(g, J); ++sc) {
      const int64_t nt = tc_trsm_count(g, J, sc);
      if (nt > 0)
        tc_timed(TC_UNIT_TRSM, st, [&] {
          hipLaunchKernelGGL(tc_fj_trsm, dim3((unsigned)(2 * nt)), dim3(TC_THREADS), 0, st, A, lda, g, J, sc, ws);
        });
      const int64_t np = tc_panel_count(g, J, sc);
      if (np > 0)
        tc_timed(TC_UNIT_PANEL, st, [&] {
          hipLaunchKernelGGL(tc_fj_panel, dim3((unsigned)np), dim3(TC_THREADS), 0, st, A, lda, g, J, sc, ws);
        });
    }
    if (tc_trailing_units(g, J) <= 0) continue;
    {
      const int64_t nu = tc_trailing_units(g, J);
      tc_timed(TC_UNIT_UPDATE, st, [&] {
        hipLaunchKernelGGL(tc_fj_update, dim3((unsigned)nu), dim3(TC_THREADS), 0, st, A, lda, g, J, ws);
      });
    }
  }
  if (scale) hipLaunchKernelGGL(tc_unscale_lower, dim3((unsigned)n), dim3(TC_THREADS), 0, st, A, lda, n, d, ws.hdr);
  return tc_chk(hipGetLastError());
}

// ---- pinned staging for host-to-device copies of launch metadata: one
// buffer per host thread, grown on demand; before it is rewritten, the event
// recorded after its last copies is waited for.
namespace {
struct TcStaging {
  char* buf = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};
thread_local TcStaging g_staging;
}  // namespace

static char* tc_staging_acquire(size_t bytes) {
  TcStaging& S = g_staging;
  if (S.ev == nullptr && hipEventCreateWithFlags(&S.ev, hipEventDisableTiming) != hipSuccess) return nullptr;
  if (S.pending) {
    if (hipEventSynchronize(S.ev) != hipSuccess) return nullptr;
    S.pending = false;
  }
  if (bytes > S.cap) {
    if (S.buf) (void)hipHostFree(S.buf);
    S.buf = nullptr;
    S.cap = 0;
    size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes * 2;
    void* p = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) return nullptr;
    S.buf = (char*)p;
    S.cap = want;
  }
  return S.buf;
}

static int tc_staging_release(hipStream_t st) {
  if (hipEventRecord(g_staging.ev, st) != hipSuccess) return TC_LAUNCH_EDEVICE;
  g_staging.pending = true;
  return 0;
}

// ---- batched launcher (workspace layout and ticket order: batch_plan.h)
int64_t tc_batched_ws_bytes(int64_t batch, const int64_t* n, const int64_t* T, int solve, int64_t chunk,
                            const int32_t* prec, bool refine) {
  return tc_batch_layout(batch, n, T, solve != 0, chunk, nullptr, prec, refine).total_bytes;
}

// Copies of the refined batched launch: the lower triangle of A0 into the
// factor's storage A, and b0 into x (one matrix per blockIdx.x, rows strided
// over blockIdx.y).
__global__ __launch_bounds__(TC_THREADS) void tc_batch_copy(const TcBatchMat* __restrict__ mats) {
  const TcBatchMat& d = mats[blockIdx.x];
  const int64_t n = d.g.n;
  if (d.A0 == nullptr || n <= 0) return;
  double* A = tc_global(d.A);
  const double* A0 = tc_global(d.A0);
  double* b = tc_global(d.b);
  const double* b0 = tc_global(d.b0);
  const int64_t lda = d.lda, lda0 = d.lda0;
  for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
    if (A != A0)
      for (int64_t j = threadIdx.x; j <= i; j += TC_THREADS) A[i * lda + j] = A0[i * lda0 + j];
    if (threadIdx.x == 0) b[i] = b0[i];
  }
}

int tc_read_batched_stats(const void* work, int64_t batch, const int64_t* n, const int64_t* T, int64_t chunk,
                          const int32_t* prec, hipStream_t st, double* eta, int64_t* iters) {
  const TcBatchLayout L = tc_batch_layout(batch, n, T, true, chunk, nullptr, prec, true);
  std::vector<double> h(2 * batch);
  if (batch > 0 && hipMemcpyAsync(h.data(), (const char*)work + L.stats, 16 * batch, hipMemcpyDeviceToHost, st) !=
                       hipSuccess)
    return TC_LAUNCH_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return TC_LAUNCH_EDEVICE;
  for (int64_t i = 0; i < batch; ++i) {
    eta[i] = h[2 * i];
    iters[i] = (int64_t)h[2 * i + 1];
  }
  return 0;
}

int tc_launch_batched(double* const* A, double* const* b, const int64_t* n, const int64_t* lda, const int64_t* T,
                      int64_t batch, void* work, hipStream_t st, int64_t grid, int64_t wait_ticks, int64_t chunk,
                      const int64_t* nrhs, const int64_t* ldb, const TcBatchMixed* mx) {
  const bool solve = b != nullptr;
  const int32_t* prec = mx ? mx->prec : nullptr;
  const bool refine = solve && mx && mx->A0;
  std::vector<TcGeom> geoms(batch);
  const TcBatchLayout L = tc_batch_layout(batch, n, T, solve, chunk, &geoms, prec, refine);
  char* base = (char*)work;
  // descriptors
  std::vector<TcBatchMat> mats(batch);
  int64_t ctr = L.counters, extra = L.extra;
  int64_t nmax = 0;
  for (int64_t i = 0; i < batch; ++i) {
    TcBatchMat& d = mats[i];
    d = TcBatchMat{};
    d.ws.hdr = (TcWsHeader*)(base + L.hdrs) + i;
    d.done = (int32_t*)(base + L.done) + i;
    if (n[i] <= 0) continue;
    const TcGeom& g = geoms[i];
    d.A = A[i];
    d.b = solve ? b[i] : nullptr;
    d.lda = lda[i];
    d.nrhs = solve ? (nrhs ? nrhs[i] : 1) : 0;
    d.ldb = solve ? (ldb ? ldb[i] : 1) : 1;
    d.g = g;
    d.ws.offs = nullptr;
    d.ws.pdone = (int32_t*)(base + ctr);
    d.ws.ver = (int32_t*)(base + ctr + tc_round256(4 * (int64_t)g.NRB));
    d.ws.noop = 0;
    ctr += tc_ctr_bytes(g);
    d.prec = prec ? prec[i] : TC_PREC_FP64;
    if (d.prec == TC_PREC_FP32 && g.M > 1) {
      d.P = (float*)(base + extra);
      d.ldp = tc_batch_ldp(g.n);
      extra += tc_round256(4 * g.n * d.ldp);
    }
    if (refine) {
      d.refine = 1;
      d.A0 = mx->A0[i];
      d.lda0 = mx->lda0[i];
      d.b0 = mx->b0[i];
      d.R = (double*)(base + extra);
      extra += tc_round256(8 * g.n);
      d.stat = (double*)(base + L.stats) + 2 * i;
      d.tol = mx->tol;
      d.max_iter = mx->max_iter;
      nmax = std::max(nmax, g.n);
    }
    int64_t nu = 0;
    for (int32_t P = 0; P < g.M; ++P) nu += tc_phase_size(g, P);
    d.nunits = nu;
  }
  std::vector<TcBatchSlot> slots;
  slots.reserve(L.nslots);
  const int64_t start = tc_batch_slots(batch, n, geoms, solve, slots);
  if ((int64_t)slots.size() > L.nslots || start != L.nunits) return TC_LAUNCH_EINVAL;  // (empty segments dropped)
  hipLaunchKernelGGL(tc_fill_zero, dim3(256), dim3(256), 0, st, (int32_t*)work, L.zero_end / 4);
  // descriptors and slots reach the device through pinned staging: the host
  // vectors die when this call returns, while the copies may still wait
  // behind earlier work on the stream
  const size_t mb = sizeof(TcBatchMat) * batch, sb = sizeof(TcBatchSlot) * slots.size();
  char* stg = tc_staging_acquire(mb + sb);
  if (stg == nullptr) return TC_LAUNCH_EDEVICE;
  memcpy(stg, mats.data(), mb);
  if (sb) memcpy(stg + mb, slots.data(), sb);
  if (hipMemcpyAsync(base + L.mats, stg, mb, hipMemcpyHostToDevice, st) != hipSuccess) return TC_LAUNCH_EDEVICE;
  if (sb && hipMemcpyAsync(base + L.slots, stg + mb, sb, hipMemcpyHostToDevice, st) != hipSuccess)
    return TC_LAUNCH_EDEVICE;
  if (tc_staging_release(st) != 0) return TC_LAUNCH_EDEVICE;
  if (slots.empty()) return tc_chk(hipGetLastError());
  if (refine)
    hipLaunchKernelGGL(tc_batch_copy, dim3((unsigned)batch, (unsigned)std::min<int64_t>(nmax, 16)), dim3(TC_THREADS),
                       0, st, (const TcBatchMat*)(base + L.mats));
  hipLaunchKernelGGL(tc_batch_units, dim3((unsigned)slots.size()), dim3(TC_THREADS), 0, st,
                     (const TcBatchMat*)(base + L.mats), (const TcBatchSlot*)(base + L.slots),
                     (TcBatchUnit*)(base + L.table));
  tc_timed(TC_TIMING_PERSISTENT, st, [&] {
    hipLaunchKernelGGL(tc_batched, dim3((unsigned)grid), dim3(TC_THREADS), 0, st,
                       (const TcBatchMat*)(base + L.mats), (const TcBatchUnit*)(base + L.table), L.nunits,
                       (int32_t*)base, wait_ticks);
  });
  return tc_chk(hipGetLastError());
}

int tc_read_batched_status(const void* work, int64_t batch, hipStream_t st, int32_t* error, int64_t* info) {
  std::vector<TcWsHeader> h(batch);
  if (batch > 0 && hipMemcpyAsync(h.data(), (const char*)work + 256, sizeof(TcWsHeader) * batch,
                                  hipMemcpyDeviceToHost, st) != hipSuccess)
    return TC_LAUNCH_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return TC_LAUNCH_EDEVICE;
  for (int64_t i = 0; i < batch; ++i) {
    error[i] = h[i].error;
    info[i] = h[i].info;
  }
  return 0;
}

int64_t tc_ws_header_bytes() { return (int64_t)sizeof(TcWsHeader); }

void tc_ws_header_read(const void* hdr, int32_t* error, int64_t* info) {
  TcWsHeader h;
  memcpy(&h, hdr, sizeof(h));
  *error = h.error;
  *info = h.info;
}

int tc_read_status(const void* work, hipStream_t st, int32_t* error, int64_t* info) {
  TcWsHeader h;
  if (hipMemcpyAsync(&h, work, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return TC_LAUNCH_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return TC_LAUNCH_EDEVICE;
  *error = h.error;
  *info = h.info;
  return 0;
}

// Co-resident workgroups of a persistent kernel on the current device
// (occupancy x CUs), cached per device and kernel.
template <typename K>
static int64_t tc_persistent_grid(K kernel, int64_t* cache) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (dev >= 0 && dev < 64 && cache[dev] > 0) return cache[dev];
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, TC_THREADS, 0) != hipSuccess) return -1;
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return -1;
  int64_t gsz = (int64_t)(per_cu > 0 ? per_cu : 1) * p.multiProcessorCount;
  if (dev >= 0 && dev < 64) cache[dev] = gsz;
  return gsz;
}

int64_t tc_async_grid_size() {
  static int64_t cached[64] = {0};
  return tc_persistent_grid(tc_async, cached);
}

int64_t tc_batched_grid_size() {
  static int64_t cached[64] = {0};
  return tc_persistent_grid(tc_batched, cached);
}

int64_t tc_sync_grid_size() {
  static int64_t cached[64] = {0};
  return tc_persistent_grid(tc_sync, cached);
}

// Co-resident workgroups of the bulk-update pool kernel.
static int64_t tc_pool_grid_size() {
  static int64_t cached[64] = {0};
  return tc_persistent_grid(tc_fj_update_pool, cached);
}

// ------------------------------------------ factorization without allocation
// A fixed device-resident workspace for callers that cannot allocate device
// memory (HIP graph capture, tight serving loops): each device holds its own
// copy of this array for the life of the process.  Host code never uses the
// array's name as an address: the address is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.  The factorization clears
// the part it uses with a fill kernel before every run, so a call needs no
// state from the previous one; calls that overlap on one device share the
// array and race.
static __device__ __align__(256) char scratch[TC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {nullptr};
}  // namespace

int64_t tc_scratch_bytes() { return TC_SCRATCH_BYTES; }

void* tc_scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
