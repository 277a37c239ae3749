// solve.hip -- A X = B with the Cholesky factor (the paper's motivating use:
// SPD linear systems through the decomposition): forward substitution
// L Y = B, then backward substitution L^T X = Y.
//
// Both sweeps are single launches over 64-row blocks, one block per
// workgroup.  Each workgroup takes its block from an atomic ticket
// (ascending for the forward sweep, descending for the backward one), so it
// only ever waits for blocks whose tickets are smaller, all held by running
// workgroups.  A finished block's solution reaches the workgroups that need
// it as a payload of device-scope atomic stores (see the hand-off section);
// a workgroup folds every earlier block as its payload arrives, and the
// step on the chain -- the neighbour block's product and the block's own
// solve -- starts the moment the neighbour's payload is complete.  The
// sweep streams L once from HBM while the chain of 64 x 64 triangular
// solves runs.
//
// Every sum runs in a fixed order (stated at each kernel), so results are
// reproducible bit for bit and independent of the timing of the sweep.  The
// in-block substitution scales each row of the diagonal block and the
// right-hand side by the reciprocal of the row's pivot, then runs
// sequentially in the column index with one FMA per entry.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gptr.h"
#include "launch.h"

#define SV_NB 64        // rows per block
// The right-hand sides go through the kernels with lane-level folds
// (sv_forward / sv_backward), one substitution chain per wave: one or two in
// a single pass of payload width 2, three or more in passes of four (payload
// width 4), up to SV_PASSES of them sharing one launch pair with their
// blocks interleaved.  A column's arithmetic does not depend on the pass
// width, so its result is the same bit for bit in either.
#define SV_RC_SMALL 2
#define SV_RC_MID 4
#define SV_PASSES 16
#define SV_THREADS 256

// The call's block tickets, then its status word: `error` is set when a
// dependency wait ran out, cleared only when a call (or a caller that groups
// several solves under one status) starts, so that the ticket reset before
// each launch pair of a many-column solve keeps it.
struct SvWs {
  int32_t ticket_f, ticket_b, reserved[2];
  int32_t error, pad[59];
};
#define SV_COUNTER_WORDS 4

__device__ __forceinline__ int32_t sv_ld(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t sv_uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Broadcast lane l's value of v to the whole wave (l wave-uniform).
__device__ __forceinline__ double sv_readlane(double v, int l) {
  const int64_t b = __builtin_bit_cast(int64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(uint64_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)((uint64_t)b >> 32), l);
  return __builtin_bit_cast(double, (int64_t)(((uint64_t)hi << 32) | lo));
}

// ------------------------------------------------------------ hand-off
// The solved entries of a block reach the workgroups that fold them as data,
// not behind a counter: the owner stores them as relaxed device-scope 64-bit
// atomics into a payload buffer that held a sentinel, and a reader loads
// them the same way until none is the sentinel.  Each entry is written once
// per sweep, so an entry that is not the sentinel is final; no fence is
// needed on either side (with a counter the publisher must write back its
// L2 and the reader invalidate its own).  The sentinel is a signalling NaN,
// which no arithmetic result is; an entry with its bit pattern is stored as
// the default quiet NaN instead.
// Payload layout: block-major, [block][64 rows][PW columns], PW = 2 for the
// one- and two-column sweeps and 16 for the others; rows past n and columns
// past the right-hand sides are stored as zero.
#define SV_SENTINEL 0x7FF4A5A5A5A5A5A5ull
#define SV_QNAN 0x7FF8000000000000ull

__device__ __forceinline__ double sv_pay_ld(const double* p) {
  return __builtin_bit_cast(double,
                            __hip_atomic_load((const uint64_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void sv_pay_st(double* p, double v) {
  uint64_t b = __builtin_bit_cast(uint64_t, v);
  b = b == SV_SENTINEL ? SV_QNAN : b;
  __hip_atomic_store((uint64_t*)p, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool sv_pending(double v) { return __builtin_bit_cast(uint64_t, v) == SV_SENTINEL; }

// Wave-level wait for a payload block: while `pending` (this lane still
// holds a sentinel) is true for some lane, the wave polls one entry of the
// block (`probe`, the same address in every lane) until it is no longer the
// sentinel, then reissues `load` and checks again.  Returns false when the
// status word is set or the wait limit runs out (which sets it).  Every lane
// of the wave takes the same path.
template <class Load, class Pending>
__device__ __forceinline__ bool sv_wave_wait(const double* probe, Load load, Pending pending, SvWs* ws,
                                             int64_t wait_ticks) {
  if (__builtin_amdgcn_ballot_w64(pending()) == 0) return true;
  const uint64_t t0 = wall_clock64();
  for (uint32_t it = 0;; ++it) {
    // the status word and the clock every 16th poll (every waiting wave
    // reads the same status word)
    if ((it & 15) == 0) {
      if (sv_ld(&ws->error)) return false;
      if (wall_clock64() - t0 > (uint64_t)wait_ticks) {
        __hip_atomic_store(&ws->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
    __builtin_amdgcn_s_sleep(1);
    if (sv_pending(sv_pay_ld(probe))) continue;
    load();
    if (__builtin_amdgcn_ballot_w64(pending()) == 0) return true;
  }
}

// Wave-level wait for a whole payload block by reloading it (one round trip
// per check; used for the one block on the chain, which one workgroup at a
// time waits for).  Same contract as sv_wave_wait.
template <class Load, class Pending>
__device__ __forceinline__ bool sv_wave_wait_full(Load load, Pending pending, SvWs* ws, int64_t wait_ticks) {
  if (__builtin_amdgcn_ballot_w64(pending()) == 0) return true;
  const uint64_t t0 = wall_clock64();
  for (uint32_t it = 0;; ++it) {
    if ((it & 15) == 0) {
      if (sv_ld(&ws->error)) return false;
      if (wall_clock64() - t0 > (uint64_t)wait_ticks) {
        __hip_atomic_store(&ws->error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
    load();
    if (__builtin_amdgcn_ballot_w64(pending()) == 0) return true;
  }
}

// Stage the diagonal block strictly lower (zero on and above the diagonal)
// and the reciprocals of its diagonal (every thread of the workgroup takes
// part).  Rows past nr take a unit pivot.  rdiag is written after the
// internal barrier: readers need one more barrier.
__device__ __forceinline__ void sv_stage_diag(const double* __restrict__ L, int64_t lda, int64_t r0, int nr,
                                              double (*Lbb)[SV_NB + 1], double* rdiag) {
  for (int e = threadIdx.x; e < SV_NB * SV_NB; e += SV_THREADS) {
    const int i = e / SV_NB, k = e % SV_NB;
    Lbb[i][k] = (i < nr && k < i) ? L[(r0 + i) * lda + r0 + k] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < SV_NB) {
    const int i = threadIdx.x;
    rdiag[i] = i < nr ? 1.0 / L[(r0 + i) * lda + r0 + i] : 1.0;
  }
}

// ------------------------------------------------- in-block substitution
// NT interleaved substitution chains of one wave against the staged
// diagonal block (strictly lower, with the reciprocals of its diagonal):
// lane k holds row k of each right-hand side.  Each lane scales its kept
// row of the block and its values by the reciprocal of its own pivot once,
// so the chain solves a system with a unit diagonal: step i broadcasts lane
// i's value, which is x_i, and every lane k subtracts (L[k][i] / L[k][k]) x_i
// with one FMA.  The kept row is zero on and past the diagonal, so a lane's
// value stays x_k once its own step has passed.
// Forward runs with L_bb (lane k keeps row k), backward with L_bb^T (lane k
// keeps column k).  This is the reference BLAS triangular solve's scaling by
// reciprocals, done ahead of the chain.
template <int NT>
__device__ __forceinline__ void sv_chains_fwd(double* v, const double (*Lbb)[SV_NB + 1], const double* rdiag,
                                              int lane) {
  const double rl = rdiag[lane];
  double lr[SV_NB];
#pragma unroll
  for (int i = 0; i < SV_NB; ++i) lr[i] = Lbb[lane][i] * rl;
#pragma unroll
  for (int t = 0; t < NT; ++t) v[t] = v[t] * rl;
#pragma unroll
  for (int i = 0; i < SV_NB; ++i) {
#pragma unroll
    for (int t = 0; t < NT; ++t) v[t] = __builtin_fma(-lr[i], sv_readlane(v[t], i), v[t]);
  }
}

template <int NT>
__device__ __forceinline__ void sv_chains_bwd(double* v, const double (*Lbb)[SV_NB + 1], const double* rdiag,
                                              int lane) {
  const double rl = rdiag[lane];
  double lc[SV_NB];
#pragma unroll
  for (int i = 0; i < SV_NB; ++i) lc[i] = Lbb[i][lane] * rl;
#pragma unroll
  for (int t = 0; t < NT; ++t) v[t] = v[t] * rl;
#pragma unroll
  for (int i = SV_NB - 1; i >= 0; --i) {
#pragma unroll
    for (int t = 0; t < NT; ++t) v[t] = __builtin_fma(-lc[i], sv_readlane(v[t], i), v[t]);
  }
}

// ---------------------------------------------------------------- forward
// y_b = L_bb^{-1} (B_b - sum_{j<b} L_bj y_j), one block per workgroup, one
// or two right-hand sides (payload width 2).  The four waves fold the blocks
// j <= b - 2 as their payloads arrive; then wave c (c < nc) takes
// right-hand side c alone: it waits for y_{b-1}, subtracts the fold and
// L_{b,b-1} y_{b-1} (the tile staged in LDS at the start), substitutes, and
// publishes its column, so the chain step involves one wave and no
// workgroup barrier.
// Fold layout: wave w, lane 16 rr + q covers rows 16 s + 4 w + rr (s < 4)
// of the block and columns 16 m + q (m < 4) of every folded block, so each
// load instruction reads four whole 128-byte row segments.  A lane
// accumulates its 4 x 4 products of every block in block order; the 16
// lanes of a row are then summed by a butterfly.
// Rounding order per entry (row i, right-hand side c): the fold as above;
// B minus it; minus L_{b,b-1} y_{b-1} as four partial sums (columns
// k = 4 i + r, ascending) added as (d0 + d1) + (d2 + d3); then the
// substitution (sv_chains_fwd).  The forward sweep does not write
// B: the backward sweep reads y_b from the payload.
// The workgroup with ticket g (counted from the solve's first) of the
// forward sweep; npass passes of RC columns share the launch, their blocks
// interleaved in ticket order: ticket g is block g / npass of pass
// g % npass, and waits only for smaller tickets of its own pass.
template <int RC>
__device__ __forceinline__ void sv_forward_run(const double* __restrict__ L, int64_t lda, int64_t n,
                                               const double* __restrict__ B, int64_t nc, int64_t ldb, double* Ypay,
                                               double* __restrict__ Xpay, SvWs* ws, int64_t wait_ticks, int32_t npass,
                                               int64_t pstride, int32_t g) {
  static_assert(RC >= 1 && RC <= SV_THREADS / 64, "one chain wave per right-hand side");
  __shared__ double part[SV_NB][RC + 1];
  __shared__ double Lbb[SV_NB][SV_NB + 1];
  __shared__ double LsubT[SV_NB][SV_NB + 1];  // L_{b,b-1}, transposed
  __shared__ double ylds[RC][SV_NB];          // y_{b-1}, broadcast to the chain wave's lanes
  __shared__ double rdiag[SV_NB];
  const int tid = threadIdx.x;
  const int32_t b = g / npass, pass = g - b * npass;
  B += pass * RC;
  nc = nc - pass * RC < RC ? nc - pass * RC : RC;
  Ypay += pass * pstride;
  Xpay += pass * pstride;
  const int64_t r0 = (int64_t)b * SV_NB;
  const int nr = n - r0 < SV_NB ? (int)(n - r0) : SV_NB;
  const int w = tid >> 6, lane = tid & 63, rr = lane >> 4, q = lane & 15;
  // the backward sweep's payload of this block starts as the sentinel
  for (int e = tid; e < SV_NB * RC; e += SV_THREADS)
    Xpay[(int64_t)b * SV_NB * RC + e] = __builtin_bit_cast(double, SV_SENTINEL);
  // a payload column with no right-hand side is published as zero at once
  if (w >= nc && w < RC) sv_pay_st(Ypay + ((int64_t)b * SV_NB + lane) * RC + w, 0.0);
  // the chain wave's own entries of B, read before any wait
  const double bown = (w < nc && lane < nr) ? B[(r0 + lane) * ldb + w] : 0.0;
  // staged before any wait: the diagonal block, and L_{b,b-1}
  sv_stage_diag(L, lda, r0, nr, Lbb, rdiag);
  for (int e = tid; e < SV_NB * SV_NB; e += SV_THREADS) {
    const int i = e / SV_NB, k = e % SV_NB;
    LsubT[k][i] = (b > 0 && i < nr) ? L[(r0 + i) * lda + r0 - SV_NB + k] : 0.0;
  }
  int frow[4];
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) frow[s2] = 16 * s2 + 4 * w + rr;
  // A full block reads its rows with plain loads, all in flight together;
  // the ragged last block clamps rows past n to row n - 1 (in bounds) and
  // selects them away after the loads (a block-uniform choice between the
  // two, so no load sits in a branch of its own).
  const bool full = r0 + SV_NB <= n;
  auto lload = [&](int32_t j, double (*dst)[4]) {
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
      const int64_t R = r0 + frow[s2];
      const double* p = L + (full || R < n ? R : n - 1) * lda + q + (int64_t)j * SV_NB;
#pragma unroll
      for (int m = 0; m < 4; ++m) dst[s2][m] = p[16 * m];
    }
    if (!full) {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int m = 0; m < 4; ++m) dst[s2][m] = r0 + frow[s2] < n ? dst[s2][m] : 0.0;
    }
  };
  auto yload = [&](int32_t j, double (*y)[RC]) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < RC; ++c) y[m][c] = sv_pay_ld(Ypay + ((int64_t)j * SV_NB + 16 * m + q) * RC + c);
  };
  const int32_t nfold = b > 1 ? b - 1 : 0;  // blocks 0 .. b - 2
  double acc[4][RC];
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[s2][c] = 0.0;
  // the last folded tile (block b - 2) is read before any wait: its fold
  // runs one step before the chain step
  double lt[4][4], lc[4][4], ya[4][RC];
  bool ok = true;
  if (nfold > 0) {
    lload(nfold - 1, lt);
    yload(0, ya);
  }
  if (nfold > 1) lload(0, lc);
  auto pending = [&] {
    bool p = false;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < RC; ++c) p = p || sv_pending(ya[m][c]);
    return p;
  };
  // the probe: the last row of column 0
  auto probe = [&](int32_t j) { return Ypay + ((int64_t)j * SV_NB + SV_NB - 1) * RC; };
  auto fold = [&](const double (*l)[4]) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (c < nc) {
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) acc[s2][c] += l[s2][m] * ya[m][c];
        }
  };
  for (int32_t j = 0; j < nfold; ++j) {
    if (!sv_wave_wait(probe(j), [&] { yload(j, ya); }, pending, ws, wait_ticks)) {
      ok = false;
      break;
    }
    if (j + 1 == nfold) {
      fold(lt);
      break;
    }
    // the next block, while this one is folded (its tile unless it is the last)
    const bool more = j + 2 < nfold;
    double ln[4][4], yn[4][RC];
    if (more) lload(j + 1, ln);
    yload(j + 1, yn);
    fold(lc);
    if (more) {
#pragma unroll
      for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int m = 0; m < 4; ++m) lc[s2][m] = ln[s2][m];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < RC; ++c) ya[m][c] = yn[m][c];
  }
  // butterfly over the 16 lanes of each row, then one lane writes the sum
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      double v = acc[s2][c];
#pragma unroll
      for (int k = 1; k < 16; k <<= 1) v += __shfl_xor(v, k, 16);
      if (q == 0) part[frow[s2]][c] = v;
    }
  const bool all_ok = __syncthreads_and(ok);
  if (w < nc) {
    // the chain wave goes first in issue on its SIMD (the other workgroup on
    // the CU streams its fold meanwhile)
    __builtin_amdgcn_s_setprio(3);
    const int c = w;
    double v = bown - (lane < nr ? part[lane][c] : 0.0);
    // row `lane` of L_{b,b-1} into registers before the wait
    double lrow[SV_NB];
#pragma unroll
    for (int k = 0; k < SV_NB; ++k) lrow[k] = LsubT[k][lane];
    // keep them in registers here (an empty statement that uses them), so the
    // compiler does not move the LDS reads behind the wait
#pragma unroll
    for (int k = 0; k < SV_NB; ++k) asm volatile("" : "+v"(lrow[k]));
    bool got = all_ok;
    if (got && b > 0) {
      // y_{b-1}, column c: lane k holds entry k
      double yp = sv_pay_ld(Ypay + ((int64_t)(b - 1) * SV_NB + lane) * RC + c);
      got = sv_wave_wait_full([&] { yp = sv_pay_ld(Ypay + ((int64_t)(b - 1) * SV_NB + lane) * RC + c); },
                              [&] { return sv_pending(yp); }, ws, wait_ticks);
      if (got) {
        // L_{b,b-1} y_{b-1}: y_{b-1} through LDS (the wave's LDS operations
        // run in order), four partial sums over k = 4 i + r, then
        // (d0 + d1) + (d2 + d3)
        ylds[c][lane] = yp;
        double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < SV_NB; ++k) d[k & 3] = __builtin_fma(lrow[k], ylds[c][k], d[k & 3]);
        v = v - ((d[0] + d[1]) + (d[2] + d[3]));
      }
    }
    if (lane >= nr) v = 0.0;
    sv_chains_fwd<1>(&v, Lbb, rdiag, lane);
    if (got) sv_pay_st(Ypay + ((int64_t)b * SV_NB + lane) * RC + c, lane < nr ? v : 0.0);
    __builtin_amdgcn_s_setprio(0);
  }
}

// --------------------------------------------------------------- backward
// x_b = L_bb^{-T} (y_b - sum_{j>b} L_jb^T x_j), one block per workgroup:
// the four waves fold the blocks j >= b + 2 as their payloads arrive, then
// wave c takes right-hand side c alone: it waits for x_{b+1}, subtracts the
// fold and L_{b+1,b}^T x_{b+1} (the tile staged in LDS at the start),
// substitutes, writes B and publishes its column.
// Fold layout: thread (r, p) covers output row r of the block (column r of
// each L_jb) and rows 16 p .. 16 p + 15 of every folded block; consecutive
// r are consecutive addresses, so each wave reads 64 contiguous doubles per
// row.  Each quarter p accumulates in block order; the quarters are then
// combined in order p = 0..3.  Then y_b minus it; minus L_{b+1,b}^T x_{b+1}
// as four partial sums (rows k = 4 i + r, ascending) added as
// (d0 + d1) + (d2 + d3); then the substitution (sv_chains_bwd).
// The workgroup with ticket g of the backward sweep (passes interleaved in
// ticket order, as in the forward sweep).
template <int RC>
__device__ __forceinline__ void sv_backward_run(const double* __restrict__ L, int64_t lda, int64_t n,
                                                double* __restrict__ B, int64_t nc, int64_t ldb,
                                                const double* __restrict__ Ypay, double* Xpay, SvWs* ws,
                                                int64_t wait_ticks, int32_t npass, int64_t pstride, int32_t g) {
  static_assert(RC >= 1 && RC <= SV_THREADS / 64, "one chain wave per right-hand side");
  __shared__ double part[4][SV_NB][RC + 1];
  __shared__ double Lbb[SV_NB][SV_NB + 1];
  __shared__ double Lsub[SV_NB][SV_NB + 1];  // L_{b+1,b}
  __shared__ double xlds[RC][SV_NB];         // x_{b+1}, broadcast to the chain wave's lanes
  __shared__ double rdiag[SV_NB];
  const int tid = threadIdx.x;
  const int32_t nb = (int32_t)((n + SV_NB - 1) / SV_NB);
  const int32_t t = g / npass, pass = g - t * npass;
  B += pass * RC;
  nc = nc - pass * RC < RC ? nc - pass * RC : RC;
  Ypay += pass * pstride;
  Xpay += pass * pstride;
  const int32_t b = nb - 1 - t;
  const int64_t r0 = (int64_t)b * SV_NB;
  const int nr = n - r0 < SV_NB ? (int)(n - r0) : SV_NB;
  const int r = tid & 63, p = tid >> 6, w = p, lane = r;
  if (w >= nc && w < RC) sv_pay_st(Xpay + ((int64_t)b * SV_NB + lane) * RC + w, 0.0);
  // the chain wave's own entries of y (published by the forward sweep, an
  // earlier launch)
  const double yown = w < nc ? Ypay[((int64_t)b * SV_NB + lane) * RC + w] : 0.0;
  sv_stage_diag(L, lda, r0, nr, Lbb, rdiag);
  {
    const int64_t j0 = r0 + SV_NB;
    for (int e = tid; e < SV_NB * SV_NB; e += SV_THREADS) {
      const int k = e / SV_NB, i = e % SV_NB;
      Lsub[k][i] = (b + 1 < nb && j0 + k < n && i < nr) ? L[(j0 + k) * lda + r0 + i] : 0.0;
    }
  }
  // Only the blocks b <= nb - 3 fold, and they are full, so the column
  // r0 + r is inside the matrix.  A full block j is read with 16 plain
  // loads in flight together; the ragged last one clamps rows past n to
  // its last row (in bounds) and selects them away (a wave-uniform choice
  // between the two, so no load sits in a branch of its own).
  auto load_col = [&](int32_t j, double* dst) {
    const int64_t j0 = (int64_t)j * SV_NB;
    const double* base = L + r0 + r;
    if (n - j0 >= SV_NB) {
#pragma unroll
      for (int k = 0; k < 16; ++k) dst[k] = base[(j0 + 16 * p + k) * lda];
    } else {
      const int njr = (int)(n - j0);
      double v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int kk = 16 * p + k;
        v[k] = base[(j0 + (kk < njr ? kk : njr - 1)) * lda];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) dst[k] = 16 * p + k < njr ? v[k] : 0.0;
    }
  };
  // this quarter's payload rows of block j, one entry per lane: lane l holds
  // row 16 p + (l & 15), column (l >> 4) % RC (lanes past 16 RC repeat)
  const int xrow = lane & 15, xcol = (lane >> 4) % RC;
  auto xload = [&](int32_t j) { return sv_pay_ld(Xpay + ((int64_t)j * SV_NB + 16 * p + xrow) * RC + xcol); };
  const int32_t jlast = b + 2;  // blocks nb - 1 down to b + 2
  double acc[RC];
#pragma unroll
  for (int c = 0; c < RC; ++c) acc[c] = 0.0;
  // the last folded tile (block b + 2) is read before any wait
  double lt[16], lc[16], xa = 0.0;
  bool ok = true;
  if (jlast < nb) {
    load_col(jlast, lt);
    xa = xload(nb - 1);
  }
  if (jlast < nb - 1) load_col(nb - 1, lc);
  // the probe: the last of this quarter's rows, column 0
  auto probe = [&](int32_t j) { return Xpay + ((int64_t)j * SV_NB + 16 * p + 15) * RC; };
  auto fold = [&](const double* l) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
#pragma unroll
      for (int c = 0; c < RC; ++c)
        if (c < nc) acc[c] += l[k] * sv_readlane(xa, k + 16 * c);
  };
  for (int32_t j = nb - 1; j >= jlast; --j) {
    if (!sv_wave_wait(probe(j), [&] { xa = xload(j); }, [&] { return sv_pending(xa); }, ws, wait_ticks)) {
      ok = false;
      break;
    }
    if (j == jlast) {
      fold(lt);
      break;
    }
    // the next block, while this one is folded (its tile unless it is the last)
    const bool more = j - 1 > jlast;
    double ln[16];
    if (more) load_col(j - 1, ln);
    const double xn = xload(j - 1);
    fold(lc);
    if (more) {
#pragma unroll
      for (int k = 0; k < 16; ++k) lc[k] = ln[k];
    }
    xa = xn;
  }
#pragma unroll
  for (int c = 0; c < RC; ++c) part[p][r][c] = acc[c];
  const bool all_ok = __syncthreads_and(ok);
  if (w < nc) {
    __builtin_amdgcn_s_setprio(3);  // the chain wave first in issue (as in the forward sweep)
    const int c = w;
    const double sm = ((part[0][lane][c] + part[1][lane][c]) + part[2][lane][c]) + part[3][lane][c];
    double v = lane < nr ? yown - sm : 0.0;
    // column `lane` of L_{b+1,b} into registers before the wait
    double lcol[SV_NB];
#pragma unroll
    for (int k = 0; k < SV_NB; ++k) lcol[k] = Lsub[k][lane];
#pragma unroll
    for (int k = 0; k < SV_NB; ++k) asm volatile("" : "+v"(lcol[k]));  // in registers before the wait
    bool got = all_ok;
    if (got && b + 1 < nb) {
      // x_{b+1}, column c: lane k holds entry k
      double xp = sv_pay_ld(Xpay + ((int64_t)(b + 1) * SV_NB + lane) * RC + c);
      got = sv_wave_wait_full([&] { xp = sv_pay_ld(Xpay + ((int64_t)(b + 1) * SV_NB + lane) * RC + c); },
                              [&] { return sv_pending(xp); }, ws, wait_ticks);
      if (got) {
        // L_{b+1,b}^T x_{b+1}: x_{b+1} through LDS, four partial sums over
        // k = 4 i + r, then (d0 + d1) + (d2 + d3)
        xlds[c][lane] = xp;
        double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < SV_NB; ++k) d[k & 3] = __builtin_fma(lcol[k], xlds[c][k], d[k & 3]);
        v = v - ((d[0] + d[1]) + (d[2] + d[3]));
      }
    }
    if (lane >= nr) v = 0.0;
    sv_chains_bwd<1>(&v, Lbb, rdiag, lane);
    if (lane < nr) B[(r0 + lane) * ldb + c] = v;
    if (got) sv_pay_st(Xpay + ((int64_t)b * SV_NB + lane) * RC + c, lane < nr ? v : 0.0);
    __builtin_amdgcn_s_setprio(0);
  }
}

// One solve per launch pair: the ticket from the solve's own counters.
template <int RC>
__global__ __launch_bounds__(SV_THREADS, 2) void sv_forward(const double* __restrict__ L, int64_t lda, int64_t n,
                                                         const double* __restrict__ B, int64_t nc, int64_t ldb,
                                                         double* Ypay, double* __restrict__ Xpay, SvWs* ws,
                                                         int64_t wait_ticks, int32_t npass, int64_t pstride) {
  __shared__ int32_t s_g;
  if (threadIdx.x == 0) s_g = __hip_atomic_fetch_add(&ws->ticket_f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  sv_forward_run<RC>(L, lda, n, B, nc, ldb, Ypay, Xpay, ws, wait_ticks, npass, pstride, sv_uniform(s_g));
}

template <int RC>
__global__ __launch_bounds__(SV_THREADS, 2) void sv_backward(const double* __restrict__ L, int64_t lda, int64_t n,
                                                          double* __restrict__ B, int64_t nc, int64_t ldb,
                                                          const double* __restrict__ Ypay, double* Xpay, SvWs* ws,
                                                          int64_t wait_ticks, int32_t npass, int64_t pstride) {
  __shared__ int32_t s_g;
  if (threadIdx.x == 0) s_g = __hip_atomic_fetch_add(&ws->ticket_b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  sv_backward_run<RC>(L, lda, n, B, nc, ldb, Ypay, Xpay, ws, wait_ticks, npass, pstride, sv_uniform(s_g));
}

// ------------------------------------------------- several solves per launch
// The sweeps of several independent solves (a serving tick's items) in one
// launch pair, all in passes of four: job j owns the tickets [first_j,
// first_{j+1}) of a launch-wide counter, its blocks and passes in the order
// of a launch of its own, so every wait is still on a smaller ticket of the
// same job (taken by a workgroup that has started).  Each job's workspace
// has the single-solve layout: its status word, then its payloads.
__host__ __device__ inline int64_t sv_jr256(int64_t x) { return (x + 255) & ~(int64_t)255; }
__host__ __device__ inline int64_t sv_job_passes(int64_t nrhs) {
  return nrhs > SV_RC_MID ? (nrhs + SV_RC_MID - 1) / SV_RC_MID : 1;
}
__host__ __device__ inline int64_t sv_job_stride(int64_t n) { return ((n + SV_NB - 1) / SV_NB) * SV_NB * SV_RC_MID; }

// This workgroup's job and its ticket within the job (every thread of the
// workgroup takes part; uniform results).
__device__ __forceinline__ void sv_take_job(const TcSolveJob* jobs, int64_t count, int32_t* ctr, int32_t& job,
                                            int32_t& g) {
  __shared__ int32_t s_g, s_j;
  if (threadIdx.x == 0) s_g = __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int64_t t = s_g;
  for (int64_t c0 = 0; c0 < count; c0 += SV_THREADS) {
    const int64_t j = c0 + threadIdx.x;
    if (j < count && jobs[j].first <= t && (j + 1 == count || t < jobs[j + 1].first)) s_j = (int32_t)j;
  }
  __syncthreads();
  job = sv_uniform(s_j);
  g = sv_uniform((int32_t)(t - jobs[job].first));
}

__global__ __launch_bounds__(SV_THREADS, 2) void sv_forward_many(const TcSolveJob* jobs, int64_t count, int32_t* ctr,
                                                              int64_t wait_ticks) {
  int32_t j, g;
  sv_take_job(jobs, count, ctr, j, g);
  const TcSolveJob J = jobs[j];
  const int64_t np = sv_job_passes(J.nrhs), stride = sv_job_stride(J.n);
  // the job's addresses in the global address space (read from memory,
  // they would otherwise be generic and every access a flat one)
  char* work = tc_global((char*)J.work);
  SvWs* ws = (SvWs*)work;
  double* ypay = (double*)(work + sv_jr256(sizeof(SvWs)));
  double* xpay = (double*)((char*)ypay + sv_jr256(8 * stride * np));
  sv_forward_run<SV_RC_MID>(tc_global(J.L), J.lda, J.n, tc_global(J.B), J.nrhs, J.ldb, ypay, xpay, ws, wait_ticks,
                            (int32_t)np, stride, g);
}

__global__ __launch_bounds__(SV_THREADS, 2) void sv_backward_many(const TcSolveJob* jobs, int64_t count, int32_t* ctr,
                                                               int64_t wait_ticks) {
  int32_t j, g;
  sv_take_job(jobs, count, ctr + 1, j, g);
  const TcSolveJob J = jobs[j];
  const int64_t np = sv_job_passes(J.nrhs), stride = sv_job_stride(J.n);
  char* work = tc_global((char*)J.work);  // as in the forward sweep
  SvWs* ws = (SvWs*)work;
  const double* ypay = (const double*)(work + sv_jr256(sizeof(SvWs)));
  double* xpay = (double*)((char*)ypay + sv_jr256(8 * stride * np));
  sv_backward_run<SV_RC_MID>(tc_global(J.L), J.lda, J.n, tc_global(J.B), J.nrhs, J.ldb, ypay, xpay, ws, wait_ticks,
                             (int32_t)np, stride, g);
}

// Jobs blockIdx.y, blockIdx.y + gridDim.y, ...: each one's status struct
// cleared (tickets and status word) and its forward payloads set to the
// sentinel; the launch's two counters cleared by the first workgroup.
__global__ void sv_fill_many(const TcSolveJob* jobs, int64_t njobs, int32_t* ctr) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 2) ctr[threadIdx.x] = 0;
  const double s = __builtin_bit_cast(double, SV_SENTINEL);
  for (int64_t j = blockIdx.y; j < njobs; j += gridDim.y) {
    const TcSolveJob J = jobs[j];
    const int64_t count = sv_job_stride(J.n) * sv_job_passes(J.nrhs);
    char* work = tc_global((char*)J.work);
    double* ypay = (double*)(work + sv_jr256(sizeof(SvWs)));
    if (blockIdx.x == 0 && threadIdx.x < sizeof(SvWs) / 4) ((int32_t*)work)[threadIdx.x] = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
      ypay[i] = s;
  }
}

// ------------------------------------------------ matrix-core operands
// The refinement sweeps below run their products on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64), 16 right-hand sides per pass (payload width 16).
// Operand layout (measured on gfx950): A-operand lane l holds row l % 16 at
// k group l / 16, B-operand lane l holds column l % 16 at k group l / 16,
// output item q of lane l is row 4 q + l / 16, column l % 16.
typedef double sv_v4d __attribute__((ext_vector_type(4)));
#define SV_MF_RC 16

__device__ __forceinline__ sv_v4d sv_mfma(double a, double b, sv_v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------- sweeps with inverted diagonals
// For repeated solves with one factor (refinement), the 64 x 64 diagonal
// blocks are inverted once per call (sv_invert_diag, by substitution
// against the identity), D_b = L_bb^-1, and so are the coupling blocks of
// neighbouring block rows (sv_couple):
//   P_b = -D_b L_{b,b-1}          (forward),
//   Q_b = -D_b^T L_{b+1,b}^T      (backward).
// The forward sweep then takes y_b = c_b + P_b y_{b-1} with
// c_b = D_b (B_b - sum_{j < b-1} L_bj y_j), and the backward sweep
// x_b = d_b + Q_b x_{b+1} with d_b = D_b^T (y_b - sum_{j > b+1} L_jb^T x_j).
// A workgroup computes c_b (or d_b) while it still waits for its neighbour,
// so a block step on the chain is one 64 x 64 by 64 x 16 product per wave
// (each wave its 16 rows), with no workgroup barrier.  The inverses and
// couplings are accurate to about kappa(L_bb) u, which the refinement
// corrects along with the error of the factor itself; the plain solve keeps
// substitution.
//
// Storage (tc_solve_inv_bytes): D, then P, then Q, each 64 x 64 row-major per
// block.  D is zero above the diagonal and the identity on rows past n in
// the last block; P and Q are zero where the factor has no entries (P_0,
// Q_{nb-1}, rows or columns past n).
__global__ __launch_bounds__(SV_THREADS) void sv_invert_diag(const double* __restrict__ L, int64_t lda, int64_t n,
                                                             double* __restrict__ Dinv) {
  __shared__ double Lbb[SV_NB][SV_NB + 1];
  __shared__ double rdiag[SV_NB];
  const int32_t b = blockIdx.x;
  const int64_t r0 = (int64_t)b * SV_NB;
  const int nr = n - r0 < SV_NB ? (int)(n - r0) : SV_NB;
  sv_stage_diag(L, lda, r0, nr, Lbb, rdiag);
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* D = Dinv + (int64_t)b * SV_NB * SV_NB;
  // wave w solves L_bb d = e_c for columns c = w + 4 t, four at a time
  for (int c0 = 0; c0 < 16; c0 += 4) {
    double v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = lane == w + 4 * (c0 + t) ? 1.0 : 0.0;
    sv_chains_fwd<4>(v, Lbb, rdiag, lane);
#pragma unroll
    for (int t = 0; t < 4; ++t) D[(int64_t)lane * SV_NB + w + 4 * (c0 + t)] = v[t];
  }
}

// P_b and Q_b from D (sv_invert_diag's output, an earlier launch) and L.
// One workgroup per block; thread (w, lane) computes entries (row r, column
// lane) for r = w, w + 4, ..., each a 64-term sum in ascending k.
__global__ __launch_bounds__(SV_THREADS) void sv_couple(const double* __restrict__ L, int64_t lda, int64_t n,
                                                        const double* __restrict__ Dinv, double* __restrict__ P,
                                                        double* __restrict__ Q) {
  __shared__ double Db[SV_NB][SV_NB + 1];
  __shared__ double Lc[SV_NB][SV_NB + 1];
  const int32_t b = blockIdx.x;
  const int32_t nb = (int32_t)((n + SV_NB - 1) / SV_NB);
  const int64_t r0 = (int64_t)b * SV_NB;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double* D = Dinv + (int64_t)b * SV_NB * SV_NB;
  for (int e = threadIdx.x; e < SV_NB * SV_NB; e += SV_THREADS) Db[e / SV_NB][e % SV_NB] = D[e];
  // Lc = L_{b,b-1} (rows past n zero)
  for (int e = threadIdx.x; e < SV_NB * SV_NB; e += SV_THREADS) {
    const int i = e / SV_NB, k = e % SV_NB;
    Lc[i][k] = (b > 0 && r0 + i < n) ? L[(r0 + i) * lda + r0 - SV_NB + k] : 0.0;
  }
  __syncthreads();
  double* Pb = P + (int64_t)b * SV_NB * SV_NB;
  for (int r = w; r < SV_NB; r += 4) {
    double acc = 0.0;
    for (int k = 0; k < SV_NB; ++k) acc = fma(Db[r][k], Lc[k][lane], acc);
    Pb[r * SV_NB + lane] = -acc;
  }
  __syncthreads();
  // Lc = L_{b+1,b} (rows past n zero)
  for (int e = threadIdx.x; e < SV_NB * SV_NB; e += SV_THREADS) {
    const int i = e / SV_NB, k = e % SV_NB;
    const int64_t row = r0 + SV_NB + i;
    Lc[i][k] = (b + 1 < nb && row < n) ? L[row * lda + r0 + k] : 0.0;
  }
  __syncthreads();
  // Q_b[r][c] = -sum_k D_b[k][r] L_{b+1,b}[c][k]
  double* Qb = Q + (int64_t)b * SV_NB * SV_NB;
  for (int r = w; r < SV_NB; r += 4) {
    double acc = 0.0;
    for (int k = 0; k < SV_NB; ++k) acc = fma(Db[k][r], Lc[lane][k], acc);
    Qb[r * SV_NB + lane] = -acc;
  }
}

// D_b into LDS (the barrier that follows the fold publishes it).
__device__ __forceinline__ void sv_stage_inv(const double* __restrict__ D, double (*Ds)[SV_NB + 1]) {
  for (int e = threadIdx.x; e < SV_NB * SV_NB; e += SV_THREADS) Ds[e / SV_NB][e % SV_NB] = D[e];
}


// The forward sweep reads its own rows of the right-hand side from B and
// publishes y_b into the payload Ypay (it does not write B); the backward
// sweep reads y_b from Ypay, publishes x_b into Xpay and writes it to B.
// Both payloads have 16 columns.  The forward sweep also resets its block of
// Xpay to the sentinel for the backward sweep (a later launch).
// Fold layout (matrix cores): wave w owns rows 16 w .. 16 w + 15 of the block
// and the 16 payload columns, so it reads whole 512-byte row segments of L;
// in a 16-wide k chunk ch, lane (r, g) brings k = 16 ch + 4 g + m to MFMA m
// for both operands.  Rounding order per output entry: the folded blocks in
// sweep order, each as 16 MFMAs in (chunk, m) order; the subtraction from B;
// the product with D_b; then the product with the coupling block added to
// it.
__global__ __launch_bounds__(SV_THREADS, 2) void sv_fwd_inv(const double* __restrict__ L, int64_t lda, int64_t n,
                                                            const double* __restrict__ Dinv,
                                                            const double* __restrict__ P,
                                                            const double* __restrict__ B, int64_t nc, int64_t ldb,
                                                            double* Ypay, double* __restrict__ Xpay, SvWs* ws,
                                                            int64_t wait_ticks) {
  __shared__ double part[SV_NB][SV_MF_RC + 1];
  __shared__ double yl[SV_NB][SV_MF_RC + 1];  // y_{b-1}, handed over by wave 0
  __shared__ double Ds[SV_NB][SV_NB + 1];
  __shared__ int32_t s_b, s_ok;
  const int tid = threadIdx.x;
  if (tid == 0) s_b = __hip_atomic_fetch_add(&ws->ticket_f, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int32_t b = sv_uniform(s_b);
  const int64_t r0 = (int64_t)b * SV_NB;
  const int nr = n - r0 < SV_NB ? (int)(n - r0) : SV_NB;
  const int w = tid >> 6, lane = tid & 63, r16 = lane & 15, g4 = (lane >> 4) * 4;
  const int arow = 16 * w + r16;
  const bool alive = arow < nr;
  const bool bok = r16 < nc;
  const double* lrow = L + (r0 + (alive ? arow : 0)) * lda + g4;
  // payload column r16, rows 4 g .. of every earlier block (columns past nc
  // are published as zero)
  const double* ypay = Ypay + (int64_t)g4 * SV_MF_RC + r16;
  sv_stage_inv(Dinv + (int64_t)b * SV_NB * SV_NB, Ds);  // D_b, staged before any wait
  for (int e = tid; e < SV_NB * SV_MF_RC; e += SV_THREADS)
    Xpay[(int64_t)b * SV_NB * SV_MF_RC + e] = __builtin_bit_cast(double, SV_SENTINEL);
  auto load_l = [&](int32_t j, double* a) {
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const double v = lrow[(int64_t)j * SV_NB + 16 * ch + m];
        a[4 * ch + m] = alive ? v : 0.0;
      }
  };
  auto load_y = [&](int32_t j, double* y) {
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
#pragma unroll
      for (int m = 0; m < 4; ++m) y[4 * ch + m] = sv_pay_ld(ypay + ((int64_t)j * SV_NB + 16 * ch + m) * SV_MF_RC);
  };
  // read before any wait: the own rows of the right-hand side, the coupling
  // block P_b (row arow), and the last folded tile L_{b,b-2}
  double bown[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = 16 * w + 4 * q + (lane >> 4);
    bown[q] = (row < nr && bok) ? B[(r0 + row) * ldb + r16] : 0.0;
  }
  double pc[16];
  {
    const double* pr = P + (int64_t)b * SV_NB * SV_NB + (int64_t)arow * SV_NB + g4;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
#pragma unroll
      for (int m = 0; m < 4; ++m) pc[4 * ch + m] = pr[16 * ch + m];
  }
  const int32_t nfold = b > 1 ? b - 1 : 0;  // blocks 0 .. b - 2 are folded
  sv_v4d acc = {0.0, 0.0, 0.0, 0.0};
  double lt[16], la[16], ya[16];
  bool ok = true;  // no wait of this wave aborted
  if (nfold > 0) {
    load_l(nfold - 1, lt);
    load_y(0, ya);
  }
  if (nfold > 1) load_l(0, la);
  auto pending = [&] {
    bool p = false;
#pragma unroll
    for (int k = 0; k < 16; ++k) p = p || sv_pending(ya[k]);
    return p;
  };
  // the probe: the block's last entry
  auto probe = [&](int32_t j) { return Ypay + ((int64_t)j * SV_NB + SV_NB - 1) * SV_MF_RC + SV_MF_RC - 1; };
  // the folded blocks but the last, in order; the next block's tile (unless
  // it is the last) and its payload are loaded while this one is folded
  for (int32_t j = 0; j + 1 < nfold; ++j) {
    if (!sv_wave_wait(probe(j), [&] { load_y(j, ya); }, pending, ws, wait_ticks)) {
      ok = false;
      break;
    }
    const int32_t jn = j + 1;
    const bool more = jn + 1 < nfold;
    double ln[16], yn[16];
    if (more) load_l(jn, ln);
    load_y(jn, yn);
#pragma unroll
    for (int k = 0; k < 16; ++k) acc = sv_mfma(la[k], ya[k], acc);
    if (more) {
#pragma unroll
      for (int k = 0; k < 16; ++k) la[k] = ln[k];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) ya[k] = yn[k];
  }
  if (ok && nfold > 0) {
    if (sv_wave_wait(probe(nfold - 1), [&] { load_y(nfold - 1, ya); }, pending, ws, wait_ticks)) {
#pragma unroll
      for (int k = 0; k < 16; ++k) acc = sv_mfma(lt[k], ya[k], acc);
    } else {
      ok = false;
    }
  }
  // the previous block's payload (wave 0), speculatively (checked below)
  if (ok && b > 0 && w == 0) load_y(b - 1, ya);
  // v = B_b - fold, into part (rows past nr and columns past nc are zero)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = 16 * w + 4 * q + (lane >> 4);
    part[row][r16] = (row < nr && bok) ? bown[q] - acc[q] : 0.0;
  }
  __syncthreads();
  // from here on this workgroup's waves are the chain: first in issue on
  // their SIMDs
  __builtin_amdgcn_s_setprio(3);
  // c_b = D_b v: rows 16 w .., right-hand side r16
  sv_v4d y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ch = 0; ch < 4; ++ch)
#pragma unroll
    for (int m = 0; m < 4; ++m) y = sv_mfma(Ds[arow][16 * ch + g4 + m], part[16 * ch + g4 + m][r16], y);
  // the chain: y_b = c_b + P_b y_{b-1}.  Every wave needs the same operand
  // fragments of y_{b-1}; wave 0 alone waits for them and hands them over
  // through LDS, so the waves finish (and publish) together.
  if (b > 0) {
    if (w == 0) {
      bool got = ok && sv_wave_wait_full([&] { load_y(b - 1, ya); }, pending, ws, wait_ticks);
      if (got) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
#pragma unroll
          for (int m = 0; m < 4; ++m) yl[16 * ch + g4 + m][r16] = ya[4 * ch + m];
      }
      if (lane == 0) s_ok = got;
    }
    __syncthreads();
    ok = ok && s_ok;
    if (ok) {
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
#pragma unroll
        for (int m = 0; m < 4; ++m) y = sv_mfma(pc[4 * ch + m], yl[16 * ch + g4 + m][r16], y);
    }
  }
  // the waves publish their rows unless a wait aborted (then the status
  // word is set and every waiter leaves)
  if (ok) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 16 * w + 4 * q + (lane >> 4);
      sv_pay_st(Ypay + ((int64_t)b * SV_NB + row) * SV_MF_RC + r16, (row < nr && bok) ? y[q] : 0.0);
    }
  }
}

// The backward sweep's fold splits k across the waves: wave w takes rows
// 16 w .. 16 w + 15 of every later block j, for all 64 output rows (columns
// r0 .. r0 + 63 of L), so it reads whole 512-byte row segments of L and only
// the 16 payload rows that wave w of block j's workgroup publishes.  MFMA
// (o, kc): output rows 16 o .., k rows 16 w + 4 kc + g; A lane (r, g) holds
// L[j0 + 16 w + 4 kc + g][r0 + 16 o + r], B lane (r, g) holds
// x_j[16 w + 4 kc + g][r].  Rounding order per output entry: each wave sums
// its blocks in sweep order, each as 4 MFMAs in kc order; the waves' sums
// are combined as (w0 + w2) + (w1 + w3); then the subtraction from y_b, the
// product with D_b^T, and the coupling product added to it.
__global__ __launch_bounds__(SV_THREADS, 2) void sv_bwd_inv(const double* __restrict__ L, int64_t lda, int64_t n,
                                                            const double* __restrict__ Dinv,
                                                            const double* __restrict__ Q, double* __restrict__ B,
                                                            int64_t nc, int64_t ldb, const double* __restrict__ Ypay,
                                                            double* Xpay, SvWs* ws, int64_t wait_ticks) {
  __shared__ double red[2][SV_NB][SV_MF_RC + 1];  // partial sums; red[0] then holds v
  __shared__ double xl[SV_NB][SV_MF_RC + 1];      // x_{b+1}, handed over by wave 0
  __shared__ double Ds[SV_NB][SV_NB + 1];
  __shared__ int32_t s_t, s_ok;
  double(*part)[SV_MF_RC + 1] = red[0];
  const int tid = threadIdx.x;
  const int32_t nb = (int32_t)((n + SV_NB - 1) / SV_NB);
  if (tid == 0) s_t = __hip_atomic_fetch_add(&ws->ticket_b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int32_t t = sv_uniform(s_t);
  const int32_t b = nb - 1 - t;
  const int64_t r0 = (int64_t)b * SV_NB;
  const int nr = n - r0 < SV_NB ? (int)(n - r0) : SV_NB;
  const int w = tid >> 6, lane = tid & 63, r16 = lane & 15, g4 = (lane >> 4) * 4, g = lane >> 4;
  const int arow = 16 * w + r16;
  const bool bok = r16 < nc;
  sv_stage_inv(Dinv + (int64_t)b * SV_NB * SV_NB, Ds);
  // tile of block j: a[4 o + kc] (rows past n and columns past n read as zero)
  auto load_l = [&](int32_t j, double* a) {
    const int64_t j0 = (int64_t)j * SV_NB;
    const int njr = n - j0 < SV_NB ? (int)(n - j0) : SV_NB;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int kr = 16 * w + 4 * kc + g;
      const bool kin = kr < njr;
      const double* rowp = L + (j0 + (kin ? kr : 0)) * lda + r0;
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        const int col = 16 * o + r16;
        const bool cin = col < nr;
        const double v = rowp[cin ? col : 0];
        a[4 * o + kc] = (kin && cin) ? v : 0.0;
      }
    }
  };
  // this wave's payload rows of block j: x[kc]
  auto load_xk = [&](int32_t j, double* x) {
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
      x[kc] = sv_pay_ld(Xpay + ((int64_t)j * SV_NB + 16 * w + 4 * kc + g) * SV_MF_RC + r16);
  };
  // the whole payload of block j in the chain product's layout (wave 0)
  auto load_x = [&](int32_t j, double* x) {
    const double* xp = Xpay + (int64_t)g4 * SV_MF_RC + r16;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
#pragma unroll
      for (int m = 0; m < 4; ++m) x[4 * ch + m] = sv_pay_ld(xp + ((int64_t)j * SV_NB + 16 * ch + m) * SV_MF_RC);
  };
  // read before any wait: the own rows of y (published by the forward sweep,
  // an earlier launch), the coupling block Q_b (row arow), and the last
  // folded tile, rows of block b + 2
  double yown[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = 16 * w + 4 * q + g;
    yown[q] = Ypay[((int64_t)b * SV_NB + row) * SV_MF_RC + r16];
  }
  double qc[16];
  {
    const double* qr = Q + (int64_t)b * SV_NB * SV_NB + (int64_t)arow * SV_NB + g4;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
#pragma unroll
      for (int m = 0; m < 4; ++m) qc[4 * ch + m] = qr[16 * ch + m];
  }
  const int32_t jlast = b + 2;  // blocks nb - 1 down to b + 2 are folded
  sv_v4d acc[4];
#pragma unroll
  for (int o = 0; o < 4; ++o) acc[o] = (sv_v4d){0.0, 0.0, 0.0, 0.0};
  double lt[16], la[16], xa[4];
  bool ok = true;
  if (jlast < nb) {
    load_l(jlast, lt);
    load_xk(nb - 1, xa);
  }
  if (jlast < nb - 1) load_l(nb - 1, la);
  auto pending = [&] { return sv_pending(xa[0]) || sv_pending(xa[1]) || sv_pending(xa[2]) || sv_pending(xa[3]); };
  // the probe: the last entry of this wave's payload rows
  auto probe = [&](int32_t j) { return Xpay + ((int64_t)j * SV_NB + 16 * w + 15) * SV_MF_RC + SV_MF_RC - 1; };
  auto fold = [&](const double* a, const double* x) {
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) acc[o] = sv_mfma(a[4 * o + kc], x[kc], acc[o]);
  };
  for (int32_t j = nb - 1; j > jlast; --j) {
    if (!sv_wave_wait(probe(j), [&] { load_xk(j, xa); }, pending, ws, wait_ticks)) {
      ok = false;
      break;
    }
    const int32_t jn = j - 1;
    const bool more = jn > jlast;
    double ln[16], xn[4];
    if (more) load_l(jn, ln);
    load_xk(jn, xn);
    fold(la, xa);
    if (more) {
#pragma unroll
      for (int k = 0; k < 16; ++k) la[k] = ln[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) xa[k] = xn[k];
  }
  if (ok && jlast < nb) {
    if (sv_wave_wait(probe(jlast), [&] { load_xk(jlast, xa); }, pending, ws, wait_ticks))
      fold(lt, xa);
    else
      ok = false;
  }
  double xc[16];  // the chain's operand (wave 0), loaded speculatively
  if (ok && b + 1 < nb && w == 0) load_x(b + 1, xc);
  // combine the waves' sums: red[0] = w0 + w2, red[1] = w1 + w3
  if (w < 2) {
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[w][16 * o + 4 * q + g][r16] = acc[o][q];
  }
  __syncthreads();
  if (w >= 2) {
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[w - 2][16 * o + 4 * q + g][r16] += acc[o][q];
  }
  __syncthreads();
  // v = y_b - fold into part (= red[0]; each entry read and rewritten by the
  // same thread; rows past nr and columns past nc are zero)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = 16 * w + 4 * q + g;
    const double f = red[0][row][r16] + red[1][row][r16];
    part[row][r16] = (row < nr && bok) ? yown[q] - f : 0.0;
  }
  __syncthreads();
  __builtin_amdgcn_s_setprio(3);  // the chain, first in issue
  // d_b = D_b^T v
  sv_v4d x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ch = 0; ch < 4; ++ch)
#pragma unroll
    for (int m = 0; m < 4; ++m) x = sv_mfma(Ds[16 * ch + g4 + m][arow], part[16 * ch + g4 + m][r16], x);
  // the chain: x_b = d_b + Q_b x_{b+1}, x_{b+1} handed over by wave 0
  if (b + 1 < nb) {
    if (w == 0) {
      auto pend16 = [&] {
        bool p = false;
#pragma unroll
        for (int k = 0; k < 16; ++k) p = p || sv_pending(xc[k]);
        return p;
      };
      bool got = ok && sv_wave_wait_full([&] { load_x(b + 1, xc); }, pend16, ws, wait_ticks);
      if (got) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
#pragma unroll
          for (int m = 0; m < 4; ++m) xl[16 * ch + g4 + m][r16] = xc[4 * ch + m];
      }
      if (lane == 0) s_ok = got;
    }
    __syncthreads();
    ok = ok && s_ok;
    if (ok) {
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
#pragma unroll
        for (int m = 0; m < 4; ++m) x = sv_mfma(qc[4 * ch + m], xl[16 * ch + g4 + m][r16], x);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int row = 16 * w + 4 * q + g;
    if (row < nr && bok) B[(r0 + row) * ldb + r16] = x[q];
    if (ok) sv_pay_st(Xpay + ((int64_t)b * SV_NB + row) * SV_MF_RC + r16, (row < nr && bok) ? x[q] : 0.0);
  }
}

// Clear the first `words` words of the workspace header and set `count`
// payload entries to the sentinel.
__global__ void sv_fill(SvWs* ws, int words, double* pay, int64_t count) {
  if (blockIdx.x == 0 && (int)threadIdx.x < words) ((int32_t*)ws)[threadIdx.x] = 0;
  const double s = __builtin_bit_cast(double, SV_SENTINEL);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    pay[i] = s;
}

// words: SV_COUNTER_WORDS clears the sweep counters only, the whole struct
// clears the status too
__global__ void sv_clear(SvWs* ws, int words) {
  if ((int)threadIdx.x < words) ((int32_t*)ws)[threadIdx.x] = 0;
}

namespace {
inline int64_t sv_r256(int64_t x) { return (x + 255) & ~(int64_t)255; }
// payload columns: 2 for one or two right-hand sides, 4 for more (passes of
// four), 16 for the refinement sweeps
inline int64_t sv_pay_width(int64_t nrhs, bool inv) {
  if (inv) return SV_MF_RC;
  return nrhs <= SV_RC_SMALL ? SV_RC_SMALL : SV_RC_MID;
}
inline int64_t sv_pay_entries(int64_t n, int64_t pw) { return ((n + SV_NB - 1) / SV_NB) * SV_NB * pw; }
// passes of four columns that share one launch pair (at most SV_PASSES;
// more columns take further launch pairs over the same payload areas), else
// one
inline int64_t sv_npass(int64_t nrhs, bool inv) {
  if (sv_pay_width(nrhs, inv) != SV_RC_MID) return 1;
  const int64_t p = (nrhs + SV_RC_MID - 1) / SV_RC_MID;
  return p < SV_PASSES ? p : SV_PASSES;
}
// header, then the forward and the backward payloads, each npass areas of
// `stride` entries
struct SvMap {
  SvWs* ws;
  double *ypay, *xpay;
  int64_t stride, entries;
};
SvMap sv_map(void* work, int64_t n, int64_t pw, int64_t npass = 1) {
  SvMap m;
  m.ws = (SvWs*)work;
  m.stride = sv_pay_entries(n, pw);
  m.entries = m.stride * npass;
  m.ypay = (double*)((char*)work + sv_r256(sizeof(SvWs)));
  m.xpay = (double*)((char*)m.ypay + sv_r256(8 * m.entries));
  return m;
}
void sv_launch_fill(const SvMap& m, hipStream_t st) {
  int64_t blocks = (m.entries + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(sv_fill, dim3((unsigned)blocks), dim3(256), 0, st, m.ws, SV_COUNTER_WORDS, m.ypay, m.entries);
}
}  // namespace

int64_t tc_solve_ws_bytes(int64_t n, int64_t nrhs, bool inv) {
  return sv_r256(sizeof(SvWs)) + 2 * sv_r256(8 * sv_pay_entries(n, sv_pay_width(nrhs, inv)) * sv_npass(nrhs, inv));
}

int tc_solve_status_reset(void* work, hipStream_t st) {
  hipLaunchKernelGGL(sv_clear, dim3(1), dim3(64), 0, st, (SvWs*)work, (int)(sizeof(SvWs) / 4));
  return hipGetLastError() == hipSuccess ? 0 : TC_LAUNCH_EDEVICE;
}

int tc_solve_status(const void* work, hipStream_t st, int32_t* error) {
  SvWs h;
  if (hipMemcpyAsync(&h, work, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return TC_LAUNCH_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return TC_LAUNCH_EDEVICE;
  *error = h.error;
  return 0;
}

int64_t tc_solve_status_offset() { return (int64_t)offsetof(SvWs, error); }

// D, P and Q: three arrays of 64 x 64 blocks
int64_t tc_solve_inv_bytes(int64_t n) { return 3 * ((n + SV_NB - 1) / SV_NB) * SV_NB * SV_NB * 8; }

int tc_launch_invert_diag(const double* L, int64_t n, int64_t lda, double* Dinv, hipStream_t st) {
  const int64_t nb = (n + SV_NB - 1) / SV_NB;
  double* P = Dinv + nb * SV_NB * SV_NB;
  double* Q = P + nb * SV_NB * SV_NB;
  hipLaunchKernelGGL(sv_invert_diag, dim3((unsigned)nb), dim3(SV_THREADS), 0, st, L, lda, n, Dinv);
  hipLaunchKernelGGL(sv_couple, dim3((unsigned)nb), dim3(SV_THREADS), 0, st, L, lda, n, (const double*)Dinv, P, Q);
  return hipGetLastError() == hipSuccess ? 0 : TC_LAUNCH_EDEVICE;
}

int tc_launch_solve_inv(const double* L, int64_t n, int64_t lda, const double* Dinv, double* B, int64_t nrhs,
                        int64_t ldb, void* work, hipStream_t st, int64_t wait_ticks) {
  const int64_t nb = (n + SV_NB - 1) / SV_NB;
  const double* P = Dinv + nb * SV_NB * SV_NB;
  const double* Q = P + nb * SV_NB * SV_NB;
  const SvMap m = sv_map(work, n, SV_MF_RC);
  for (int64_t c0 = 0; c0 < nrhs; c0 += SV_MF_RC) {
    const int64_t nc = nrhs - c0 < SV_MF_RC ? nrhs - c0 : SV_MF_RC;
    sv_launch_fill(m, st);
    hipLaunchKernelGGL(sv_fwd_inv, dim3((unsigned)nb), dim3(SV_THREADS), 0, st, L, lda, n, Dinv, P,
                       (const double*)(B + c0), nc, ldb, m.ypay, m.xpay, m.ws, wait_ticks);
    hipLaunchKernelGGL(sv_bwd_inv, dim3((unsigned)nb), dim3(SV_THREADS), 0, st, L, lda, n, Dinv, Q, B + c0, nc, ldb,
                       (const double*)m.ypay, m.xpay, m.ws, wait_ticks);
  }
  return hipGetLastError() == hipSuccess ? 0 : TC_LAUNCH_EDEVICE;
}

int64_t tc_solve_many_ws_bytes(int64_t n, int64_t nrhs) {
  return sv_jr256(sizeof(SvWs)) + 2 * sv_jr256(8 * sv_job_stride(n) * sv_job_passes(nrhs));
}

int64_t tc_solve_many_tickets(int64_t n, int64_t nrhs) { return ((n + SV_NB - 1) / SV_NB) * sv_job_passes(nrhs); }

int tc_launch_solve_many(const TcSolveJob* jobs, int64_t count, int64_t tickets, int64_t max_entries, int32_t* ctr,
                         hipStream_t st, int64_t wait_ticks) {
  if (count <= 0 || tickets <= 0) return 0;
  int64_t bx = (max_entries + 255) / 256;
  bx = bx < 1 ? 1 : (bx > 64 ? 64 : bx);
  const int64_t by = count < 65535 ? count : 65535;
  hipLaunchKernelGGL(sv_fill_many, dim3((unsigned)bx, (unsigned)by), dim3(256), 0, st, jobs, count, ctr);
  hipLaunchKernelGGL(sv_forward_many, dim3((unsigned)tickets), dim3(SV_THREADS), 0, st, jobs, count, ctr, wait_ticks);
  hipLaunchKernelGGL(sv_backward_many, dim3((unsigned)tickets), dim3(SV_THREADS), 0, st, jobs, count, ctr, wait_ticks);
  return hipGetLastError() == hipSuccess ? 0 : TC_LAUNCH_EDEVICE;
}

int tc_launch_solve(const double* L, int64_t n, int64_t lda, int64_t T, double* B, int64_t nrhs, int64_t ldb,
                    void* work, hipStream_t st, int64_t wait_ticks) {
  (void)T;
  const int64_t nb = (n + SV_NB - 1) / SV_NB;
  SvWs* ws = (SvWs*)work;
  if (nrhs <= SV_RC_SMALL) {  // measured faster for one or two right-hand sides
    const SvMap m = sv_map(work, n, SV_RC_SMALL);
    sv_launch_fill(m, st);
    hipLaunchKernelGGL(sv_forward<SV_RC_SMALL>, dim3((unsigned)nb), dim3(SV_THREADS), 0, st, L, lda, n,
                       (const double*)B, nrhs, ldb, m.ypay, m.xpay, ws, wait_ticks, 1, m.stride);
    hipLaunchKernelGGL(sv_backward<SV_RC_SMALL>, dim3((unsigned)nb), dim3(SV_THREADS), 0, st, L, lda, n, B, nrhs,
                       ldb, (const double*)m.ypay, m.xpay, ws, wait_ticks, 1, m.stride);
    return hipGetLastError() == hipSuccess ? 0 : TC_LAUNCH_EDEVICE;
  }
  // one chain per wave, up to SV_PASSES passes of four in one launch pair
  // (measured faster at every size than 16-column passes whose folds ran on
  // the matrix cores, four chains per wave)
  const int64_t npass = sv_npass(nrhs, false);
  const SvMap m = sv_map(work, n, SV_RC_MID, npass);
  const int64_t cols = npass * SV_RC_MID;
  for (int64_t c0 = 0; c0 < nrhs; c0 += cols) {
    const int64_t nc = nrhs - c0 < cols ? nrhs - c0 : cols;
    const int64_t np = (nc + SV_RC_MID - 1) / SV_RC_MID;
    sv_launch_fill(m, st);
    hipLaunchKernelGGL(sv_forward<SV_RC_MID>, dim3((unsigned)(nb * np)), dim3(SV_THREADS), 0, st, L, lda, n,
                       (const double*)(B + c0), nc, ldb, m.ypay, m.xpay, ws, wait_ticks, (int32_t)np, m.stride);
    hipLaunchKernelGGL(sv_backward<SV_RC_MID>, dim3((unsigned)(nb * np)), dim3(SV_THREADS), 0, st, L, lda, n,
                       B + c0, nc, ldb, (const double*)m.ypay, m.xpay, ws, wait_ticks, (int32_t)np, m.stride);
  }
  return hipGetLastError() == hipSuccess ? 0 : TC_LAUNCH_EDEVICE;
}
