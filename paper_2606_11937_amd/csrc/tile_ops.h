// tile_ops.h -- gfx950 device bodies of the four tile operations (Methods,
// "Tiled Cholesky Decomposition": POTRF, TRSM, SYRK, GEMM).  Both schedules
// call exactly these bodies, so they produce bit-identical factors.
//
// Every body runs on one workgroup of TC_THREADS = 256 threads (4 wave64s).
// Matrices are row-major with leading dimension lda; only lower-triangle
// entries are read or written.
//
// The contraction core is v_mfma_f64_16x16x4_f64 (FP64 matrix cores).  Its
// operand/result lane layout, measured on gfx950 with one-hot inputs:
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, item q holds D[4 q + l / 16][l % 16]
// All three tile products here are of the "NT" form X Y^T with X and Y both
// row-major with the contraction index contiguous, so A and B fragments are
// loaded the same way: lane (r = l % 16, s = l / 16) reads four consecutive
// doubles k0 + 4s .. k0 + 4s + 3 of row r, and MFMA number m of a 16-wide k
// chunk consumes element m.  The contraction order inside one output entry is
// therefore fixed (chunk by chunk; within a chunk, MFMA m sums k0+m, k0+4+m,
// k0+8+m, k0+12+m) and identical for every entry and both schedules.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TC_THREADS 256

typedef double tc_v4d __attribute__((ext_vector_type(4)));
typedef double tc_d2 __attribute__((ext_vector_type(2), aligned(8)));

// Broadcast lane 0's value to the whole wave as a uniform (scalar) value.
// Values read from LDS that steer loops or branches containing barriers go
// through these, so the compiler sees the control flow as uniform and keeps
// every wave's barrier sequence identical to the source.
// Thread index behind a compiler-only barrier.  Tile bodies derive their
// lane offsets from it, so the persistent kernel recomputes them at the start
// of each body instead of hoisting them out of its unit loop, where they would
// stay live (and spill) across the other bodies.
__device__ __forceinline__ int tc_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

__device__ __forceinline__ int32_t tc_uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t tc_uniform(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(uint64_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double tc_uniform(double v) {
  const int64_t b = tc_uniform((int64_t)__builtin_bit_cast(int64_t, v));
  return __builtin_bit_cast(double, b);
}

__device__ __forceinline__ tc_v4d tc_mfma(double a, double b, tc_v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Four consecutive doubles of one row, as two 16-byte loads.
struct tc_q4 {
  tc_d2 lo, hi;
};
__device__ __forceinline__ tc_q4 tc_ld4(const double* p) {
  tc_q4 q;
  q.lo = *(const tc_d2*)p;
  q.hi = *(const tc_d2*)(p + 2);
  return q;
}
// Same, but elements at or beyond `lim` (relative to p) read as zero.
__device__ __forceinline__ tc_q4 tc_ld4_tail(const double* p, int lim) {
  tc_q4 q;
  q.lo.x = lim > 0 ? p[0] : 0.0;
  q.lo.y = lim > 1 ? p[1] : 0.0;
  q.hi.x = lim > 2 ? p[2] : 0.0;
  q.hi.y = lim > 3 ? p[3] : 0.0;
  return q;
}
__device__ __forceinline__ double tc_el(const tc_q4& q, int m) {
  return m == 0 ? q.lo.x : m == 1 ? q.lo.y : m == 2 ? q.hi.x : q.hi.y;
}

// ---------------------------------------------------------------------------
// SYRK / GEMM update of one output block (the trailing-update tile ops):
//   C[r][c] -= sum_{t < kd} PA[r][t] * PB[c][t]     0 <= r < mr, 0 <= c < mc
// restricted to r >= c when `diag` (a block on the matrix diagonal, SYRK).
// mr, mc <= 128.  Wave w computes the 64 x 64 quadrant (w & 1, w >> 1) with
// 4 x 4 MFMA accumulators.
//
// Operands are staged through LDS in 16-wide k chunks, two stages deep, with
// direct-to-LDS buffer loads (16 bytes per lane, no registers involved).
// LDS layout of one operand tile: 128 rows x 8 slots of 16 bytes (two k
// values); slot j of row r sits at position j ^ (r & 7) of its row, which
// keeps the 128-bit fragment reads of the MFMAs free of bank conflicts.  A
// direct-to-LDS load writes lane i's 16 bytes to slot i of a 64-slot window,
// so each lane fetches the global element that belongs in its slot.  The
// buffer resource spans exactly the block's mr (mc) rows: rows beyond them
// read as zero and are never stored.
//
// Fragment registers roll half a chunk ahead: the high halves (k steps 2, 3)
// of chunk c are read while the MFMAs of its low halves run; the barrier that
// publishes chunk c+1 sits in the middle of chunk c; the low halves of chunk
// c+1 are read while the MFMAs of chunk c's high halves run.  One 64-register
// fragment set and a 64 KB stage pair let two workgroups share a CU.
// ---------------------------------------------------------------------------
#define TC_UPD_STAGES 2
// The swizzle below is conflict-free only relative to a bank-period-aligned
// base, and the 128-bit reads need 16-byte alignment: the stages are placed
// on a 512-byte boundary wherever the struct is declared (alone, or inside the
// persistent kernel's union next to other shared variables).
struct alignas(512) TcUpdSmem {
  double tile[TC_UPD_STAGES][2][128 * 16];  // [stage][A|B][row * 16 + slot * 2 + e]
};

typedef __attribute__((address_space(3))) void tc_lds_void;
typedef double tc_d2a16 __attribute__((ext_vector_type(2), aligned(16)));

__device__ __forceinline__ int tc_swz(int r) { return r & 7; }

__device__ __forceinline__ void tc_update_block(double* __restrict__ C, const double* __restrict__ PA,
                                                const double* __restrict__ PB, int64_t lda, int mr, int mc,
                                                int kd, bool diag, TcUpdSmem& sm) {
  const int tid = tc_tid();
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  // waves with nothing to store still stage operands and take part in barriers
  const bool active = !(diag && wn > wm) && wm * 64 < mr && wn * 64 < mc;
  const int r16 = lane & 15, s2 = (lane >> 4) * 2;

  // --- staging: waves 0,1 fetch A rows, waves 2,3 B rows; load q of wave w
  //     fills LDS slots [(w*8+q)*64, +64) = rows (w&1)*64 + q*8 .. +8
  const int nrow = w < 2 ? mr : mc;
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(w < 2 ? PA : PB), (short)0, (int)((int64_t)nrow * lda * 8), 0x00020000);
  const int rl0 = (w & 1) * 64 + (lane >> 3);
  const unsigned vof0 = (unsigned)(rl0 * lda * 8 + 16 * ((lane & 7) ^ tc_swz(rl0)));
  const unsigned rowstep = (unsigned)(8 * lda * 8);
  auto stage_load = [&](int st, int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsrc,
          (tc_lds_void*)((char __attribute__((address_space(3)))*)(tc_lds_void*)&sm.tile[st][0][0] +
                         (w * 8 + q) * 1024),
          16, vof0 + q * rowstep, (unsigned)(k0 * 8), 0, 0);
  };
  // the ragged last chunk (kd % 16 != 0): ordinary guarded loads, zero past
  // kd or past the block's rows, stored where the direct loads would put them
  auto stage_tail = [&](int st, int k0) {
    const double* gb = w < 2 ? PA : PB;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = rl0 + q * 8;
      const int j = (lane & 7) ^ tc_swz(r);
      const int k = k0 + 2 * j;
      const double* src = gb + (int64_t)(r < nrow ? r : 0) * lda + k;
      tc_d2 v;
      v.x = (r < nrow && k < kd) ? src[0] : 0.0;
      v.y = (r < nrow && k + 1 < kd) ? src[1] : 0.0;
      *(tc_d2*)(&sm.tile[st][0][0] + ((w * 8 + q) * 64 + lane) * 2) = v;
    }
  };
  auto stage = [&](int st, int c, int nfull) {
    if (c < nfull) stage_load(st, c * 16); else stage_tail(st, c * 16);
  };
  // fragment half h (k = 4s + 2h, 4s + 2h + 1) of row-block i of operand t
  // (0 = A rows wm*64.., 1 = B rows wn*64..)
  auto rd = [&](int st, int t, int i, int h) -> tc_d2 {
    const int r = (t == 0 ? wm : wn) * 64 + i * 16 + r16;
    const tc_d2a16 v = *(const tc_d2a16*)(&sm.tile[st][t][r * 16] + 2 * ((s2 + h) ^ tc_swz(r)));
    tc_d2 o;
    o.x = v.x;
    o.y = v.y;
    return o;
  };

  tc_v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = tc_v4d{0.0, 0.0, 0.0, 0.0};

  // (s_waitcnt encodings: 0x0F70 = vmcnt(0); 0x0070 = vmcnt(0) lgkmcnt(0);
  //  expcnt and unnamed counters at their maxima)
  const int nfull = kd >> 4;
  const int nch = (kd + 15) >> 4;
  tc_d2 La[4], Lb[4], Ha[4], Hb[4];
  if (nch > 0) stage(0, 0, nfull);
  if (nch > 1) stage(1, 1, nfull);
  __builtin_amdgcn_s_waitcnt(0x0070);
  __builtin_amdgcn_s_barrier();
  if (active && nch > 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      La[i] = rd(0, 0, i, 0);
      Lb[i] = rd(0, 1, i, 0);
    }
  }
  for (int c = 0; c < nch; ++c) {
    const int st = c & 1;
    if (active) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        Ha[i] = rd(st, 0, i, 1);
        Hb[i] = rd(st, 1, i, 1);
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = tc_mfma(m ? La[i].y : La[i].x, m ? Lb[j].y : Lb[j].x, acc[i][j]);
    }
    if (c + 1 < nch) {
      // chunk c+1 has landed and this wave's reads of chunk c are complete;
      // a plain barrier (a fenced one would also wait for unrelated traffic)
      __builtin_amdgcn_s_waitcnt(0x0070);
      __builtin_amdgcn_s_barrier();
      if (c + 2 < nch) stage(st, c + 2, nfull);  // chunk c's stage is free now
      if (active) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          La[i] = rd(st ^ 1, 0, i, 0);
          Lb[i] = rd(st ^ 1, 1, i, 0);
        }
      }
    }
    if (active) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = tc_mfma(m ? Ha[i].y : Ha[i].x, m ? Hb[j].y : Hb[j].x, acc[i][j]);
    }
  }
  if (!active) return;

  // epilogue: C -= acc on the stored part, one 16-row group at a time (the
  // scheduling barriers keep the compiler from hoisting all 64 loads of C
  // ahead of the first subtraction, which would need 128 more registers)
  const int orow = lane >> 4, ocol = lane & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * 64 + i * 16 + 4 * q + orow;
        const int c = wn * 64 + j * 16 + ocol;
        if (r < mr && c < mc && (!diag || r >= c)) {
          double* p = C + (int64_t)r * lda + c;
          *p = *p - acc[i][j][q];
        }
      }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// ---------------------------------------------------------------------------
// Left-looking MFMA products of G 16-row groups against one 16-row group:
//   acc[g][r][j] += sum over the 16-wide k chunks c = cs, cs + step, ... < kd/16
//                   of X[16 g + r][k] Y[j][k],
// X rows clamped to xr valid rows, Y rows to yr valid rows, kd % 16 == 0.
// Each group has one accumulator, so a group's sum runs over its chunks in
// ascending order; splitting the chunks of a product over several waves
// (cs = wave, step = number of waves) gives partial sums that the caller adds
// in a fixed order.  The Y fragment is shared by the G groups, whose
// independent MFMA chains hide one another's latency, and the loads of the
// next chunk are issued before the MFMAs of the current one.
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ void tc_ntg(const double* __restrict__ X, int xr, const double* __restrict__ Y, int yr,
                                       int64_t lda, int kd, int cs, int step, tc_v4d acc[G]) {
  const int lane = tc_tid() & 63;
  const int r16 = lane & 15, s4 = (lane >> 4) * 4;
  const double* py = Y + (int64_t)(r16 < yr ? r16 : yr - 1) * lda + s4;
  const double* px[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int r = 16 * g + r16;
    px[g] = X + (int64_t)(r < xr ? r : xr - 1) * lda + s4;
  }
  const int nch = kd >> 4;
  if (cs >= nch) return;
  tc_q4 y = tc_ld4(py + 16 * cs), x[G];
#pragma unroll
  for (int g = 0; g < G; ++g) x[g] = tc_ld4(px[g] + 16 * cs);
  for (int c = cs; c < nch; c += step) {
    const int cn = c + step < nch ? c + step : c;  // the last pass re-reads its own chunk
    const tc_q4 yn = tc_ld4(py + 16 * cn);
    tc_q4 xn[G];
#pragma unroll
    for (int g = 0; g < G; ++g) xn[g] = tc_ld4(px[g] + 16 * cn);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int g = 0; g < G; ++g) acc[g] = tc_mfma(tc_el(x[g], m), tc_el(y, m), acc[g]);
    y = yn;
#pragma unroll
    for (int g = 0; g < G; ++g) x[g] = xn[g];
  }
}

// Scatter a 16 x 16 MFMA result into a row-major LDS buffer (ld 17).
__device__ __forceinline__ void tc_acc_to_lds(double* buf, tc_v4d acc) {
  const int lane = tc_tid() & 63;
  const int orow = lane >> 4, ocol = lane & 15;
#pragma unroll
  for (int q = 0; q < 4; ++q) buf[(4 * q + orow) * 17 + ocol] = acc[q];
}

// The G-group products of tc_ntg written to LDS as 16 G rows of ld 17.
template <int G>
__device__ __forceinline__ void tc_ntg_lds(const double* __restrict__ X, int xr, const double* __restrict__ Y,
                                           int yr, int64_t lda, int kd, int cs, int step, double* buf) {
  tc_v4d acc[G];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g] = tc_v4d{0.0, 0.0, 0.0, 0.0};
  tc_ntg<G>(X, xr, Y, yr, lda, kd, cs, step, acc);
#pragma unroll
  for (int g = 0; g < G; ++g) tc_acc_to_lds(buf + g * 16 * 17, acc[g]);
}

// The factored 16 x 16 diagonal block is kept in LDS transposed, one column
// of L per TC_LT-double row (16-byte aligned): Lt[j * TC_LT + i] = L[i][j]
// for i >= j, zero above; Lt[j * TC_LT + 16] holds 1 / L[j][j].  Columns j
// past the block's order nb hold a unit diagonal, so a substitution can run
// all 16 steps unconditionally (their values stay zero).  The values one
// step needs are contiguous and every lane reads the same address.
#define TC_LT 18

// x / d from the correctly rounded reciprocal r = 1 / d and one residual
// correction (Markstein's method): q0 = x r, e = x - q0 d (exact with an
// FMA), q = q0 + e r.  The result is exact whenever x / d is representable
// and otherwise within one unit in the last place of the rounded quotient.
// It takes three dependent operations instead of a full division.
__device__ __forceinline__ double tc_div_rcp(double x, double d, double r) {
  const double q0 = x * r;
  const double e = __builtin_fma(-q0, d, x);
  return __builtin_fma(e, r, q0);
}

// Forward substitution of one row against the factored diagonal block:
//   x_j = (v_j - sum_{q<j} x_q L[j][q]) / L[j][j].
// v holds the row on entry, x on exit (entries past nb are zero on entry and
// stay zero).  Column-oriented: step j finishes x_j and then subtracts
// x_j L[i][j] from every later v_i, so each v_i receives the subtractions of
// the row-oriented form in the same ascending order of q; the column of L
// for step j + 1 is read while step j computes.
__device__ __forceinline__ void tc_subst_row(double v[16], const double* Lt) {
  double cur[17];
#pragma unroll
  for (int i = 0; i < 17; ++i) cur[i] = Lt[i];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    // a compiler-only barrier per step that also pins the previous result:
    // the LDS loads of column j + 1 may overlap step j, but neither loads are
    // hoisted nor arithmetic sunk across steps (each column held in registers
    // costs 34 of them)
    if (j > 0) asm volatile("" : "+v"(v[j - 1]) : : "memory");
    double nxt[17];
    if (j + 1 < 16) {
#pragma unroll
      for (int i = j + 1; i < 17; ++i) nxt[i] = Lt[(j + 1) * TC_LT + i];
    }
    v[j] = tc_div_rcp(v[j], cur[j], cur[16]);
#pragma unroll
    for (int i = j + 1; i < 16; ++i) v[i] = v[i] - v[j] * cur[i];
    if (j + 1 < 16) {
#pragma unroll
      for (int i = j + 1; i < 17; ++i) cur[i] = nxt[i];
    }
  }
}

// Stage the lower nb x nb part of the 16 x 16 block at B (row-major, ld lda)
// into Lt (transposed, zero-filled, unit diagonal past nb, reciprocals of
// the diagonal); all TC_THREADS threads take part.
__device__ __forceinline__ void tc_stage_lt(double* Lt, const double* B, int64_t lda, int nb) {
  const int tid = tc_tid();
  const int i = tid >> 4, j = tid & 15;
  const double val = (i < nb && j <= i) ? B[(int64_t)i * lda + j] : (i == j ? 1.0 : 0.0);
  Lt[j * TC_LT + i] = val;
  if (i == j) Lt[j * TC_LT + 16] = 1.0 / val;
}

__device__ __forceinline__ double tc_readlane(double v, int l) {
  const int64_t b = __builtin_bit_cast(int64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(uint64_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)((uint64_t)b >> 32), l);
  return __builtin_bit_cast(double, (int64_t)(((uint64_t)hi << 32) | lo));
}

// ---------------------------------------------------------------------------
// TRSM work unit: X <- X L^{-T} for mr <= 128 rows of a tile (I, J), I > J,
// with L = L_JJ (td x td, factored).  Left-looking over 16-column blocks:
// for each block c0, v = X[:, c0:c0+16] - X[:, :c0] L[c0:c0+16, :c0]^T (MFMA),
// then forward substitution against the 16 x 16 diagonal block of L.
// Waves 0 and 1 own rows 0..63 and 64..127: they form the even-chunk part of
// the products of their rows and substitute them, one row per lane; waves 2
// and 3 form the odd-chunk part of the same rows.  A row's 16 inputs are
// fetched before the products so that their latency hides behind them.
// ---------------------------------------------------------------------------
struct alignas(16) TcTrsmSmem {
  double buf[4][64 * 17];  // [wave] products: even chunks (waves 0, 1), odd (2, 3)
  double Lt[16 * TC_LT];
};

__device__ __forceinline__ void tc_trsm_block(double* __restrict__ X, const double* __restrict__ L, int64_t lda, int mr, int td,
                              TcTrsmSmem& sm) {
  const int tid = tc_tid(), lane = tid & 63, w = tid >> 6;
  const int half = w & 1;
  const int row0 = half * 64;
  const int nrows = mr - row0 < 64 ? mr - row0 : 64;  // rows of this half (may be <= 0)
  const bool mine = w < 2 && lane < nrows;
  double* xr0 = X + (int64_t)(row0 + (mine ? lane : 0)) * lda;
  for (int c0 = 0; c0 < td; c0 += 16) {
    const int nb = td - c0 < 16 ? td - c0 : 16;
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = (mine && j < nb) ? xr0[c0 + j] : 0.0;
    tc_stage_lt(sm.Lt, L + (int64_t)c0 * lda + c0, lda, nb);
    if (nrows > 0 && c0 > 0)
      tc_ntg_lds<4>(X + (int64_t)row0 * lda, nrows, L + (int64_t)c0 * lda, nb, lda, c0, w >> 1, 2, sm.buf[w]);
    __syncthreads();
    if (mine) {
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (j < nb && c0 > 0) v[j] = v[j] - (sm.buf[half][lane * 17 + j] + sm.buf[half + 2][lane * 17 + j]);
      tc_subst_row(v, sm.Lt);
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (j < nb) xr0[c0 + j] = v[j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// POTRF work unit: in-place lower Cholesky of the td x td diagonal tile D.
// Left-looking over 16-column blocks c0:
//   1. diagonal group v = D[c0:, c0:] - D[c0:, :c0] D[c0:, :c0]^T (16 x 16,
//      MFMA, the k chunks dealt to the four waves and their partial sums
//      added in wave order), then by wave 0 the unblocked factorization in
//      registers (right-looking, sequential over the column, the POTRF
//      definition on a 16 x 16 block): lane i holds row i, and the pivot
//      and the column entries each step needs are read from their owner
//      lanes;
//   2. waves 0 and 1: the rows below, 64 per wave at a time (one per lane):
//      MFMA products, then forward substitution against the new diagonal
//      block (the in-tile TRSM).
// A pivot d <= 0 or NaN stops the factorization: returns the 0-based
// in-tile column, else -1.
// ---------------------------------------------------------------------------
struct alignas(16) TcPotrfSmem {
  double buf[2][64 * 17];    // products of the rows below (waves 0 and 1)
  double dpart[4][16 * 17];  // partial products of the diagonal group
  double Lt[16 * TC_LT];
  int fail;
};

__device__ __forceinline__ int tc_potrf_tile(double* __restrict__ D, int64_t lda, int td, TcPotrfSmem& sm) {
  const int tid = tc_tid(), lane = tid & 63, w = tid >> 6;
  if (tid == 0) sm.fail = -1;
  __syncthreads();
  for (int c0 = 0; c0 < td; c0 += 16) {
    const int nb = td - c0 < 16 ? td - c0 : 16;
    double* Dc = D + (int64_t)c0 * lda;  // row c0
    const bool own = w == 0 && lane < nb;
    const double* dr = Dc + (int64_t)(own ? lane : 0) * lda + c0;
    double a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = (own && k <= lane) ? dr[k] : 0.0;
    // diagonal group products, the chunks dealt to the four waves
    if (c0 > 0) tc_ntg_lds<1>(Dc, nb, Dc, nb, lda, c0, w, 4, sm.dpart[w]);
    __syncthreads();
    if (w == 0) {
      if (c0 > 0) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (own && k <= lane) {
            const int q = lane * 17 + k;
            a[k] = a[k] - (((sm.dpart[0][q] + sm.dpart[1][q]) + sm.dpart[2][q]) + sm.dpart[3][q]);
          }
      }
      // unblocked factorization; every branch below is wave-uniform
      int bad = -1;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        double rj = 1.0;
        if (j < nb && bad < 0) {
          const double d = tc_readlane(a[j], j);
          if (!(d > 0.0)) {
            bad = j;
          } else {
            const double ljj = sqrt(d);
            rj = 1.0 / ljj;
            if (lane == j) a[j] = ljj;
            else if (lane > j) a[j] = tc_div_rcp(a[j], ljj, rj);
            // trailing update a_ik -= l_ij l_kj for j < k <= i
#pragma unroll
            for (int k = j + 1; k < 16; ++k) {
              const double lkj = tc_readlane(a[j], k);
              if (lane >= k) a[k] = a[k] - a[j] * lkj;
            }
          }
        }
        if (lane == 0) sm.Lt[j * TC_LT + 16] = rj;
      }
      if (lane == 0 && bad >= 0) sm.fail = c0 + bad;
      if (lane < 16) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
          sm.Lt[k * TC_LT + lane] = (own && k <= lane) ? a[k] : (k == lane ? 1.0 : 0.0);
      }
      if (own && bad < 0) {
        double* o = Dc + (int64_t)lane * lda + c0;
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k <= lane) o[k] = a[k];
      }
    }
    __syncthreads();
    const int fail = tc_uniform((int32_t)sm.fail);
    if (fail >= 0) return fail;
    // rows below the diagonal block, 64 per wave of waves 0 and 1 at a time
    const int below = td - c0 - nb;
    for (int rb = 0; rb < below; rb += 128) {
      const int rw0 = c0 + nb + rb + 64 * w;
      const int myrows = w < 2 ? (td - rw0 < 64 ? td - rw0 : 64) : 0;
      if (myrows > 0) {
        const bool mine = lane < myrows;
        double* xr = D + (int64_t)(rw0 + (mine ? lane : 0)) * lda + c0;
        double v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = (mine && j < nb) ? xr[j] : 0.0;
        if (c0 > 0) {
          tc_ntg_lds<4>(D + (int64_t)rw0 * lda, myrows, Dc, nb, lda, c0, 0, 1, sm.buf[w]);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (mine) {
          if (c0 > 0) {
#pragma unroll
            for (int j = 0; j < 16; ++j)
              if (j < nb) v[j] = v[j] - sm.buf[w][lane * 17 + j];
          }
          tc_subst_row(v, sm.Lt);
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (j < nb) xr[j] = v[j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
  }
  return -1;
}
