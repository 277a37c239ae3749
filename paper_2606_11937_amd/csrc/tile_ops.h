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
// Left-looking MFMA accumulation for one 16 x 16 output group:
//   acc[r][j] = sum_{t < kd} X[r][t] * Y[j][t],  r < 16 (rows of X), j < 16
// X rows clamped to xr valid rows, Y rows to yr valid rows; kd % 16 == 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ tc_v4d tc_nt16(const double* __restrict__ X, int xr, const double* __restrict__ Y,
                                          int yr, int64_t lda, int kd) {
  const int lane = tc_tid() & 63;
  const int r16 = lane & 15, s4 = (lane >> 4) * 4;
  const double* px = X + (int64_t)(r16 < xr ? r16 : xr - 1) * lda + s4;
  const double* py = Y + (int64_t)(r16 < yr ? r16 : yr - 1) * lda + s4;
  tc_v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  int k0 = 0;
  // two independent accumulators over alternating chunks keep two MFMA chains
  // in flight; they are summed at the end (fixed order).
  for (; k0 + 32 <= kd; k0 += 32) {
    tc_q4 x0 = tc_ld4(px + k0), y0 = tc_ld4(py + k0);
    tc_q4 x1 = tc_ld4(px + k0 + 16), y1 = tc_ld4(py + k0 + 16);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      acc0 = tc_mfma(tc_el(x0, m), tc_el(y0, m), acc0);
      acc1 = tc_mfma(tc_el(x1, m), tc_el(y1, m), acc1);
    }
  }
  if (k0 < kd) {
    tc_q4 x0 = tc_ld4(px + k0), y0 = tc_ld4(py + k0);
#pragma unroll
    for (int m = 0; m < 4; ++m) acc0 = tc_mfma(tc_el(x0, m), tc_el(y0, m), acc0);
  }
  return acc0 + acc1;
}

// Scatter a 16 x 16 MFMA result into a row-major LDS buffer (ld 17).
__device__ __forceinline__ void tc_acc_to_lds(double* buf, tc_v4d acc) {
  const int lane = tc_tid() & 63;
  const int orow = lane >> 4, ocol = lane & 15;
#pragma unroll
  for (int q = 0; q < 4; ++q) buf[(4 * q + orow) * 17 + ocol] = acc[q];
}

// Forward substitution of one row against a factored nb x nb diagonal block
// held in LDS (Lc, ld 17):  x_j = (v_j - sum_{q<j} x_q Lc[j][q]) / Lc[j][j].
// v holds the row on entry, x on exit.  Sequential in q (ascending).
__device__ __forceinline__ void tc_subst_row(double v[16], const double* Lc, int nb) {
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    if (j < nb) {
      double s = v[j];
#pragma unroll
      for (int q = 0; q < j; ++q) s = s - v[q] * Lc[j * 17 + q];
      v[j] = s / Lc[j * 17 + j];
    }
  }
}

// ---------------------------------------------------------------------------
// TRSM work unit: X <- X L^{-T} for mr <= 128 rows of a tile (I, J), I > J,
// with L = L_JJ (td x td, factored).  Left-looking over 16-column blocks:
// for each block c0, v = X[:, c0:c0+16] - X[:, :c0] L[c0:c0+16, :c0]^T (MFMA),
// then forward substitution against the 16 x 16 diagonal block of L.
// Wave w owns rows 32w .. 32w+31 (two 16-row MFMA groups).
// LDS: 4 waves x 32 x 17 doubles + 16 x 17 doubles.
// ---------------------------------------------------------------------------
struct TcTrsmSmem {
  double buf[4][32 * 17];
  double Lc[16 * 17];
};

__device__ __forceinline__ void tc_trsm_block(double* __restrict__ X, const double* __restrict__ L, int64_t lda, int mr, int td,
                              TcTrsmSmem& sm) {
  const int tid = tc_tid(), lane = tid & 63, w = tid >> 6;
  const int row0 = w * 32;
  for (int c0 = 0; c0 < td; c0 += 16) {
    const int nb = td - c0 < 16 ? td - c0 : 16;
    // stage the diagonal block L[c0.., c0..] (lower part; rest zero)
    {
      const int i = tid >> 4, j = tid & 15;
      sm.Lc[i * 17 + j] = (i < nb && j <= i) ? L[(int64_t)(c0 + i) * lda + c0 + j] : 0.0;
    }
    // left-looking products for this wave's two row groups
    if (row0 < mr) {
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int rr = row0 + 16 * g;
        tc_v4d acc = {0.0, 0.0, 0.0, 0.0};
        if (rr < mr && c0 > 0) acc = tc_nt16(X + (int64_t)rr * lda, mr - rr, L + (int64_t)c0 * lda, nb, lda, c0);
        tc_acc_to_lds(&sm.buf[w][g * 16 * 17], acc);
      }
    }
    __syncthreads();
    if (lane < 32 && row0 + lane < mr) {
      const int r = row0 + lane;
      double* xr = X + (int64_t)r * lda + c0;
      double v[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) v[j] = j < nb ? xr[j] - sm.buf[w][lane * 17 + j] : 0.0;
      tc_subst_row(v, sm.Lc, nb);
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (j < nb) xr[j] = v[j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// POTRF work unit: in-place lower Cholesky of the td x td diagonal tile D.
// Left-looking over 16-column blocks c0:
//   1. wave 0: diagonal group v = D[c0:, c0:] - D[c0:, :c0] D[c0:, :c0]^T
//      (16 x 16, MFMA), factored unblocked in LDS (right-looking, sequential
//      over the column, the POTRF definition on a 16 x 16 block);
//   2. all waves: the 16-row groups below, MFMA products then forward
//      substitution against the new diagonal block (the in-tile TRSM).
// A pivot d <= 0 or NaN stops the factorization: returns the 0-based
// in-tile column, else -1.
// ---------------------------------------------------------------------------
struct TcPotrfSmem {
  double buf[4][16 * 17];
  double Lc[16 * 17];
  int fail;
};

__device__ __forceinline__ int tc_potrf_tile(double* __restrict__ D, int64_t lda, int td, TcPotrfSmem& sm) {
  const int tid = tc_tid(), lane = tid & 63, w = tid >> 6;
  if (tid == 0) sm.fail = -1;
  __syncthreads();
  for (int c0 = 0; c0 < td; c0 += 16) {
    const int nb = td - c0 < 16 ? td - c0 : 16;
    double* Dc = D + (int64_t)c0 * lda;  // row c0
    if (w == 0) {
      tc_v4d acc = {0.0, 0.0, 0.0, 0.0};
      if (c0 > 0) acc = tc_nt16(Dc, nb, Dc, nb, lda, c0);
      tc_acc_to_lds(sm.buf[0], acc);
    }
    __syncthreads();
    if (tid < 256) {
      const int i = tid >> 4, j = tid & 15;
      sm.Lc[i * 17 + j] = (i < nb && j <= i) ? Dc[(int64_t)i * lda + c0 + j] - sm.buf[0][i * 17 + j] : 0.0;
    }
    __syncthreads();
    // unblocked factorization of the 16 x 16 block by wave 0, column by column
    if (w == 0) {
      const int i = lane >> 2;        // row handled (16 rows x 4 lanes)
      const int kq = lane & 3;        // this lane updates columns k = kq, kq+4, ...
      for (int j = 0; j < nb; ++j) {
        const double d = tc_uniform(sm.Lc[j * 17 + j]);
        const bool ok = d > 0.0;
        if (!ok) {
          if (lane == 0 && sm.fail < 0) sm.fail = c0 + j;
          break;
        }
        const double ljj = sqrt(d);
        __builtin_amdgcn_wave_barrier();
        // column j below the diagonal; lane (i, kq==0) owns l_ij
        double lij = 0.0;
        if (i > j && i < nb) lij = sm.Lc[i * 17 + j] / ljj;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0);
        if (kq == 0) {
          if (i == j) sm.Lc[j * 17 + j] = ljj;
          else if (i > j && i < nb) sm.Lc[i * 17 + j] = lij;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // trailing update a_ik -= l_ij l_kj for j < k <= i
        if (i > j && i < nb) {
          for (int k = j + 1 + ((kq - (j + 1)) & 3); k <= i; k += 4)
            sm.Lc[i * 17 + k] = sm.Lc[i * 17 + k] - lij * sm.Lc[k * 17 + j];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    const int fail = tc_uniform((int32_t)sm.fail);
    if (fail >= 0) return fail;
    // write the factored diagonal block back
    {
      const int i = tid >> 4, j = tid & 15;
      if (i < nb && j <= i) Dc[(int64_t)i * lda + c0 + j] = sm.Lc[i * 17 + j];
    }
    // rows below the diagonal block, one 16-row group per wave at a time
    const int ngroups = (td - c0 - nb + 15) / 16;
    for (int gbase = 0; gbase < ngroups; gbase += 4) {
      const int g = gbase + w;
      const int r0 = c0 + nb + 16 * g;
      if (g < ngroups) {
        const int rows = td - r0 < 16 ? td - r0 : 16;
        tc_v4d acc = {0.0, 0.0, 0.0, 0.0};
        if (c0 > 0) acc = tc_nt16(D + (int64_t)r0 * lda, rows, Dc, nb, lda, c0);
        tc_acc_to_lds(sm.buf[w], acc);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < rows) {
          double* xr = D + (int64_t)(r0 + lane) * lda + c0;
          double v[16];
#pragma unroll
          for (int j = 0; j < 16; ++j) v[j] = j < nb ? xr[j] - sm.buf[w][lane * 17 + j] : 0.0;
          tc_subst_row(v, sm.Lc, nb);
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
