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
  //     fills LDS slots [(w*8+q)*64, +64) = rows (w&1)*64 + q*8 .. +8.
  //     The operand, its row count and the LDS window depend on the wave
  //     only: taken as scalars, the buffer resource and the LDS base sit in
  //     scalar registers (a resource in vector registers would turn every
  //     load into a loop over the distinct values the lanes hold).
  const int ws = tc_uniform((int32_t)w);
  const int nrow = ws < 2 ? tc_uniform((int32_t)mr) : tc_uniform((int32_t)mc);
  const double* src = (const double*)tc_uniform((int64_t)(ws < 2 ? PA : PB));
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)src, (short)0, (int)((int64_t)nrow * tc_uniform(lda) * 8), 0x00020000);
  const int rl0 = (w & 1) * 64 + (lane >> 3);
  const unsigned vof0 = (unsigned)(rl0 * lda * 8 + 16 * ((lane & 7) ^ tc_swz(rl0)));
  const unsigned rowstep = (unsigned)(8 * lda * 8);
  auto stage_load = [&](int st, int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsrc,
          (tc_lds_void*)((char __attribute__((address_space(3)))*)(tc_lds_void*)&sm.tile[st][0][0] +
                         (ws * 8 + q) * 1024),
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

  // epilogue: C -= acc on the stored part, one 16-row group at a time.  A
  // full block reads its C values unconditionally (for a diagonal block the
  // entries above the diagonal are read and left alone), the loads of the
  // next group issued before the current one is stored, so each wave has at
  // most one memory round trip outstanding per group instead of one per
  // element; the scheduling barriers keep the compiler from hoisting more
  // loads (each group takes 32 registers).  A ragged block reads from
  // clamped positions and guards its stores.
  const int orow = lane >> 4, ocol = lane & 15;
  if (mr == 128 && mc == 128) {
    double* cb = C + (int64_t)(wm * 64 + orow) * lda + wn * 64 + ocol;
    double cv[2][16];
    auto cload = [&](double(&v)[16], int i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double* rp = cb + (int64_t)(i * 16 + 4 * q) * lda;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[4 * q + j] = rp[16 * j];
      }
    };
    auto cstore = [&](const double(&v)[16], int i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double* rp = cb + (int64_t)(i * 16 + 4 * q) * lda;
        const int r = wm * 64 + i * 16 + 4 * q + orow;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = wn * 64 + j * 16 + ocol;
          if (!diag || r >= c) rp[16 * j] = v[4 * q + j] - acc[i][j][q];
        }
      }
    };
    cload(cv[0], 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i + 1 < 4) cload(cv[(i + 1) & 1], i + 1);
      __builtin_amdgcn_sched_barrier(0);
      cstore(cv[i & 1], i);
    }
  } else {
    // ragged: the same pipeline, loads from clamped (in-block) positions,
    // stores guarded
    double cv[2][16];
    auto cload = [&](double(&v)[16], int i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * 64 + i * 16 + 4 * q + orow;
        const double* rp = C + (int64_t)(r < mr ? r : mr - 1) * lda;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = wn * 64 + j * 16 + ocol;
          v[4 * q + j] = rp[c < mc ? c : mc - 1];
        }
      }
    };
    auto cstore = [&](const double(&v)[16], int i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * 64 + i * 16 + 4 * q + orow;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = wn * 64 + j * 16 + ocol;
          if (r < mr && c < mc && (!diag || r >= c)) C[(int64_t)r * lda + c] = v[4 * q + j] - acc[i][j][q];
        }
      }
    };
    cload(cv[0], 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i + 1 < 4) cload(cv[(i + 1) & 1], i + 1);
      __builtin_amdgcn_sched_barrier(0);
      cstore(cv[i & 1], i);
    }
  }
}

// ---------------------------------------------------------------------------
// Division and lane reads used by the substitutions.
// ---------------------------------------------------------------------------

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

__device__ __forceinline__ double tc_readlane(double v, int l) {
  const int64_t b = __builtin_bit_cast(int64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)(uint64_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)((uint64_t)b >> 32), l);
  return __builtin_bit_cast(double, (int64_t)(((uint64_t)hi << 32) | lo));
}

// Orders this wave's LDS writes before its later reads of them from other
// lanes (LDS operations of one wave complete in order; the fences keep the
// compiler from moving them).
__device__ __forceinline__ void tc_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// LDS images of 16 x 16 blocks.  A block row is 128 bytes: eight 16-byte
// slots of two doubles.  Slot s of row r sits at position s ^ (r & 7) of the
// row (the swizzle of the update kernel), so that one slot read by 16 rows,
// or whole rows read by 8 lanes, spread over the banks.  `rs` is the row
// stride in doubles of the array the block sits in.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tc_bo(int r, int c, int rs) { return r * rs + ((((c >> 1) ^ r) & 7) << 1) + (c & 1); }

// Row r of a block (16 doubles), as eight 16-byte accesses.
__device__ __forceinline__ void tc_row_get(const double* blk, int r, int rs, double v[16]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const tc_d2a16 p = *(const tc_d2a16*)(blk + r * rs + ((s ^ (r & 7)) << 1));
    v[2 * s] = p.x;
    v[2 * s + 1] = p.y;
  }
}
__device__ __forceinline__ void tc_row_put(double* blk, int r, int rs, const double v[16]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    tc_d2a16 p;
    p.x = v[2 * s];
    p.y = v[2 * s + 1];
    *(tc_d2a16*)(blk + r * rs + ((s ^ (r & 7)) << 1)) = p;
  }
}
// MFMA operand fragment of lane (r, s): row r, columns 4 s .. 4 s + 3.
__device__ __forceinline__ tc_q4 tc_frag_get(const double* blk, int r, int s, int rs) {
  const tc_d2a16 a = *(const tc_d2a16*)(blk + r * rs + (((2 * s) ^ (r & 7)) << 1));
  const tc_d2a16 b = *(const tc_d2a16*)(blk + r * rs + (((2 * s + 1) ^ (r & 7)) << 1));
  tc_q4 q;
  q.lo = tc_d2{a.x, a.y};
  q.hi = tc_d2{b.x, b.y};
  return q;
}
// A block in the MFMA result layout: lane l, item q is element (4 q + l / 16, l % 16).
__device__ __forceinline__ tc_v4d tc_acc_get(const double* blk, int lane, int rs) {
  tc_v4d a;
#pragma unroll
  for (int q = 0; q < 4; ++q) a[q] = blk[tc_bo(4 * q + (lane >> 4), lane & 15, rs)];
  return a;
}
__device__ __forceinline__ void tc_acc_put(double* blk, int lane, int rs, tc_v4d a) {
#pragma unroll
  for (int q = 0; q < 4; ++q) blk[tc_bo(4 * q + (lane >> 4), lane & 15, rs)] = a[q];
}
// c - X Y^T for 16 x 16 blocks and K = 16: x, y are the fragments of lane
// (l % 16, l / 16) of X and Y, c is in the result layout.  MFMA m sums the
// k = 4 s + m of the four lane groups s, so the contraction order is fixed.
__device__ __forceinline__ tc_v4d tc_nt16(const tc_q4& x, const tc_q4& y, tc_v4d c) {
#pragma unroll
  for (int m = 0; m < 4; ++m) c = tc_mfma(-tc_el(x, m), tc_el(y, m), c);
  return c;
}

// ---------------------------------------------------------------------------
// A factored 16 x 16 diagonal block packed by columns for the substitutions:
// column j holds 1 / L[j][j], then L[j+1 .. 15][j], padded to an even count
// (from offset tc_ltp(j), which is even, so pairs are read 16 bytes at a
// time; 144 doubles in all).  Columns past the block's order hold a unit
// diagonal and zeros, so a substitution runs all 16 steps unconditionally
// (entries past the order stay zero).
// ---------------------------------------------------------------------------
#define TC_LTP 144
__host__ __device__ constexpr int tc_ltp(int j) {
  int o = 0;
  for (int q = 0; q < j; ++q) o += (17 - q) & ~1;
  return o;
}

// 1 / x from the hardware estimate and two Newton-Raphson steps
// (r <- r + r (1 - x r)); within one unit in the last place.
__device__ __forceinline__ double tc_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// Forward substitution of one row against a packed diagonal block:
//   x_j = (v_j - sum_{q<j} x_q L[j][q]) (1 / L[j][j]).
// v holds the row on entry, x on exit.  Column-oriented: step j finishes x_j
// and then subtracts x_j L[i][j] from every later v_i, so each v_i receives
// the subtractions of the row-oriented form in ascending order of q; the
// column for step j + 1 is read while step j computes.  Scaling by the
// reciprocal of the pivot is the reference BLAS triangular solve's choice.
__device__ __forceinline__ void tc_subst_row(double v[16], const double* lt) {
  double cur[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) cur[t] = lt[t];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    // a compiler-only barrier per step that also pins the previous result:
    // the LDS loads of column j + 1 may overlap step j, but neither loads are
    // hoisted nor arithmetic sunk across steps
    if (j > 0) asm volatile("" : "+v"(v[j - 1]) : : "memory");
    double nxt[16];
    if (j + 1 < 16) {
#pragma unroll
      for (int t = 0; t < 15 - j; ++t) nxt[t] = lt[tc_ltp(j + 1) + t];
    }
    v[j] = v[j] * cur[0];
#pragma unroll
    for (int i = j + 1; i < 16; ++i) v[i] = v[i] - v[j] * cur[i - j];
    if (j + 1 < 16) {
#pragma unroll
      for (int t = 0; t < 15 - j; ++t) cur[t] = nxt[t];
    }
  }
}

// ---------------------------------------------------------------------------
// TRSM work unit: X <- X L^{-T} for mr <= 128 rows of a tile (I, J), I > J,
// with L = L_JJ (td x td, factored).  Right-looking over 16-column blocks b:
// forward substitution of X[:, b] against L_bb, then X[:, j] -= X[:, b] L_jb^T
// for every block j > b (MFMA, K = 16).
// Rows are independent, so the work is split by rows and kept in LDS, 64
// rows at a time: wave w owns 16 of them and sweeps them alone (lanes 0..15
// substitute one row each, all 64 lanes form the products), with no
// workgroup barrier inside the sweep.  The diagonal blocks of L are staged
// packed in LDS; the L_jb fragments are read from global memory one step
// ahead (every row block of the sub-column reads them, so they stay in L2).
// ---------------------------------------------------------------------------
#define TC_XRS 128  // row stride of the X image, doubles
struct alignas(16) TcTrsmSmem {
  double x[64 * TC_XRS];  // 64 rows x 8 column blocks, swizzled within a block
  double lt[8 * TC_LTP];  // packed diagonal blocks of L
};

// The packed diagonal blocks of L (td x td, td <= 128); all threads take
// part, every load issued before the first store.
__device__ __forceinline__ void tc_trsm_stage_lt(const double* __restrict__ L, int64_t lda, int td, TcTrsmSmem& sm) {
  const int tot = ((td + 15) >> 4) * TC_LTP;
  double val[5];
  bool rcp[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {  // 5 * 256 >= 8 * 144
    const int e = tc_tid() + k * TC_THREADS;
    const int b = e / TC_LTP, q = e - b * TC_LTP;
    int j = 0;
#pragma unroll
    for (int t = 1; t < 16; ++t) j += q >= tc_ltp(t);
    const int i = j + q - tc_ltp(j);  // row of the entry (i == j: the pivot's reciprocal)
    const int gr = 16 * b + i, gc = 16 * b + j;
    rcp[k] = i == j;
    val[k] = (e < tot && i < 16 && gr < td) ? L[(int64_t)gr * lda + gc] : (i == j ? 1.0 : 0.0);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int e = tc_tid() + k * TC_THREADS;
    if (e < tot) sm.lt[e] = rcp[k] ? 1.0 / val[k] : val[k];
  }
}

// Up to 64 rows (mr) of X against the staged diagonal blocks of L.  Starts
// with a workgroup barrier after staging X (which also publishes the staged
// diagonal blocks); each wave writes its own rows back at the end.
__device__ __forceinline__ void tc_trsm_half(double* __restrict__ X, const double* __restrict__ L, int64_t lda, int mr,
                                             int td, TcTrsmSmem& sm) {
  const int tid = tc_tid(), lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, s4 = lane >> 4;
  const int nbk = (td + 15) >> 4;
  {  // X rows [0, mr) x columns [0, td), zero elsewhere: 16 slots per thread
    tc_d2 v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int row = 4 * k + w, c = 2 * lane;
      const double* p = X + (int64_t)row * lda + c;
      v[k].x = (row < mr && c < td) ? p[0] : 0.0;
      v[k].y = (row < mr && c + 1 < td) ? p[1] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int row = 4 * k + w;
      tc_d2a16 p;
      p.x = v[k].x;
      p.y = v[k].y;
      *(tc_d2a16*)(sm.x + row * TC_XRS + (lane >> 3) * 16 + (((lane & 7) ^ (row & 7)) << 1)) = p;
    }
  }
  // fragments of L_jb (lane (r16, s4): row 16 j + r16, columns 16 b + 4 s4 ..)
  tc_q4 fa[7], fb[7];
  auto load_frags = [&](tc_q4 f[7], int b) {
#pragma unroll
    for (int jj = 0; jj < 7; ++jj) {
      const int row = 16 * (b + 1 + jj) + r16;
      if (b + 1 + jj < nbk) {
        if (row < td) {
          f[jj] = tc_ld4(L + (int64_t)row * lda + 16 * b + 4 * s4);
        } else {
          f[jj].lo = tc_d2{0.0, 0.0};
          f[jj].hi = tc_d2{0.0, 0.0};
        }
      }
    }
  };
  if (nbk > 1) load_frags(fa, 0);
  __syncthreads();

  double* xw = sm.x + 16 * w * TC_XRS;  // this wave's 16 rows
  // step b with its fragments in cur; the next step's are loaded into nxt
  // between the substitution and the products, so they land behind this
  // step's products and the next substitution
  auto step = [&](int b, tc_q4 (&cur)[7], tc_q4 (&nxt)[7]) {
    if (lane < 16) {
      double v[16];
      tc_row_get(xw + 16 * b, lane, TC_XRS, v);
      tc_subst_row(v, sm.lt + b * TC_LTP);
      tc_row_put(xw + 16 * b, lane, TC_XRS, v);
    }
    tc_wave_sync();
    if (b + 1 < nbk) {
      if (b + 2 < nbk) load_frags(nxt, b + 1);
      const tc_q4 xb = tc_frag_get(xw + 16 * b, r16, s4, TC_XRS);
      // blocks j = b + 1 + jj in two groups (4 + 3), each group's MFMA
      // chains interleaved
#pragma unroll
      for (int g0 = 0; g0 < 7; g0 += 4) {
        tc_v4d acc[4];
#pragma unroll
        for (int jj = g0; jj < g0 + 4 && jj < 7; ++jj)
          if (b + 1 + jj < nbk) acc[jj - g0] = tc_acc_get(xw + 16 * (b + 1 + jj), lane, TC_XRS);
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int jj = g0; jj < g0 + 4 && jj < 7; ++jj)
            if (b + 1 + jj < nbk) acc[jj - g0] = tc_mfma(-tc_el(xb, m), tc_el(cur[jj], m), acc[jj - g0]);
#pragma unroll
        for (int jj = g0; jj < g0 + 4 && jj < 7; ++jj)
          if (b + 1 + jj < nbk) tc_acc_put(xw + 16 * (b + 1 + jj), lane, TC_XRS, acc[jj - g0]);
      }
      tc_wave_sync();
    }
  };
  for (int b = 0; b < nbk; b += 2) {
    step(b, fa, fb);
    if (b + 1 < nbk) step(b + 1, fb, fa);
  }
  // this wave's rows back to X
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int row = 16 * w + k, c = 2 * lane;
    if (row < mr) {
      const tc_d2a16 p = *(const tc_d2a16*)(sm.x + row * TC_XRS + (lane >> 3) * 16 + (((lane & 7) ^ (row & 7)) << 1));
      double* g = X + (int64_t)row * lda + c;
      if (c < td) g[0] = p.x;
      if (c + 1 < td) g[1] = p.y;
    }
  }
}

// One half (mr <= 64 rows) of a TRSM unit, as a workgroup of its own.
__device__ __forceinline__ void tc_trsm_rows(double* __restrict__ X, const double* __restrict__ L, int64_t lda, int mr,
                                             int td, TcTrsmSmem& sm) {
  mr = tc_uniform((int32_t)mr);
  td = tc_uniform((int32_t)td);
  tc_trsm_stage_lt(L, lda, td, sm);
  tc_trsm_half(X, L, lda, mr, td, sm);
}

// A whole TRSM unit (mr <= 128 rows): its halves one after the other.  Each
// row's arithmetic is the same as in tc_trsm_rows.
__device__ __forceinline__ void tc_trsm_block(double* __restrict__ X, const double* __restrict__ L, int64_t lda, int mr,
                                              int td, TcTrsmSmem& sm) {
  mr = tc_uniform((int32_t)mr);
  td = tc_uniform((int32_t)td);
  tc_trsm_stage_lt(L, lda, td, sm);
  for (int h = 0; h < mr; h += 64) {
    if (h > 0) __syncthreads();  // the previous half's write-back has read the X image
    tc_trsm_half(X + (int64_t)h * lda, L, lda, mr - h < 64 ? mr - h : 64, td, sm);
  }
}

// ---------------------------------------------------------------------------
// POTRF work unit: in-place lower Cholesky of the td x td diagonal tile D
// (td <= 128).  The lower triangle is copied once into LDS as packed 16 x 16
// blocks (block (i, j), j <= i, at index i (i + 1) / 2 + j), factored there
// right-looking over 16-column blocks b, and copied back once:
//   1. diagonal block (b, b): unblocked factorization in registers by wave 0
//      (lane i holds row i; right-looking over the block's columns, the
//      POTRF definition on the block; the pivot and the column entries each
//      step needs are read from their owner lanes);
//   2. blocks (i, b), i > b: forward substitution against L_bb, one row per
//      thread;
//   3. blocks (i, j), b < j <= i: A_ij -= L_ib L_jb^T (MFMA, K = 16).
// In step 3 wave 0 updates only block (b+1, b+1) and then factors it (step 1
// of b+1) while waves 1..3 update the other blocks.
// A pivot d <= 0 or NaN stops the factorization: returns the 0-based in-tile
// column, else -1 (the tile is then left partly factored).
// ---------------------------------------------------------------------------
struct alignas(16) TcPotrfSmem {
  double blk[36][256];  // packed lower triangle
  double lt[TC_LTP];    // the current diagonal block, packed by columns
  int fail;
};

__device__ __forceinline__ int tc_pk(int i, int j) { return i * (i + 1) / 2 + j; }

// Lower triangle of D (rows and columns < td) into the packed blocks (zeros
// elsewhere), or (OUT) back into D.  Pass k moves blocks 2 k and 2 k + 1
// (waves 0-1 and 2-3, 16 rows x 8 slots each), so the block of a pass is
// uniform per wave; all loads are issued before the first store.
template <bool OUT>
__device__ __forceinline__ void tc_pk_copy(double* __restrict__ D, int64_t lda, int td, TcPotrfSmem& sm) {
  const int tid = tc_tid();
  const int nbk = (td + 15) >> 4;
  const int nblk = nbk * (nbk + 1) / 2;
  const int hi = tc_uniform((int32_t)(tid >> 7));
  const int r = (tid >> 3) & 15, s = tid & 7;
  double* const lrow = &sm.blk[0][0] + r * 16 + ((s ^ (r & 7)) << 1);
  tc_d2 v[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    const int p = 2 * k + hi;
    if (p < nblk) {
      int bi = 0;
#pragma unroll
      for (int q = 1; q < 8; ++q) bi += p >= q * (q + 1) / 2;
      const int bj = p - bi * (bi + 1) / 2;
      const int R = 16 * bi + r, C = 16 * bj + 2 * s;
      double* g = D + (int64_t)R * lda + C;
      if (OUT) {
        if (R < td) {
          const tc_d2a16 x = *(const tc_d2a16*)(lrow + p * 256);
          if (C <= R) g[0] = x.x;
          if (C + 1 <= R) g[1] = x.y;
        }
      } else {
        v[k].x = (R < td && C <= R) ? g[0] : 0.0;
        v[k].y = (R < td && C + 1 <= R) ? g[1] : 0.0;
      }
    }
  }
  if (!OUT) {
#pragma unroll
    for (int k = 0; k < 18; ++k) {
      const int p = 2 * k + hi;
      if (p < nblk) {
        tc_d2a16 x;
        x.x = v[k].x;
        x.y = v[k].y;
        *(tc_d2a16*)(lrow + p * 256) = x;
      }
    }
  }
}

// Step 1 on diagonal block b (nb valid columns, column offset c0 in the
// tile) by the calling wave: factors the block in place, stages it packed in
// lt, and records the first failing pivot in fail.  Lane i < 16 holds row i.
// The 16 steps are free of branches, so the compiler can overlap a step's
// trailing update with the next pivot: entries above the diagonal are
// updated too (they never feed an entry on or below it and are never
// stored), columns past nb take a unit pivot, and after a failing pivot the
// values are unspecified.
__device__ __forceinline__ void tc_pk_diag(TcPotrfSmem& sm, int b, int nb, int c0) {
  const int lane = tc_tid() & 63;
  double* blk = sm.blk[tc_pk(b, b)];
  double a[16];
  tc_row_get(blk, lane & 15, 16, a);
  // the 16 steps form one branch-free block (selects only; lane j keeps its
  // pivot's reciprocal and stores it after the loop), so the scheduler can
  // run a step's remaining updates under the next pivot's square root
  int bad = -1;
  double myr = 1.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const bool live = j < nb;
    const double d = tc_readlane(a[j], j);
    bad = (bad < 0 && live && !(d > 0.0)) ? j : bad;
    const double ljj = sqrt(live ? d : 1.0);
    const double rj = tc_rcp(ljj);
    a[j] = lane == j ? ljj : a[j] * rj;
    myr = lane == j ? rj : myr;
    // trailing update a_ik -= l_ij l_kj for k > j
#pragma unroll
    for (int k = j + 1; k < 16; ++k) a[k] = __builtin_fma(-a[j], tc_readlane(a[j], k), a[k]);
  }
  if (lane == 0 && bad >= 0) sm.fail = c0 + bad;
  if (lane < 16) {
    sm.lt[tc_ltp(lane)] = myr;
#pragma unroll
    for (int k = 0; k < 15; ++k)
      if (k < lane) sm.lt[tc_ltp(k) + (lane - k)] = lane < nb ? a[k] : 0.0;
  }
  if (lane < nb) tc_row_put(blk, lane, 16, a);
}

__device__ __forceinline__ int tc_potrf_tile(double* __restrict__ D, int64_t lda, int td_in, TcPotrfSmem& sm) {
  const int td = tc_uniform((int32_t)td_in);
  const int tid = tc_tid(), lane = tid & 63, w = tid >> 6;
  const int wu = tc_uniform((int32_t)w);
  const int r16 = lane & 15, s4 = lane >> 4;
  const int nbk = (td + 15) >> 4;
  tc_pk_copy<false>(D, lda, td, sm);
  if (tid == 0) sm.fail = -1;
  __syncthreads();
  if (wu == 0) tc_pk_diag(sm, 0, td < 16 ? td : 16, 0);
  __syncthreads();
  int fail = tc_uniform((int32_t)sm.fail);
  for (int b = 0; fail < 0 && b + 1 < nbk; ++b) {
    // 2. the blocks below diagonal block b, one row per thread
    if (tid < td - 16 * (b + 1)) {
      double* blk = sm.blk[tc_pk(b + 1 + (tid >> 4), b)];
      double v[16];
      tc_row_get(blk, tid & 15, 16, v);
      tc_subst_row(v, sm.lt);
      tc_row_put(blk, tid & 15, 16, v);
    }
    __syncthreads();
    // 3. the trailing blocks, numbered u = ii (ii + 1) / 2 + jj for block
    //    (b + 1 + ii, b + 1 + jj), jj <= ii; u = 0 is the next diagonal block
    if (wu == 0) {
      double* cb = sm.blk[tc_pk(b + 1, b + 1)];
      const tc_q4 x = tc_frag_get(sm.blk[tc_pk(b + 1, b)], r16, s4, 16);
      tc_acc_put(cb, lane, 16, tc_nt16(x, x, tc_acc_get(cb, lane, 16)));
      tc_wave_sync();
      const int c1 = 16 * (b + 1);
      tc_pk_diag(sm, b + 1, td - c1 < 16 ? td - c1 : 16, c1);
    } else {
      // wave w takes u = w, w + 3, ..., four blocks at a time with their
      // MFMA chains interleaved
      const int m = nbk - 1 - b, cnt = m * (m + 1) / 2;
      for (int u0 = wu; u0 < cnt; u0 += 12) {
        int off[4];
        tc_q4 x[4], y[4];
        tc_v4d acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int u = u0 + 3 * q;
          int ii = 0;
#pragma unroll
          for (int t = 1; t < 7; ++t) ii += u >= t * (t + 1) / 2;
          const int i = b + 1 + ii, j = b + 1 + u - ii * (ii + 1) / 2;
          off[q] = tc_pk(i, j) * 256;
          if (u < cnt) {
            x[q] = tc_frag_get(sm.blk[tc_pk(i, b)], r16, s4, 16);
            y[q] = tc_frag_get(sm.blk[tc_pk(j, b)], r16, s4, 16);
            acc[q] = tc_acc_get(&sm.blk[0][0] + off[q], lane, 16);
          }
        }
#pragma unroll
        for (int mm = 0; mm < 4; ++mm)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (u0 + 3 * q < cnt) acc[q] = tc_mfma(-tc_el(x[q], mm), tc_el(y[q], mm), acc[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (u0 + 3 * q < cnt) tc_acc_put(&sm.blk[0][0] + off[q], lane, 16, acc[q]);
      }
    }
    __syncthreads();
    fail = tc_uniform((int32_t)sm.fail);
  }
  tc_pk_copy<true>(D, lda, td, sm);
  return fail;
}
