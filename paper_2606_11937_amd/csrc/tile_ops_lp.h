// tile_ops_lp.h -- the trailing-update tile operation (SYRK / GEMM of Methods,
// "Tiled Cholesky Decomposition") with low-precision products:
//
//   C[r][c] -= sum_{t < kd} PA[r][t] * PB[c][t]     0 <= r < mr, 0 <= c < mc
//
// where PA, PB are the panel entries rounded once to FP32 or BF16 (a copy of
// the panel kept beside the FP64 factor), every product entry is summed in
// FP32 by the matrix cores, and the sum is subtracted from FP64 C.  POTRF and
// TRSM stay in FP64 (tile_ops.h); only this operation, which carries almost
// all of the flops, changes precision.
//
// Matrix cores:
//   FP32:  v_mfma_f32_16x16x4_f32   (A, B: one float per lane)
//   BF16:  v_mfma_f32_16x16x32_bf16 (A, B: eight bf16 per lane)
// Output layout of both (FP32 accumulators): lane l, item q holds
// D[4 (l / 16) + q][l % 16], four consecutive rows per lane; the FP64 core
// interleaves them instead (D[4 q + l / 16][l % 16]).
// A lane with row index l % 16 and k group l / 16 supplies the same k
// positions of its row for both operands, so each MFMA sums matching k of
// row r of PA and row c of PB, whatever the order of k inside the group.
//
// Staging is byte-for-byte the FP64 kernel's: 128-byte k chunks of each of
// 128 operand rows (32 FP32 or 64 BF16 values), direct-to-LDS buffer loads of
// 16 bytes per lane into XOR-swizzled slots, two stages, fragments rolled
// half a chunk ahead, one plain barrier per chunk.  A lane's 16-byte
// fragment (slot 2 s + h of its row) feeds four FP32 MFMAs or one BF16 MFMA.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tile_ops.h"

#define TC_PREC_FP64 0
#define TC_PREC_FP32 1
#define TC_PREC_BF16 2

typedef float tc_v4f __attribute__((ext_vector_type(4)));
typedef __bf16 tc_v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t tc_u4 __attribute__((ext_vector_type(4), aligned(16)));

template <int PREC>
struct TcLp;
template <>
struct TcLp<TC_PREC_FP32> {
  typedef float elem;
  static constexpr int kChunk = 32;  // k values per 128-byte row chunk
};
template <>
struct TcLp<TC_PREC_BF16> {
  typedef uint16_t elem;  // bf16 bit pattern
  static constexpr int kChunk = 64;
};

// ---------------------------------------------------------------- rounding
// FP64 -> FP32, round to nearest even (the conversion's default mode).
__device__ __forceinline__ float tc_to_fp32(double x) { return (float)x; }

// FP64 -> BF16 bit pattern, round to nearest even, without double rounding:
// first to FP32 rounding to odd (truncate toward zero, set the last bit if
// anything was lost), then to the upper 16 bits with round to nearest even
// (add 0x7FFF plus the lowest kept bit, drop the low half).  Rounding to odd
// at a width at least two bits above the target makes the second rounding
// correct (Boldo and Melquiond, 2008).
__device__ __forceinline__ uint16_t tc_to_bf16(double x) {
  float f = (float)x;
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if (fabs((double)f) > fabs(x)) u -= 1;  // one step back toward zero
  if ((double)__builtin_bit_cast(float, u) != x) u |= 1u;
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int PREC>
__device__ __forceinline__ typename TcLp<PREC>::elem tc_round_lp(double x);
template <>
__device__ __forceinline__ float tc_round_lp<TC_PREC_FP32>(double x) {
  return tc_to_fp32(x);
}
template <>
__device__ __forceinline__ uint16_t tc_round_lp<TC_PREC_BF16>(double x) {
  return tc_to_bf16(x);
}

// ------------------------------------------------------------ the MFMAs
// acc += (fragment a) x (fragment b) over the k positions the two 16-byte
// fragments hold.
template <int PREC>
__device__ __forceinline__ tc_v4f tc_mfma_lp(const tc_u4& a, const tc_u4& b, tc_v4f c);
template <>
__device__ __forceinline__ tc_v4f tc_mfma_lp<TC_PREC_FP32>(const tc_u4& a, const tc_u4& b, tc_v4f c) {
  // reinterpret the whole 16-byte fragment (a bit cast of a single vector
  // element is not used: it is easy to get wrong and gains nothing)
  const tc_v4f af = __builtin_bit_cast(tc_v4f, a), bf = __builtin_bit_cast(tc_v4f, b);
#pragma unroll
  for (int e = 0; e < 4; ++e) c = __builtin_amdgcn_mfma_f32_16x16x4f32(af[e], bf[e], c, 0, 0, 0);
  return c;
}
template <>
__device__ __forceinline__ tc_v4f tc_mfma_lp<TC_PREC_BF16>(const tc_u4& a, const tc_u4& b, tc_v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(tc_v8bf, a), __builtin_bit_cast(tc_v8bf, b), c,
                                                 0, 0, 0);
}

// ------------------------------------------------------------ the tile op
// Same contract as tc_update_block with PA, PB low-precision rows of leading
// dimension ldp (elements); mr, mc <= 128.  The shared memory is the FP64
// kernel's (the same 128 x 128-byte stage layout).
template <int PREC>
__device__ __forceinline__ void tc_update_block_lp(double* __restrict__ C, const typename TcLp<PREC>::elem* __restrict__ PA,
                                                   const typename TcLp<PREC>::elem* __restrict__ PB, int64_t lda,
                                                   int64_t ldp, int mr, int mc, int kd, bool diag, TcUpdSmem& sm) {
  typedef typename TcLp<PREC>::elem E;
  constexpr int KC = TcLp<PREC>::kChunk;
  constexpr int EPS = 16 / (int)sizeof(E);  // elements per 16-byte slot
  const int tid = tc_tid();
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  const bool active = !(diag && wn > wm) && wm * 64 < mr && wn * 64 < mc;
  const int r16 = lane & 15, s2 = (lane >> 4) * 2;
  char* const lds = (char*)&sm.tile[0][0][0];  // [stage][A|B][row][128 bytes]

  // operand, row count and LDS window as scalars (see tc_update_block)
  const int ws = tc_uniform((int32_t)w);
  const int nrow = ws < 2 ? tc_uniform((int32_t)mr) : tc_uniform((int32_t)mc);
  const int64_t rowb = tc_uniform(ldp) * (int64_t)sizeof(E);  // operand row stride in bytes
  const E* src = (const E*)tc_uniform((int64_t)(ws < 2 ? PA : PB));
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      (void*)src, (short)0, (int)((int64_t)nrow * rowb), 0x00020000);
  const int rl0 = (w & 1) * 64 + (lane >> 3);
  const unsigned vof0 = (unsigned)(rl0 * rowb + 16 * ((lane & 7) ^ tc_swz(rl0)));
  const unsigned rowstep = (unsigned)(8 * rowb);
  auto stage_load = [&](int st, int k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsrc, (tc_lds_void*)((char __attribute__((address_space(3)))*)(tc_lds_void*)lds + st * 32768 + (ws * 8 + q) * 1024),
          16, vof0 + q * rowstep, (unsigned)(k0 * (int)sizeof(E)), 0, 0);
  };
  // the ragged last chunk: guarded element loads, zero past kd or past the
  // block's rows, stored where the direct loads would put them
  auto stage_tail = [&](int st, int k0) {
    const E* gb = w < 2 ? PA : PB;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int r = rl0 + q * 8;
      const int j = (lane & 7) ^ tc_swz(r);
      const int k = k0 + EPS * j;
      const E* src = gb + (int64_t)(r < nrow ? r : 0) * ldp + k;
      E v[EPS];
#pragma unroll
      for (int e = 0; e < EPS; ++e) v[e] = (r < nrow && k + e < kd) ? src[e] : (E)0;
      tc_u4 pk;
      __builtin_memcpy(&pk, v, 16);
      *(tc_u4*)(lds + st * 32768 + ((w * 8 + q) * 64 + lane) * 16) = pk;
    }
  };
  auto stage = [&](int st, int c, int nfull) {
    if (c < nfull) stage_load(st, c * KC); else stage_tail(st, c * KC);
  };
  // 16-byte fragment: half h (slot s2 + h) of row-block i of operand t
  auto rd = [&](int st, int t, int i, int h) -> tc_u4 {
    const int r = (t == 0 ? wm : wn) * 64 + i * 16 + r16;
    return *(const tc_u4*)(lds + st * 32768 + t * 16384 + r * 128 + 16 * ((s2 + h) ^ tc_swz(r)));
  };

  tc_v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = tc_v4f{0.f, 0.f, 0.f, 0.f};

  const int nfull = kd / KC;
  const int nch = (kd + KC - 1) / KC;
  tc_u4 La[4], Lb[4], Ha[4], Hb[4];
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
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = tc_mfma_lp<PREC>(La[i], Lb[j], acc[i][j]);
    }
    if (c + 1 < nch) {
      __builtin_amdgcn_s_waitcnt(0x0070);
      __builtin_amdgcn_s_barrier();
      if (c + 2 < nch) stage(st, c + 2, nfull);
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
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = tc_mfma_lp<PREC>(Ha[i], Hb[j], acc[i][j]);
    }
  }
  if (!active) return;

  // epilogue as in tc_update_block: each 16-row group of C is loaded ahead of
  // the previous group's stores (a ragged block from clamped positions, with
  // its stores guarded)
  const int orow = (lane >> 4) * 4, ocol = lane & 15;
  if (mr == 128 && mc == 128) {
    double* cb = C + (int64_t)(wm * 64 + orow) * lda + wn * 64 + ocol;
    double cv[2][16];
    auto cload = [&](double(&v)[16], int i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double* rp = cb + (int64_t)(i * 16 + q) * lda;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[4 * q + j] = rp[16 * j];
      }
    };
    auto cstore = [&](const double(&v)[16], int i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double* rp = cb + (int64_t)(i * 16 + q) * lda;
        const int r = wm * 64 + i * 16 + orow + q;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = wn * 64 + j * 16 + ocol;
          if (!diag || r >= c) rp[16 * j] = v[4 * q + j] - (double)acc[i][j][q];
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
    // ragged: loads from clamped (in-block) positions, stores guarded
    double cv[2][16];
    auto cload = [&](double(&v)[16], int i) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wm * 64 + i * 16 + orow + q;
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
        const int r = wm * 64 + i * 16 + orow + q;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = wn * 64 + j * 16 + ocol;
          if (r < mr && c < mc && (!diag || r >= c))
            C[(int64_t)r * lda + c] = v[4 * q + j] - (double)acc[i][j][q];
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
