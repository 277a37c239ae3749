// dag.h -- tile geometry, work units and dispatch order of the tiled
// right-looking Cholesky (Methods, Fig. 1 and the task graph of Fig. 3).
// Shared by the host (enumeration, workspace sizing) and the device
// (persistent-kernel ticket decoding); pure integer arithmetic, no memory.
//
// Tiles.  n is split into M = ceil(n/T) tile rows/columns; tile I spans rows
// [I*T, min(n, (I+1)*T)).  Each tile is further split into sub-blocks of
// TC_BLK rows; sub-block a of tile I has global row-block id g = I*SB + a.
//
// Work units (the pieces the schedules execute):
//   POTRF(J)              the whole diagonal tile J,
//   TRSM(I, J, a)         rows of sub-block a of tile I against L_JJ,
//   UPDATE(I, a, K, b, J) the TC_BLK x TC_BLK output block (a, b) of tile
//                         (I, K) at step J: SYRK when I == K (only b <= a),
//                         GEMM when I > K.
//
// Dispatch order of the asynchronous schedule.  Units are grouped in phases
// P = 0 .. M-1.  Phase P holds, in this order:
//   [col]   the step-(P-1) updates of tile column P (they feed POTRF(P)),
//   [potrf] POTRF(P),
//   [bulk1] the first Q step-(P-1) updates of the columns K > P,
//   [trsm]  TRSM(I, P, a) for I > P,
//   [bulk2] the remaining step-(P-1) updates of the columns K > P.
// Within [col] units go by tile row I, within the bulk by column K then row
// I, so tile column P+1 is updated first.  Every unit depends only on units
// of earlier phases or earlier segments (checked by enumeration tests), so
// ticket order is a topological order of the tile DAG and a worker that
// waits on a dependency always waits on a unit another running worker holds.
// Placing [potrf] and [trsm] ahead of the bulk update of the previous step
// is a one-step lookahead: the panel of step P is factored while the
// trailing update of step P-1 still runs, the GPU counterpart of removing
// the per-step barrier of the fork-join variants.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define TC_HD __host__ __device__ __forceinline__
#else
#define TC_HD inline
#endif

#define TC_BLK 128

enum { TC_UNIT_POTRF = 0, TC_UNIT_TRSM = 1, TC_UNIT_UPDATE = 2 };

struct TcGeom {
  int64_t n, T;
  int32_t M;    // tiles per dimension
  int32_t SB;   // sub-blocks of a full tile
  int32_t SBL;  // sub-blocks of the last tile
  int32_t NRB;  // total row blocks
  int64_t Q;    // bulk units placed ahead of each TRSM panel
};

struct TcUnit {
  int32_t kind, J, I, a, K, b;
};

TC_HD int64_t tc_cdiv(int64_t x, int64_t y) { return (x + y - 1) / y; }

TC_HD TcGeom tc_geom(int64_t n, int64_t T, int64_t Q) {
  TcGeom g;
  g.n = n;
  g.T = T;
  g.M = (int32_t)tc_cdiv(n, T);
  g.SB = (int32_t)tc_cdiv(T < n ? T : n, TC_BLK);
  int64_t tl = n - (int64_t)(g.M - 1) * T;
  g.SBL = (int32_t)tc_cdiv(tl, TC_BLK);
  g.NRB = (g.M - 1) * g.SB + g.SBL;
  g.Q = Q;
  return g;
}

// side of tile I and its sub-block count
TC_HD int64_t tc_tdim(const TcGeom& g, int32_t I) {
  int64_t r = g.n - (int64_t)I * g.T;
  return r < g.T ? r : g.T;
}
TC_HD int32_t tc_sb(const TcGeom& g, int32_t I) { return I == g.M - 1 ? g.SBL : g.SB; }
TC_HD int32_t tc_gid(const TcGeom& g, int32_t I, int32_t a) { return I * g.SB + a; }
// first row and row count of sub-block a of tile I
TC_HD int64_t tc_row0(const TcGeom& g, int32_t I, int32_t a) { return (int64_t)I * g.T + (int64_t)a * TC_BLK; }
TC_HD int32_t tc_rows(const TcGeom& g, int32_t I, int32_t a) {
  int64_t r = tc_tdim(g, I) - (int64_t)a * TC_BLK;
  return (int32_t)(r < TC_BLK ? r : TC_BLK);
}

// row blocks strictly below tile K
TC_HD int64_t tc_rows_below(const TcGeom& g, int32_t K) {
  if (K + 1 > g.M - 1) return 0;
  return (int64_t)(g.M - 2 - K) * g.SB + g.SBL;
}
// update units of tile column K for one step (SYRK on (K,K) + GEMMs below)
TC_HD int64_t tc_colsize(const TcGeom& g, int32_t K) {
  int64_t s = tc_sb(g, K);
  return s * (s + 1) / 2 + s * tc_rows_below(g, K);
}
// sum of tc_colsize over the first m columns K = P+1 .. P+m (all K <= M-2)
TC_HD int64_t tc_colsum(const TcGeom& g, int32_t P, int64_t m) {
  int64_t SB = g.SB;
  int64_t alpha = SB * (SB + 1) / 2 + SB * g.SBL;
  int64_t beta = SB * SB;
  return m * alpha + beta * (m * (int64_t)(g.M - 2 - P) - m * (m + 1) / 2);
}
// update units of one step over all tile columns K > P
TC_HD int64_t tc_trailing_units(const TcGeom& g, int32_t P) {
  if (P >= g.M - 1) return 0;
  int64_t m = (int64_t)(g.M - 2 - P);  // full columns P+1 .. M-2
  return tc_colsum(g, P, m) + tc_colsize(g, g.M - 1);
}
// all step-(P-1) update units of columns K > P (the bulk of phase P)
TC_HD int64_t tc_bulk(const TcGeom& g, int32_t P) { return P >= 1 ? tc_trailing_units(g, P) : 0; }

struct TcPhase {
  int64_t col, potrf, bulk1, trsm, bulk2;
};

TC_HD TcPhase tc_phase(const TcGeom& g, int32_t P) {
  TcPhase ph;
  ph.col = P >= 1 ? tc_colsize(g, P) : 0;
  ph.potrf = 1;
  int64_t bulk = tc_bulk(g, P);
  ph.bulk1 = bulk < g.Q ? bulk : g.Q;
  ph.bulk2 = bulk - ph.bulk1;
  ph.trsm = tc_rows_below(g, P);
  return ph;
}
TC_HD int64_t tc_phase_size(const TcGeom& g, int32_t P) {
  TcPhase ph = tc_phase(g, P);
  return ph.col + ph.potrf + ph.bulk1 + ph.trsm + ph.bulk2;
}

// r-th unit (step J) of tile column K: SYRK sub-blocks (a >= b) of (K, K)
// first, then tile rows I > K with sub-blocks (a, b) row-major.
TC_HD TcUnit tc_decode_col(const TcGeom& g, int32_t J, int32_t K, int64_t r) {
  TcUnit u;
  u.kind = TC_UNIT_UPDATE;
  u.J = J;
  u.K = K;
  int64_t sk = tc_sb(g, K);
  int64_t dk = sk * (sk + 1) / 2;
  if (r < dk) {
    int32_t a = 0;
    while ((int64_t)(a + 1) * (a + 2) / 2 <= r) ++a;
    u.I = K;
    u.a = a;
    u.b = (int32_t)(r - (int64_t)a * (a + 1) / 2);
  } else {
    r -= dk;
    int64_t per = (int64_t)g.SB * sk;
    u.I = K + 1 + (int32_t)(r / per);
    int64_t q = r % per;
    u.a = (int32_t)(q / sk);
    u.b = (int32_t)(q % sk);
  }
  return u;
}

// r-th update unit, labelled step J, over the tile columns K > P
// (column-major over K, then tile row, then sub-block).
TC_HD TcUnit tc_decode_trailing(const TcGeom& g, int32_t P, int32_t J, int64_t r) {
  // largest m in [0, M-2-P] with colsum(m) <= r  (columns P+1 .. P+m full)
  int64_t lo = 0, hi = (int64_t)(g.M - 2 - P);
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    if (tc_colsum(g, P, mid) <= r) lo = mid; else hi = mid - 1;
  }
  int32_t K = P + 1 + (int32_t)lo;
  return tc_decode_col(g, J, K, r - tc_colsum(g, P, lo));
}
TC_HD TcUnit tc_decode_bulk(const TcGeom& g, int32_t P, int64_t r) { return tc_decode_trailing(g, P, P - 1, r); }

// Unit at position r within phase P.
TC_HD TcUnit tc_decode_in_phase(const TcGeom& g, int32_t P, int64_t r) {
  TcPhase ph = tc_phase(g, P);
  if (r < ph.col) return tc_decode_col(g, P - 1, P, r);
  r -= ph.col;
  if (r < 1) {
    TcUnit u;
    u.kind = TC_UNIT_POTRF; u.J = P; u.I = P; u.a = -1; u.K = -1; u.b = -1;
    return u;
  }
  r -= 1;
  if (r < ph.bulk1) return tc_decode_bulk(g, P, r);
  r -= ph.bulk1;
  if (r < ph.trsm) {
    TcUnit u;
    u.kind = TC_UNIT_TRSM;
    u.J = P;
    u.I = P + 1 + (int32_t)(r / g.SB);
    u.a = (int32_t)(r % g.SB);
    u.K = -1;
    u.b = -1;
    return u;
  }
  r -= ph.trsm;
  return tc_decode_bulk(g, P, ph.bulk1 + r);
}

// Tile-task counts (Results, problem-size scaling: M POTRF, M(M-1)/2 TRSM
// and SYRK, M(M-1)(M-2)/6 GEMM).
TC_HD void tc_task_counts(const TcGeom& g, int64_t c[4]) {
  int64_t M = g.M;
  c[0] = M;
  c[1] = M * (M - 1) / 2;
  c[2] = M * (M - 1) / 2;
  c[3] = M * (M - 1) * (M - 2) / 6;
}

