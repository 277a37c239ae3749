// dag.h -- tile geometry, work units and dispatch order of the tiled
// right-looking Cholesky (Methods, Fig. 1 and the task graph of Fig. 3).
// Shared by the host (enumeration, workspace sizing) and the device
// (persistent-kernel ticket decoding); pure integer arithmetic, no memory.
//
// Tiles.  n is split into M = ceil(n/T) tile rows/columns; tile I spans rows
// [I*T, min(n, (I+1)*T)).  Each tile is further split into sub-blocks of
// TC_BLK rows; sub-block a of tile I has global block id g = I*SB + a, and
// the same ids number the block columns.
//
// Work units.  The panel of tile column J (its POTRF and TRSM tasks) is
// factored one TC_BLK-wide sub-column s at a time, the blocked form of the
// same operations; the trailing SYRK/GEMM update of step J keeps the full
// K-depth T:
//   POTRF(J, s)              the diagonal block gs = gid(J, s),
//   TRSM(J, s, r)            block (r, gs) against it, for every r > gs,
//   PANEL(J, s, r, s')       block (r, gid(J, s')) -= (r, gs) (gid(J,s'), gs)^T
//                            for s < s' and r >= gid(J, s') (the update of the
//                            panel's later sub-columns, K-depth TC_BLK),
//   UPDATE(J, r, c)          the TC_BLK x TC_BLK output block (r, c) of the
//                            step-J trailing update, c beyond tile J, r >= c:
//                            SYRK when r and c lie in one tile, else GEMM.
// A block receives its updates in a fixed order: the trailing updates of
// steps 0, 1, ... and then, inside its own panel, the panel updates of
// sub-columns 0, 1, ...; both schedules apply exactly these units in that
// order, so they produce the same bits.
//
// Dispatch order of the asynchronous schedule.  Units are grouped in phases
// P = 0 .. M-1.  Phase P holds, in this order:
//   [col]  the step-(P-1) updates of tile column P (they feed its panel),
//   then for each sub-column s of panel P the chain
//          POTRF(P, s) [chunk] TRSM(P, s, *) [chunk] PANEL(P, s, *) [chunk]
//   where every [chunk] is the next (up to) Q step-(P-1) updates of the
//   columns beyond tile P, and finally
//   [rest] the remaining step-(P-1) updates.
// Within [col] units go by tile row, within the bulk by column then row, so
// tile column P+1 is updated first.  Every unit depends only on units of
// earlier phases or earlier segments (checked by enumeration tests), so
// ticket order is a topological order and a worker that waits on a
// dependency always waits on a unit another running worker holds.  Threading
// the panel chain of step P through the bulk update of step P-1 is the
// lookahead that replaces the per-step barrier of the fork-join variants.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define TC_HD __host__ __device__ __forceinline__
#else
#define TC_HD inline
#endif

#define TC_BLK 128

// Bulk updates placed after each link of a panel chain.  By default half a
// unit per persistent workgroup (the fastest of 16 .. 512 per link measured
// on MI355X at n = 32768); `setting` >= 0 overrides it (0 puts each whole
// chain ahead of the bulk, a value at least the bulk size puts the bulk
// ahead of the chain, i.e. no lookahead).
TC_HD int64_t tc_lookahead_chunk(int64_t grid, int64_t setting) {
  if (setting >= 0) return setting;
  return grid > 1 ? grid / 2 : 128;
}

enum { TC_UNIT_POTRF = 0, TC_UNIT_TRSM = 1, TC_UNIT_UPDATE = 2, TC_UNIT_PANEL = 3 };

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

// ---- panel chain of tile column P (sub-columns s = 0 .. sb(P)-1)
// TRSM units of sub-column s: every global block below gid(P, s).
TC_HD int64_t tc_trsm_count(const TcGeom& g, int32_t P, int32_t s) {
  return (int64_t)g.NRB - tc_gid(g, P, s) - 1;
}
// PANEL units of sub-column s: for each later sub-column s' of the panel,
// every block row r >= gid(P, s').
TC_HD int64_t tc_panel_count(const TcGeom& g, int32_t P, int32_t s) {
  int64_t c = 0;
  for (int32_t t = s + 1; t < tc_sb(g, P); ++t) c += (int64_t)g.NRB - tc_gid(g, P, t);
  return c;
}
// global block id -> (tile, sub-block)
TC_HD void tc_split_gid(const TcGeom& g, int64_t r, int32_t& I, int32_t& a) {
  I = (int32_t)(r / g.SB);
  a = (int32_t)(r % g.SB);
}
TC_HD TcUnit tc_decode_trsm(const TcGeom& g, int32_t P, int32_t s, int64_t k) {
  TcUnit u;
  u.kind = TC_UNIT_TRSM;
  u.J = P;
  tc_split_gid(g, tc_gid(g, P, s) + 1 + k, u.I, u.a);
  u.K = s;
  u.b = -1;
  return u;
}
TC_HD TcUnit tc_decode_panel(const TcGeom& g, int32_t P, int32_t s, int64_t k) {
  TcUnit u;
  u.kind = TC_UNIT_PANEL;
  u.J = P;
  u.K = s;
  int32_t t = s + 1;
  for (;;) {
    const int64_t rows = (int64_t)g.NRB - tc_gid(g, P, t);
    if (k < rows || t + 1 >= tc_sb(g, P)) break;
    k -= rows;
    ++t;
  }
  u.b = t;
  tc_split_gid(g, tc_gid(g, P, t) + k, u.I, u.a);
  return u;
}
TC_HD TcUnit tc_decode_potrf(int32_t P, int32_t s) {
  TcUnit u;
  u.kind = TC_UNIT_POTRF;
  u.J = P;
  u.I = P;
  u.a = s;
  u.K = -1;
  u.b = -1;
  return u;
}
// units of the whole panel chain of P
TC_HD int64_t tc_chain_units(const TcGeom& g, int32_t P) {
  int64_t c = 0;
  for (int32_t s = 0; s < tc_sb(g, P); ++s) c += 1 + tc_trsm_count(g, P, s) + tc_panel_count(g, P, s);
  return c;
}

TC_HD int64_t tc_phase_size(const TcGeom& g, int32_t P) {
  return (P >= 1 ? tc_colsize(g, P) : 0) + tc_chain_units(g, P) + tc_bulk(g, P);
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
  const int64_t col = P >= 1 ? tc_colsize(g, P) : 0;
  if (r < col) return tc_decode_col(g, P - 1, P, r);
  r -= col;
  const int64_t bulk = tc_bulk(g, P);
  int64_t used = 0;  // bulk units placed so far
  for (int32_t s = 0; s < tc_sb(g, P); ++s) {
    for (int32_t link = 0; link < 3; ++link) {
      const int64_t sz = link == 0 ? 1 : link == 1 ? tc_trsm_count(g, P, s) : tc_panel_count(g, P, s);
      if (r < sz)
        return link == 0 ? tc_decode_potrf(P, s) : link == 1 ? tc_decode_trsm(g, P, s, r) : tc_decode_panel(g, P, s, r);
      r -= sz;
      const int64_t ch = bulk - used < g.Q ? bulk - used : g.Q;
      if (r < ch) return tc_decode_bulk(g, P, used + r);
      r -= ch;
      used += ch;
    }
  }
  return tc_decode_bulk(g, P, used + r);
}

// Segments of phase P in ticket order (see tc_decode_in_phase): the column
// updates, then for each sub-column s its three chain links, each followed
// by its bulk chunk, then the rest of the bulk.  Writes the sizes to `sz`
// (if not null; some may be 0) and returns their number, 2 + 6 SB(P).
TC_HD int64_t tc_phase_segments(const TcGeom& g, int32_t P, int64_t* sz) {
  int64_t k = 0;
  if (sz) sz[k] = P >= 1 ? tc_colsize(g, P) : 0;
  ++k;
  const int64_t bulk = tc_bulk(g, P);
  int64_t used = 0;
  for (int32_t s = 0; s < tc_sb(g, P); ++s) {
    for (int32_t link = 0; link < 3; ++link) {
      if (sz) sz[k] = link == 0 ? 1 : link == 1 ? tc_trsm_count(g, P, s) : tc_panel_count(g, P, s);
      ++k;
      const int64_t ch = bulk - used < g.Q ? bulk - used : g.Q;
      if (sz) sz[k] = ch;
      ++k;
      used += ch;
    }
  }
  if (sz) sz[k] = bulk - used;
  ++k;
  return k;
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


// ---- dependency counters (the asynchronous schedule and the batched launch)
// pdone[r]     sub-columns of block row r finished (they finish in order:
//              the POTRF or TRSM of sub-column s is the (s+1)-th);
// ver[r][c]    updates applied to block (r, c): the trailing updates of
//              steps 0, 1, ... and then, inside its own panel, the panel
//              updates of sub-columns 0, 1, ....
// `ld(p)` reads a counter (an atomic load on the device, a plain read in the
// host emulation) and `add(p)` increments one.
template <typename Ld>
TC_HD bool tc_unit_ready_with(const TcGeom& g, const int32_t* pdone, const int32_t* ver, const TcUnit& u, Ld ld) {
  const int64_t NRB = g.NRB;
  if (u.kind == TC_UNIT_UPDATE) {
    const int32_t gi = tc_gid(g, u.I, u.a), gk = tc_gid(g, u.K, u.b);
    const int32_t need = tc_gid(g, u.J, 0) + tc_sb(g, u.J);  // whole panel J finished
    return ld(pdone + gi) >= need && ld(pdone + gk) >= need && ld(ver + gi * NRB + gk) >= u.J;
  }
  if (u.kind == TC_UNIT_PANEL) {
    const int32_t gs = tc_gid(g, u.J, u.K), gt = tc_gid(g, u.J, u.b), gi = tc_gid(g, u.I, u.a);
    return ld(pdone + gi) > gs && ld(pdone + gt) > gs && ld(ver + gi * NRB + gt) >= u.J + u.K;
  }
  if (u.kind == TC_UNIT_TRSM) {
    const int32_t gs = tc_gid(g, u.J, u.K), gi = tc_gid(g, u.I, u.a);
    return ld(pdone + gs) > gs && ld(ver + gi * NRB + gs) >= u.J + u.K;
  }
  const int32_t gs = tc_gid(g, u.J, u.a);
  return ld(ver + (int64_t)gs * NRB + gs) >= u.J + u.a;
}

template <typename Add>
TC_HD void tc_unit_publish_with(const TcGeom& g, int32_t* pdone, int32_t* ver, const TcUnit& u, Add add) {
  if (u.kind == TC_UNIT_UPDATE) {
    add(ver + (int64_t)tc_gid(g, u.I, u.a) * g.NRB + tc_gid(g, u.K, u.b));
  } else if (u.kind == TC_UNIT_PANEL) {
    add(ver + (int64_t)tc_gid(g, u.I, u.a) * g.NRB + tc_gid(g, u.J, u.b));
  } else if (u.kind == TC_UNIT_TRSM) {
    add(pdone + tc_gid(g, u.I, u.a));
  } else {
    add(pdone + tc_gid(g, u.J, u.a));
  }
}
