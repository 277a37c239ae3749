// batch_plan.h -- workspace layouts and the merged ticket order of the
// batched launch, plus the status header every factorization workspace
// starts with.  Plain C++ shared by the HIP launchers and by host-only
// builds (the CPU emulation of the dependency counters compiles this header
// with g++ and sanitizers); pure host arithmetic, no device calls.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "dag.h"

// Status header at the start of a factorization workspace (and one per
// matrix of a batched launch).
struct TcWsHeader {
  int32_t ticket;
  int32_t error;  // 0 ok, 1 not SPD, 2 dependency-wait timeout
  int64_t info;   // failing global column + 1, or 1 + the ticket that waited
  int32_t bar;    // arrivals at the grid barriers of the synchronous schedule
};

// Device addresses of one factorization's status and counters.
struct TcWs {
  TcWsHeader* hdr;
  int64_t* offs;
  int32_t* pdone;
  int32_t* ver;
  int32_t noop;  // measurement mode: run the schedule with empty unit bodies
};

inline int64_t tc_round256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// ---- batched launch
#define TC_UNIT_SOLVE 4

struct TcBatchMat {
  double* A;
  double* b;  // right-hand sides (n x nrhs row-major, leading dimension ldb) or null
  int64_t lda;
  int64_t nrhs, ldb;
  TcGeom g;
  TcWs ws;        // per-matrix status header and counters
  int32_t* done;  // factor units finished
  int64_t nunits;
  // FP32 trailing products (prec 1): P holds every finished panel row of the
  // factor rounded once to FP32 (row r, column c at P[r * ldp + c]); the
  // last TRSM of a row block in a tile column writes that row block's panel
  // strip, and the update units read their operands from it.
  int32_t prec, refine;
  float* P;
  int64_t ldp;
  // Refinement of the solve (refine != 0, one right-hand side): the original
  // matrix A0 (lower triangle, lda0) and right-hand side b0 stay untouched;
  // the solve unit iterates x += (L L^T)^-1 (b0 - A0 x) until the backward
  // error is <= tol or max_iter corrections are applied, using R (n
  // doubles) as scratch, and writes {eta, corrections} to stat.
  const double* A0;
  int64_t lda0;
  const double* b0;
  double* R;
  double* stat;
  double tol;
  int64_t max_iter;
};
struct TcBatchUnit {
  int32_t m, kind, J, I, a, K, b, pad;
};
struct TcBatchSlot {
  int32_t m, P;   // P < 0: the solve unit
  int64_t start;  // first global ticket
  int64_t pos;    // first position inside phase P of matrix m
  int64_t size;
};

// Workspace of a batched launch (each part 256-byte aligned):
//   ticket | per-matrix status headers | done counters | per-matrix pdone and
//   ver counters (all zeroed by one fill) | descriptors | slots | unit table |
//   refinement statistics {eta, corrections} per matrix (with refinement) |
//   per matrix: FP32 panel copy (FP32 products), refinement scratch vector
struct TcBatchLayout {
  int64_t hdrs, done, counters, zero_end, mats, slots, table, stats, extra, total_bytes;
  int64_t nslots, nunits;
};

// Leading dimension (floats) of an FP32 panel copy of order n.
inline int64_t tc_batch_ldp(int64_t n) { return (n + 63) & ~(int64_t)63; }
// Per-matrix bytes after the statistics: the FP32 panel copy (prec 1, more
// than one tile) and, with refinement, the scratch vector.
inline int64_t tc_batch_extra_bytes(const TcGeom& g, int32_t prec, bool refine) {
  int64_t b = 0;
  if (prec == 1 && g.M > 1) b += tc_round256(4 * g.n * tc_batch_ldp(g.n));
  if (refine) b += tc_round256(8 * g.n);
  return b;
}

inline int64_t tc_ctr_bytes(const TcGeom& g) {
  return tc_round256(4 * (int64_t)g.NRB) + tc_round256(4 * (int64_t)g.NRB * g.NRB);
}

// Layout for `batch` matrices of orders n[i] (n[i] <= 0 skipped) and tile
// sides T[i]; geoms (if given, sized batch) receives each matrix's geometry.
// prec: per-matrix precision of the trailing products (null: all FP64);
// refine: the solve units refine against the original matrices.
inline TcBatchLayout tc_batch_layout(int64_t batch, const int64_t* n, const int64_t* T, bool solve, int64_t chunk,
                                     std::vector<TcGeom>* geoms, const int32_t* prec = nullptr, bool refine = false) {
  TcBatchLayout L{};
  int64_t ctr = 0, units = 0, slots = 0, extra = 0;
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] <= 0) continue;
    const TcGeom g = tc_geom(n[i], T[i], chunk);
    if (geoms) (*geoms)[i] = g;
    ctr += tc_ctr_bytes(g);
    extra += tc_batch_extra_bytes(g, prec ? prec[i] : 0, refine);
    for (int32_t P = 0; P < g.M; ++P) {
      units += tc_phase_size(g, P);
      slots += tc_phase_segments(g, P, nullptr);
    }
    if (solve) {
      units += 1;
      slots += 1;
    }
  }
  L.hdrs = 256;
  L.done = L.hdrs + tc_round256((int64_t)sizeof(TcWsHeader) * batch);
  L.counters = L.done + tc_round256(4 * batch);
  L.zero_end = L.counters + ctr;
  L.mats = L.zero_end;
  L.slots = L.mats + tc_round256((int64_t)sizeof(TcBatchMat) * batch);
  L.table = L.slots + tc_round256((int64_t)sizeof(TcBatchSlot) * slots);
  L.stats = L.table + tc_round256((int64_t)sizeof(TcBatchUnit) * units);
  L.extra = L.stats + (refine ? tc_round256(16 * batch) : 0);
  L.total_bytes = L.extra + extra;
  L.nslots = slots;
  L.nunits = units;
  return L;
}

// The merged ticket order of the batched launch: segment k of phase P of
// every matrix that has one, largest matrix first, for (P, k) in order (the
// segments of dag.h: the column updates that open the phase, each panel
// sub-column's POTRF, TRSM column and panel updates, each followed by its
// lookahead chunk of bulk updates, then the rest of the bulk), and each
// matrix's solve unit (when `solve`) right after its last segment.  Every
// matrix's own units keep their single-matrix ticket order, so a unit waits
// only on smaller tickets of its own matrix.  Empty segments take no slot.
// Returns the number of tickets.
inline int64_t tc_batch_slots(int64_t batch, const int64_t* n, const std::vector<TcGeom>& geoms, bool solve,
                              std::vector<TcBatchSlot>& slots) {
  slots.clear();
  std::vector<int64_t> order;
  int32_t maxM = 0;
  for (int64_t i = 0; i < batch; ++i)
    if (n[i] > 0) {
      order.push_back(i);
      maxM = std::max(maxM, geoms[i].M);
    }
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return n[x] > n[y]; });
  int64_t start = 0;
  std::vector<int64_t> live, segs, segoff, pos;
  for (int32_t P = 0; P < maxM; ++P) {
    live.clear();
    segoff.clear();
    segs.clear();
    int64_t kmax = 0;
    for (int64_t i : order) {
      if (P >= geoms[i].M) continue;
      const int64_t ns = tc_phase_segments(geoms[i], P, nullptr);
      live.push_back(i);
      segoff.push_back((int64_t)segs.size());
      segs.resize(segs.size() + ns);
      tc_phase_segments(geoms[i], P, segs.data() + segoff.back());
      kmax = std::max(kmax, ns);
    }
    segoff.push_back((int64_t)segs.size());
    pos.assign(live.size(), 0);
    for (int64_t k = 0; k < kmax; ++k) {
      for (size_t q = 0; q < live.size(); ++q) {
        const int64_t i = live[q];
        const int64_t nseg = segoff[q + 1] - segoff[q];
        if (k >= nseg) continue;
        const int64_t sz = segs[segoff[q] + k];
        if (sz > 0) {
          slots.push_back({(int32_t)i, P, start, pos[q], sz});
          start += sz;
          pos[q] += sz;
        }
        if (solve && P == geoms[i].M - 1 && k == nseg - 1) {
          slots.push_back({(int32_t)i, -1, start, 0, 1});
          start += 1;
        }
      }
    }
  }
  return start;
}

// Unit at ticket position r of a slot (what the device-side table expansion
// writes for it).
TC_HD TcBatchUnit tc_batch_slot_unit(const TcBatchSlot& sl, const TcGeom& g, int64_t r) {
  if (sl.P < 0) return {sl.m, TC_UNIT_SOLVE, 0, 0, 0, 0, 0, 0};
  const TcUnit u = tc_decode_in_phase(g, sl.P, sl.pos + r);
  return {sl.m, u.kind, u.J, u.I, u.a, u.K, u.b, 0};
}
