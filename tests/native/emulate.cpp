// emulate.cpp -- CPU emulation of the device-side dependency protocol of the
// batched launch and of the server's host bookkeeping.  Built with g++ and
// the address and undefined-behaviour sanitizers by tests/test_emulation.py.
//
//   emulate dag <seed> <cases>    random ticks of the serving workload and of
//                                 edge geometries: the workspace layout, the
//                                 merged ticket order and the counter
//                                 protocol (dag.h's readiness and publish
//                                 rules) under random completion orders
//                                 with 1 .. 512 workers
//   emulate serve <seed> <steps>  the server core (serve_core.h) with a fake
//                                 arena, clock and device results
//
// The dependency model here is independent of dag.h: every unit's blocks
// read and written, in the blocked program order of the tiled algorithm
// (for each step J and panel sub-column s: POTRF, the TRSMs below it, the
// panel updates of the later sub-columns; then the trailing update), give
// each unit the set of earlier units it conflicts with.  A unit that the
// counters let start before all of them have finished is a failure, and so
// is a state where every worker waits and none can start (deadlock).
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <random>
#include <set>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "batch_plan.h"
#include "serve_core.h"
#include "tuned_tiles.h"

static int g_fail = 0;
#define CHECK(c, ...)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      fprintf(stdout, "FAIL %s:%d ", __FILE__, __LINE__); \
      fprintf(stdout, __VA_ARGS__);                     \
      fprintf(stdout, "\n");                            \
      g_fail = 1;                                       \
      return false;                                     \
    }                                                   \
  } while (0)

// ---------------------------------------------------------------- DAG model
namespace {
typedef std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t, int32_t> Key;
Key key_of(const TcUnit& u) { return Key(u.kind, u.J, u.I, u.a, u.K, u.b); }

struct Model {
  std::vector<TcUnit> prog;                  // units in program order
  std::map<Key, int64_t> index;              // unit -> program index
  std::vector<std::vector<int64_t>> preds;   // conflicting earlier units
};

// Blocks read (R) and written (W) by a unit, as global (row, column) block ids.
void access(const TcGeom& g, const TcUnit& u, std::vector<std::pair<int64_t, int64_t>>& R,
            std::vector<std::pair<int64_t, int64_t>>& W) {
  R.clear();
  W.clear();
  auto gid = [&](int32_t I, int32_t a) { return (int64_t)I * g.SB + a; };
  if (u.kind == TC_UNIT_POTRF) {
    const int64_t d = gid(u.J, u.a);
    R.push_back({d, d});
    W.push_back({d, d});
  } else if (u.kind == TC_UNIT_TRSM) {
    const int64_t d = gid(u.J, u.K), r = gid(u.I, u.a);
    R.push_back({d, d});
    R.push_back({r, d});
    W.push_back({r, d});
  } else if (u.kind == TC_UNIT_PANEL) {
    const int64_t s = gid(u.J, u.K), t = gid(u.J, u.b), r = gid(u.I, u.a);
    R.push_back({r, s});
    R.push_back({t, s});
    R.push_back({r, t});
    W.push_back({r, t});
  } else {
    const int64_t r = gid(u.I, u.a), c = gid(u.K, u.b);
    for (int32_t s = 0; s < tc_sb(g, u.J); ++s) {
      R.push_back({r, gid(u.J, s)});
      R.push_back({c, gid(u.J, s)});
    }
    R.push_back({r, c});
    W.push_back({r, c});
  }
}

// The blocked program order, written from the algorithm (not from dag.h's
// decoders): the panel of tile column J one 128-wide sub-column at a time,
// then the trailing update of every block (r, c), c beyond tile J, r >= c.
Model build_model(const TcGeom& g) {
  Model m;
  std::vector<int64_t> tile_of_block, sub_of_block;
  for (int32_t I = 0; I < g.M; ++I)
    for (int32_t a = 0; a < tc_sb(g, I); ++a) {
      tile_of_block.push_back(I);
      sub_of_block.push_back(a);
    }
  const int64_t NRB = (int64_t)tile_of_block.size();
  auto gid = [&](int32_t I, int32_t a) { return (int64_t)I * g.SB + a; };
  for (int32_t J = 0; J < g.M; ++J) {
    const int32_t sbJ = tc_sb(g, J);
    for (int32_t s = 0; s < sbJ; ++s) {
      m.prog.push_back({TC_UNIT_POTRF, J, J, s, -1, -1});
      for (int64_t r = gid(J, s) + 1; r < NRB; ++r)
        m.prog.push_back({TC_UNIT_TRSM, J, (int32_t)tile_of_block[r], (int32_t)sub_of_block[r], s, -1});
      for (int32_t t = s + 1; t < sbJ; ++t)
        for (int64_t r = gid(J, t); r < NRB; ++r)
          m.prog.push_back({TC_UNIT_PANEL, J, (int32_t)tile_of_block[r], (int32_t)sub_of_block[r], s, t});
    }
    for (int64_t c = gid(J + 1, 0); c < NRB; ++c)
      for (int64_t r = c; r < NRB; ++r)
        m.prog.push_back({TC_UNIT_UPDATE, J, (int32_t)tile_of_block[r], (int32_t)sub_of_block[r],
                          (int32_t)tile_of_block[c], (int32_t)sub_of_block[c]});
  }
  std::map<std::pair<int64_t, int64_t>, std::pair<int64_t, std::vector<int64_t>>> st;  // last writer, readers since
  std::vector<std::pair<int64_t, int64_t>> R, W;
  m.preds.resize(m.prog.size());
  for (int64_t k = 0; k < (int64_t)m.prog.size(); ++k) {
    m.index[key_of(m.prog[k])] = k;
    access(g, m.prog[k], R, W);
    std::set<int64_t> p;
    for (auto& b : R) {
      auto it = st.find(b);
      if (it != st.end() && it->second.first >= 0) p.insert(it->second.first);
    }
    for (auto& b : W) {
      auto it = st.find(b);
      if (it != st.end()) {
        if (it->second.first >= 0) p.insert(it->second.first);
        for (int64_t rd : it->second.second) p.insert(rd);
      }
    }
    p.erase(k);
    m.preds[k].assign(p.begin(), p.end());
    for (auto& b : R) {
      auto& e = st.emplace(b, std::make_pair((int64_t)-1, std::vector<int64_t>())).first->second;
      e.second.push_back(k);
    }
    for (auto& b : W) {
      auto& e = st[b];
      e.first = k;
      e.second.clear();
    }
  }
  return m;
}

// Emulate one batched launch: tickets in order, `workers` persistent
// workers, completions in random order.
bool emulate_tick(const std::vector<int64_t>& n, const std::vector<int64_t>& T, int64_t chunk, int workers,
                  bool solve, std::mt19937_64& rng) {
  const int64_t batch = (int64_t)n.size();
  std::vector<TcGeom> geoms(batch);
  const TcBatchLayout L = tc_batch_layout(batch, n.data(), T.data(), solve, chunk, &geoms);
  // ---- layout: ordered, aligned, disjoint
  const int64_t parts[] = {0, L.hdrs, L.done, L.counters, L.zero_end, L.mats, L.slots, L.table, L.stats, L.extra,
                           L.total_bytes};
  for (size_t k = 1; k < sizeof(parts) / sizeof(parts[0]); ++k) {
    CHECK(parts[k] >= parts[k - 1], "layout part %zu before part %zu", k, k - 1);
    CHECK(parts[k] % 256 == 0, "layout part %zu not 256-aligned", k);
  }
  CHECK(L.hdrs + (int64_t)sizeof(TcWsHeader) * batch <= L.done, "status headers overflow");
  CHECK(L.done + 4 * batch <= L.counters, "done counters overflow");
  int64_t ctr = L.counters;
  for (int64_t i = 0; i < batch; ++i)
    if (n[i] > 0) ctr += tc_ctr_bytes(geoms[i]);
  CHECK(ctr == L.zero_end, "counter regions do not tile the zeroed part");
  // ---- the merged order
  std::vector<TcBatchSlot> slots;
  const int64_t total = tc_batch_slots(batch, n.data(), geoms, solve, slots);
  CHECK(total == L.nunits, "tickets %lld != units %lld", (long long)total, (long long)L.nunits);
  CHECK((int64_t)slots.size() <= L.nslots, "slots overflow");
  std::vector<TcBatchUnit> table(total);
  int64_t next = 0;
  for (const TcBatchSlot& sl : slots) {
    CHECK(sl.start == next, "slot start %lld != %lld", (long long)sl.start, (long long)next);
    for (int64_t r = 0; r < sl.size; ++r) table[sl.start + r] = tc_batch_slot_unit(sl, geoms[sl.m], r);
    next += sl.size;
  }
  // each matrix's units in its single-matrix ticket order, every unit once
  std::vector<Model> models(batch);
  std::vector<std::vector<int64_t>> own(batch);
  for (int64_t t = 0; t < total; ++t) own[table[t].m].push_back(t);
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] <= 0) continue;
    const TcGeom& g = geoms[i];
    models[i] = build_model(g);
    int64_t k = 0;
    for (int32_t P = 0; P < g.M; ++P)
      for (int64_t r = 0; r < tc_phase_size(g, P); ++r, ++k) {
        CHECK(k < (int64_t)own[i].size(), "matrix %lld has too few tickets", (long long)i);
        const TcBatchUnit& e = table[own[i][k]];
        const TcUnit u = tc_decode_in_phase(g, P, r);
        CHECK(e.kind == u.kind && e.J == u.J && e.I == u.I && e.a == u.a && e.K == u.K && e.b == u.b,
              "matrix %lld ticket %lld differs from its own order", (long long)i, (long long)k);
      }
    CHECK(k == (int64_t)models[i].prog.size(), "matrix %lld: %lld tickets for %zu units", (long long)i,
          (long long)k, models[i].prog.size());
    if (solve) {
      CHECK((int64_t)own[i].size() == k + 1 && table[own[i][k]].kind == TC_UNIT_SOLVE,
            "matrix %lld: solve unit missing or misplaced", (long long)i);
    } else {
      CHECK((int64_t)own[i].size() == k, "matrix %lld: extra tickets", (long long)i);
    }
  }
  // ---- counters and the emulated grid
  std::vector<std::vector<int32_t>> pdone(batch), ver(batch);
  std::vector<int32_t> done(batch, 0);
  std::vector<std::vector<char>> finished(batch);
  std::vector<int64_t> nunits(batch, 0);
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] <= 0) continue;
    pdone[i].assign(geoms[i].NRB, 0);
    ver[i].assign((size_t)geoms[i].NRB * geoms[i].NRB, 0);
    finished[i].assign(models[i].prog.size(), 0);
    nunits[i] = (int64_t)models[i].prog.size();
  }
  auto ld = [](const int32_t* p) { return *p; };
  auto add = [](int32_t* p) { *p += 1; };
  struct W {
    int64_t ticket = -1;
    int state = 0;  // 0 idle, 1 waiting, 2 running
  };
  std::vector<W> w(workers);
  int64_t next_ticket = 0, completed = 0;
  auto ready = [&](int64_t t) {
    const TcBatchUnit& e = table[t];
    if (e.kind == TC_UNIT_SOLVE) return done[e.m] >= nunits[e.m];
    const TcUnit u = {e.kind, e.J, e.I, e.a, e.K, e.b};
    return tc_unit_ready_with(geoms[e.m], pdone[e.m].data(), ver[e.m].data(), u, ld);
  };
  std::vector<int> running;
  while (completed < total) {
    // idle workers take tickets; waiting workers start what is ready
    for (int k = 0; k < workers; ++k) {
      if (w[k].state == 0 && next_ticket < total) {
        w[k].ticket = next_ticket++;
        w[k].state = 1;
      }
      if (w[k].state == 1 && ready(w[k].ticket)) {
        const TcBatchUnit& e = table[w[k].ticket];
        if (e.kind == TC_UNIT_SOLVE) {
          for (char f : finished[e.m]) CHECK(f, "solve unit of matrix %d started early", e.m);
        } else {
          const TcUnit u = {e.kind, e.J, e.I, e.a, e.K, e.b};
          const int64_t pi = models[e.m].index.at(key_of(u));
          for (int64_t p : models[e.m].preds[pi])
            CHECK(finished[e.m][p], "matrix %d unit (%d,%d,%d,%d,%d,%d) started before its predecessor %lld",
                  e.m, u.kind, u.J, u.I, u.a, u.K, u.b, (long long)p);
        }
        w[k].state = 2;
        running.push_back(k);
      }
    }
    CHECK(!running.empty(), "deadlock: %lld of %lld units finished, no worker can start", (long long)completed,
          (long long)total);
    // one running unit finishes (random order) and publishes
    const size_t pick = rng() % running.size();
    const int k = running[pick];
    running[pick] = running.back();
    running.pop_back();
    const TcBatchUnit& e = table[w[k].ticket];
    if (e.kind != TC_UNIT_SOLVE) {
      const TcUnit u = {e.kind, e.J, e.I, e.a, e.K, e.b};
      tc_unit_publish_with(geoms[e.m], pdone[e.m].data(), ver[e.m].data(), u, add);
      finished[e.m][models[e.m].index.at(key_of(u))] = 1;
      done[e.m] += 1;
    }
    w[k].state = 0;
    ++completed;
  }
  // every counter at its final value
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] <= 0) continue;
    CHECK(done[i] == nunits[i], "matrix %lld: %d of %lld units published", (long long)i, done[i],
          (long long)nunits[i]);
    for (int32_t r = 0; r < geoms[i].NRB; ++r) {
      CHECK(pdone[i][r] == r + 1, "matrix %lld block row %d: pdone %d", (long long)i, r, pdone[i][r]);
    }
  }
  return true;
}

int64_t log_uniform(std::mt19937_64& rng, double lo, double hi) {
  std::uniform_real_distribution<double> u(std::log(lo), std::log(hi));
  return (int64_t)std::llround(std::exp(u(rng)));
}

int run_dag(uint64_t seed, int cases) {
  std::mt19937_64 rng(seed);
  int done = 0;
  const int grids[] = {1, 8, 64, 512};
  for (int c = 0; c < cases && !g_fail; ++c) {
    std::vector<int64_t> n, T;
    const int kind = c % 3;
    if (kind == 0) {  // a serving tick: orders log-uniform in [64, 8192], the tuned tiles
      const int m = 1 + (int)(rng() % 12);
      for (int i = 0; i < m; ++i) {
        const int64_t ni = log_uniform(rng, 64, c % 6 == 0 ? 8192 : 2048);
        const int prec = (int)(rng() % 2);
        n.push_back(ni);
        T.push_back(tc_tuned_batched_tile_prec(ni, prec));
      }
    } else if (kind == 1) {  // edge geometries: ragged tiles, tiles below a block, one tile
      const int64_t edges[][2] = {{1, 1},    {17, 8},   {129, 128}, {255, 100}, {300, 64},  {383, 128},
                                  {449, 256}, {513, 512}, {700, 96}, {1025, 1024}, {640, 1024}, {777, 256}};
      const int m = 1 + (int)(rng() % 5);
      for (int i = 0; i < m; ++i) {
        const auto& e = edges[rng() % (sizeof(edges) / sizeof(edges[0]))];
        n.push_back(e[0]);
        T.push_back(e[1]);
      }
      if (rng() % 3 == 0) {
        n.push_back(0);  // an empty member
        T.push_back(64);
      }
    } else {  // the batched workload's orders, log-uniform in [32, 2048]
      const int m = 1 + (int)(rng() % 24);
      for (int i = 0; i < m; ++i) {
        const int64_t ni = log_uniform(rng, 32, 2048);
        n.push_back(ni);
        T.push_back(tc_tuned_batched_tile(ni));
      }
    }
    const int grid = grids[rng() % 4];
    const int64_t chunk = tc_lookahead_chunk(grid, -1);
    const int workers = 1 + (int)(rng() % (grid > 64 ? 64 : grid)) + (grid == 512 ? 448 : 0);
    const bool solve = rng() % 2 == 0;
    if (!emulate_tick(n, T, chunk, workers, solve, rng)) {
      printf("case %d: %zu matrices, grid %d, %d workers, solve %d:", c, n.size(), grid, workers, (int)solve);
      for (size_t i = 0; i < n.size(); ++i) printf(" (%lld,%lld)", (long long)n[i], (long long)T[i]);
      printf("\n");
      return 1;
    }
    ++done;
  }
  printf("OK dag cases=%d\n", done);
  return g_fail;
}

// ---------------------------------------------------------------- server core
struct Region {
  int64_t off, bytes;
  std::string what;
};

bool disjoint(std::vector<Region> v, int64_t size, const char* arena) {
  std::sort(v.begin(), v.end(), [](const Region& a, const Region& b) { return a.off < b.off; });
  for (size_t k = 0; k < v.size(); ++k) {
    CHECK(v[k].off >= 0 && v[k].off % 256 == 0, "%s region %s at %lld", arena, v[k].what.c_str(),
          (long long)v[k].off);
    CHECK(v[k].off + tcs::r256(v[k].bytes) <= size, "%s region %s past the end", arena, v[k].what.c_str());
    if (k)
      CHECK(v[k - 1].off + tcs::r256(v[k - 1].bytes) <= v[k].off, "%s regions %s and %s overlap", arena,
            v[k - 1].what.c_str(), v[k].what.c_str());
  }
  return true;
}

int run_serve(uint64_t seed, int steps) {
  std::mt19937_64 rng(seed);
  for (int mode = 0; mode < 2 && !g_fail; ++mode) {
    tcs::WsSizer z;
    z.batched = [](const std::vector<int64_t>& n, const std::vector<int64_t>& T, const std::vector<int32_t>& p) {
      return tc_batch_layout((int64_t)n.size(), n.data(), T.data(), false, 256, nullptr, p.data()).total_bytes;
    };
    z.fifo = [](int64_t n) { return (int64_t)(1 << 20) + 4 * (n / 128 + 1) * (n / 128 + 1); };
    z.tile = [](int64_t n, int prec) { return tc_tuned_batched_tile_prec(n, prec); };
    // a solve workspace of the real shape (the server's solves share one
    // launch, in passes of four): a header, then two payloads of 64-row
    // blocks with 4 columns per pass
    z.solve_ws = [](int64_t n, int64_t nrhs) {
      return (int64_t)256 + 2 * tcs::r256(8 * ((n + 63) / 64) * 64 * 4 * ((nrhs + 3) / 4));
    };
    tcs::PlanTable pt;
    pt.fp32_min_n_loose = 700;
    pt.fp32_min_n_strict = 1500;
    const int64_t arena = (int64_t)(96 + rng() % 64) << 20, pinned = (int64_t)(6 + rng() % 8) << 20;
    tcs::Core core(arena, pinned, mode, 1 + (int64_t)(rng() % 40), z, pt);
    std::vector<tcs::Tick> flight;
    std::vector<int64_t> kept;  // factor handles seen
    std::set<int64_t> in_flight_reqs;
    int64_t clock = 0, last_first_admitted = -1, submitted = 0;
    std::map<int64_t, int> first_seen;
    for (int s = 0; s < steps || !core.idle(); ++s) {
      clock += 1 + (int64_t)(rng() % 100);
      const int act = (int)(rng() % 10);
      if (s < steps && act < 4) {  // a factor + solve request
        const int64_t nn = log_uniform(rng, 64, 2500), nrhs = 1 + (int64_t)(rng() % 8);
        const bool keep = rng() % 3 == 0;
        core.submit_factor(std::vector<double>(2 * nn, 0.5), nn, 0.2, 1e-2, std::vector<double>(nn * nrhs, 1.0),
                           nrhs, rng() % 2 ? 1e-6 : 1e-12, keep, clock);
        ++submitted;
      } else if (s < steps && act == 4 && !kept.empty()) {  // a solve with a (maybe evicted) resident factor
        const int64_t fid = kept[rng() % kept.size()];
        auto it = core.factors().find(fid);
        const int64_t nn = it != core.factors().end() ? it->second.n : 64;
        const int64_t id = core.submit_solve(fid, std::vector<double>(nn * 2, 1.0), 2, 1e-12, clock);
        CHECK(id >= 0 || it == core.factors().end(), "solve refused with its factor resident");
        if (id >= 0) ++submitted;
      } else if (s < steps && act == 5 && !kept.empty() && rng() % 4 == 0) {
        core.release_factor(kept[rng() % kept.size()]);
      } else if (act < 8 && core.inflight() < 2) {  // admit a tick
        tcs::Tick t;
        if (core.admit(t, clock)) {
          for (const tcs::TickItem& it : t.items) {
            CHECK(!in_flight_reqs.count(it.req), "request %lld in two ticks", (long long)it.req);
            in_flight_reqs.insert(it.req);
            const tcs::Request& R = core.req(it.req);
            CHECK(R.state == tcs::ST_RUNNING, "request %lld admitted in state %d", (long long)it.req, R.state);
            if (!first_seen.count(it.req)) {
              first_seen[it.req] = 1;
              // new requests start in arrival order
              CHECK(it.req > last_first_admitted, "request %lld admitted after %lld", (long long)it.req,
                    (long long)last_first_admitted);
              last_first_admitted = it.req;
            }
          }
          CHECK(mode == 0 || t.items.size() == 1, "FIFO tick with %zu items", t.items.size());
          flight.push_back(t);
        }
        (void)core.take_finished();
      } else if (!flight.empty()) {  // a tick finishes with random device results
        const size_t k = rng() % flight.size();
        const tcs::Tick t = flight[k];
        flight.erase(flight.begin() + k);
        std::vector<tcs::ItemResult> res(t.items.size());
        for (size_t q = 0; q < t.items.size(); ++q) {
          in_flight_reqs.erase(t.items[q].req);
          const tcs::Request& R = core.req(t.items[q].req);
          res[q].eta = rng() % 10 < 3 ? R.tol * 10 : R.tol / 10;
          if (t.items[q].item == tcs::ITEM_FACTOR && rng() % 50 == 0) {
            res[q].factor_err = 1;
            res[q].factor_info = 7;
          }
          if (rng() % 100 == 0) res[q].solve_err = 1;
        }
        core.finish(t, res, clock);
        for (int64_t id : core.take_finished()) {
          const tcs::Request& R = core.req(id);
          CHECK(R.state >= tcs::ST_DONE, "finished request %lld in state %d", (long long)id, R.state);
          if (R.keep && R.state == tcs::ST_DONE && R.factor_id >= 0) kept.push_back(R.factor_id);
        }
      }
      // ---- invariants: every live region once, disjoint, accounted for
      std::vector<Region> dev, pin;
      for (const tcs::Tick& t : flight) {
        dev.push_back({t.ws_off, t.ws_bytes, "tick ws"});
        dev.push_back({t.meta_dev, t.meta_bytes, "tick meta"});
        pin.push_back({t.meta_pin, t.pin_meta_bytes, "tick pinned"});
      }
      for (int64_t id = 0; id < core.num_requests(); ++id) {
        const tcs::Request& R = core.req(id);
        if (R.state != tcs::ST_RUNNING) continue;
        if (R.fac_owned) dev.push_back({R.fac_off, R.fac_bytes, "factor of " + std::to_string(id)});
        dev.push_back({R.work_off, R.work_bytes, "work of " + std::to_string(id)});
        pin.push_back({R.pin_off, R.pin_bytes, "staging of " + std::to_string(id)});
        if (R.kind == tcs::REQ_SOLVE)
          CHECK(core.factors().count(R.factor_id), "request %lld uses evicted factor %lld", (long long)id,
                (long long)R.factor_id);
      }
      for (const auto& kv : core.factors()) dev.push_back({kv.second.dev_off, kv.second.dev_bytes, "resident"});
      if (!disjoint(dev, core.dev().size(), "device") || !disjoint(pin, core.pin().size(), "pinned")) return 1;
      int64_t ud = 0, up = 0;
      for (auto& r : dev) ud += tcs::r256(r.bytes);
      for (auto& r : pin) up += tcs::r256(r.bytes);
      CHECK(ud == core.dev().used(), "device bytes in use %lld, live regions %lld", (long long)core.dev().used(),
            (long long)ud);
      CHECK(up == core.pin().used(), "pinned bytes in use %lld, live regions %lld", (long long)core.pin().used(),
            (long long)up);
      CHECK(s < steps + 200000, "the server does not drain");
    }
    for (int64_t id = 0; id < core.num_requests(); ++id)
      CHECK(core.req(id).state >= tcs::ST_DONE, "request %lld left in state %d", (long long)id, core.req(id).state);
    for (int64_t f : kept) core.release_factor(f);
    CHECK(core.dev().used() == 0 && core.pin().used() == 0, "memory left after the drain");
    printf("OK serve mode=%d requests=%lld evictions=%lld\n", mode, (long long)submitted, (long long)core.evictions());
  }
  return g_fail;
}
}  // namespace

int main(int argc, char** argv) {
  if (argc < 4) {
    fprintf(stderr, "usage: emulate dag|serve <seed> <count>\n");
    return 2;
  }
  const std::string what = argv[1];
  const uint64_t seed = strtoull(argv[2], nullptr, 10);
  const int count = atoi(argv[3]);
  int rv = 2;
  if (what == "dag") rv = run_dag(seed, count);
  if (what == "serve") rv = run_serve(seed, count);
  if (rv == 2) return 2;
  return (rv || g_fail) ? 1 : 0;
}
