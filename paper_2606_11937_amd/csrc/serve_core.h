// serve_core.h -- host-side bookkeeping of the factor + solve server, with
// no device calls: request states, first-fit arenas (device memory and
// pinned staging), admission by footprint in arrival order, the precision
// plan of each request, refinement and fallback steps, resident factors with
// LRU eviction, and the per-tick layout.  The server (serve.hip) asks it what
// to launch and reports back what the device computed; the CPU tests drive
// it with fake arenas, clocks and results (under sanitizers).
//
// Work items.  A request becomes one or more items, each run in some tick:
//   FACTOR    assemble the kernel matrix, factor it (batched launch, the
//             request's precision), solve, residual;
//   CORRECT   solve the residual left by the previous item, add it to X,
//             residual again (iterative refinement in FP64);
//   SOLVE     against a resident factor: solve, residual.
// After each item the device has computed the request's backward error eta.
// The core then finishes the request (eta <= tol), schedules a CORRECT item
// (corrections left), or refactors in FP64 (a low-precision factor whose
// corrections ran out), else finishes it above its tolerance.
#pragma once
#include <stdint.h>

#include <algorithm>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <vector>

namespace tcs {

inline int64_t r256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// First-fit allocator over [0, size) with 256-byte granularity.
class FirstFit {
 public:
  explicit FirstFit(int64_t size = 0) : size_(size) {
    if (size > 0) free_[0] = size;
  }
  int64_t size() const { return size_; }
  int64_t alloc(int64_t bytes) {
    bytes = r256(bytes > 0 ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        used_ += bytes;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = r256(bytes > 0 ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t used() const { return used_; }
  const std::map<int64_t, int64_t>& free_list() const { return free_; }

 private:
  int64_t size_ = 0, used_ = 0;
  std::map<int64_t, int64_t> free_;
};

enum Kind { REQ_FACTOR_SOLVE = 0, REQ_SOLVE = 1 };
enum Item { ITEM_FACTOR = 0, ITEM_CORRECT = 1, ITEM_SOLVE = 2 };
// request states (values shared with the C ABI mapping)
enum State {
  ST_PENDING = 0,
  ST_RUNNING = 1,
  ST_DONE = 2,
  ST_NOT_SPD = 3,
  ST_REJECTED = 4,
  ST_STALLED = 6,
  ST_NO_FACTOR = 7
};
enum { PREC_FP64 = 0, PREC_FP32 = 1 };

// Precision plan of a factor + solve request, from (n, tol) only.
struct Plan {
  int prec = PREC_FP64;
  int max_corr = 1;  // corrections before giving up (low precision: before the FP64 refactor)
};

// The plan table: FP32 trailing products where they pay (orders whose
// factorization has enough update work, below the tolerance class's FP32
// reach after refinement), else FP64.
struct PlanTable {
  int64_t fp32_min_n_loose = 1 << 30;   // tol >= loose_tol: FP32 from this order on
  int64_t fp32_min_n_strict = 1 << 30;  // tol <  loose_tol
  double loose_tol = 1e-8;
  int fp32_corr = 3;
  Plan plan(int64_t n, double tol) const {
    Plan p;
    const bool loose = tol >= loose_tol;
    if (n >= (loose ? fp32_min_n_loose : fp32_min_n_strict)) {
      p.prec = PREC_FP32;
      p.max_corr = fp32_corr;
    }
    return p;
  }
};

// Device bytes of the pieces of a request.
inline int64_t factor_bytes(int64_t n) { return r256(8 * n * n) + r256(16 * n); }  // L (n x n) + points
// ||A||_inf, per column max|r|, max|x|, max|b|, then eta and the solve's status word
inline int64_t stats_doubles(int64_t nrhs) { return 1 + 3 * nrhs + 2; }
inline int64_t work_bytes(int64_t n, int64_t nrhs) {  // B, X, R, stats
  return 3 * r256(8 * n * nrhs) + r256(8 * stats_doubles(nrhs));
}
// pinned bytes: points and B in, X, eta and the solve status out
inline int64_t pin_bytes(int64_t n, int64_t nrhs) { return r256(16 * n) + 2 * r256(8 * n * nrhs) + r256(8); }

struct Request {
  int kind = REQ_FACTOR_SOLVE;
  int64_t n = 0, nrhs = 0;
  double lengthscale = 0, nugget = 0, tol = 0;
  bool keep = false;        // keep the factor resident (its handle in factor_id)
  int64_t factor_id = -1;   // SOLVE: the resident factor used; FACTOR_SOLVE with keep: the one made
  std::vector<double> pts, B, X;
  double eta = 0;
  int64_t t_arrive = 0, t_done = 0, info = 0;
  int state = ST_PENDING;
  Plan plan;
  int prec = PREC_FP64;     // precision of the factor in use
  int corrections = 0, refactors = 0, items = 0;
  int stall_retries = 0;  // runs restarted after a dependency wait ran out
  int next_item = ITEM_FACTOR;
  // regions: the factor (L + points; for SOLVE requests the resident
  // factor's) and the request's own work region; pinned staging
  int64_t fac_off = -1, fac_bytes = 0, work_off = -1, work_bytes = 0, pin_off = -1, pin_bytes = 0;
  bool fac_owned = false;   // the factor region belongs to this request (not resident)
};

struct Factor {
  int64_t id = -1, n = 0, dev_off = -1, dev_bytes = 0;
  double lengthscale = 0, nugget = 0;
  int prec = PREC_FP64;
  int64_t last_use = 0;
  int refs = 0;  // requests using it (admitted or pending)
  bool alive = true;
};

struct TickItem {
  int64_t req;
  int item;
};

struct Tick {
  std::vector<TickItem> items;
  int stream = 0;
  int64_t ws_off = -1, ws_bytes = 0, meta_dev = -1, meta_bytes = 0;
  int64_t meta_pin = -1, pin_meta_bytes = 0, hdr_off = 0;
  std::vector<int64_t> solve_off;  // per item: its solve workspace, from ws_off
  int64_t seq = 0;
};

// What the device reported for one item of a finished tick.
struct ItemResult {
  int32_t factor_err = 0;  // 0, 1 not SPD, 2 dependency-wait limit
  int64_t factor_info = 0;
  int32_t solve_err = 0;   // a solve sweep's dependency wait ran out
  double eta = 0;
};

// Sizes of the device workspaces a tick needs, given its items (the server
// passes functions of the real launchers; the tests pass fakes).
struct WsSizer {
  // batched factorization workspace of the tick's FACTOR items (orders, tiles, precisions)
  std::function<int64_t(const std::vector<int64_t>&, const std::vector<int64_t>&, const std::vector<int32_t>&)>
      batched;
  std::function<int64_t(int64_t)> fifo;  // one-at-a-time factorization workspace of order n
  std::function<int64_t(int64_t, int)> tile;  // tile side of order n and precision
  // one item's solve workspace, of order n with nrhs right-hand sides
  std::function<int64_t(int64_t, int64_t)> solve_ws = [](int64_t, int64_t) { return (int64_t)256; };
  int64_t header = 24;      // one factorization status header
  int64_t desc = 128;       // one item descriptor
};

class Core {
 public:
  Core(int64_t arena_bytes, int64_t pinned_bytes, int mode, int64_t max_per_tick, WsSizer sizer, PlanTable plans)
      : dev_(arena_bytes & ~(int64_t)255), pin_(pinned_bytes & ~(int64_t)255), mode_(mode),
        max_per_tick_(max_per_tick), sz_(std::move(sizer)), plans_(plans) {}

  // ---- requests
  int64_t submit_factor(std::vector<double> pts, int64_t n, double ell, double nugget, std::vector<double> B,
                        int64_t nrhs, double tol, bool keep, int64_t now) {
    auto R = std::make_unique<Request>();
    R->kind = REQ_FACTOR_SOLVE;
    R->n = n;
    R->nrhs = nrhs;
    R->lengthscale = ell;
    R->nugget = nugget;
    R->tol = tol;
    R->keep = keep;
    R->pts = std::move(pts);
    R->B = std::move(B);
    R->t_arrive = now;
    R->plan = mode_ == 0 ? plans_.plan(n, tol) : Plan{};
    R->prec = R->plan.prec;
    R->next_item = ITEM_FACTOR;
    const int64_t id = (int64_t)reqs_.size();
    reqs_.push_back(std::move(R));
    pending_.push_back(id);
    return id;
  }
  // A solve against resident factor `fid`; returns -1 if no such factor is
  // resident (never made, or evicted).
  int64_t submit_solve(int64_t fid, std::vector<double> B, int64_t nrhs, double tol, int64_t now) {
    auto it = factors_.find(fid);
    if (it == factors_.end() || !it->second.alive) return -1;
    Factor& F = it->second;
    auto R = std::make_unique<Request>();
    R->kind = REQ_SOLVE;
    R->n = F.n;
    R->nrhs = nrhs;
    R->lengthscale = F.lengthscale;
    R->nugget = F.nugget;
    R->tol = tol;
    R->factor_id = fid;
    R->B = std::move(B);
    R->t_arrive = now;
    R->prec = F.prec;
    R->plan.prec = F.prec;
    R->plan.max_corr = F.prec == PREC_FP64 ? 1 : plans_.fp32_corr;
    R->next_item = ITEM_SOLVE;
    F.refs += 1;  // held until the request is done
    F.last_use = now;
    const int64_t id = (int64_t)reqs_.size();
    reqs_.push_back(std::move(R));
    pending_.push_back(id);
    return id;
  }
  // The precision plan of requests submitted from now on.
  void set_plans(const PlanTable& p) { plans_ = p; }
  const PlanTable& plans() const { return plans_; }
  Request& req(int64_t id) { return *reqs_[id]; }
  const Request& req(int64_t id) const { return *reqs_[id]; }
  int64_t num_requests() const { return (int64_t)reqs_.size(); }
  bool idle() const { return pending_.empty() && inflight_ == 0 && ready_.empty(); }
  int inflight() const { return inflight_; }
  const std::map<int64_t, Factor>& factors() const { return factors_; }
  const FirstFit& dev() const { return dev_; }
  const FirstFit& pin() const { return pin_; }
  int64_t evictions() const { return evictions_; }

  // ---- admission: the next tick, or false when nothing can run now.
  // Items whose request already holds its regions (corrections, FP64
  // refactors) go first; then pending requests in arrival order while their
  // regions fit (evicting unused resident factors, least recently used
  // first, when the arena is short).  A request that cannot fit even in an
  // empty arena is rejected.
  bool admit(Tick& t, int64_t now) {
    t = Tick{};
    const int64_t cap = mode_ == 0 ? max_per_tick_ : 1;
    while (!ready_.empty() && (int64_t)t.items.size() < cap) {
      const int64_t id = ready_.front();
      ready_.pop_front();
      t.items.push_back({id, reqs_[id]->next_item});
    }
    while (!pending_.empty() && (int64_t)t.items.size() < cap) {
      const int64_t id = pending_.front();
      Request& R = *reqs_[id];
      if (!take_regions(R, now, t.items.empty() && inflight_ == 0)) {
        if (R.state == ST_REJECTED) {
          pending_.pop_front();
          finished_.push_back(id);
          continue;
        }
        break;  // wait for memory (arrival order is kept)
      }
      R.state = ST_RUNNING;
      pending_.pop_front();
      t.items.push_back({id, R.next_item});
    }
    // the tick's workspace and descriptors; if they do not fit, give the last
    // new requests back and retry with fewer
    while (!t.items.empty()) {
      if (tick_regions(t)) {
        t.stream = next_stream_;
        next_stream_ ^= 1;
        t.seq = ticks_++;
        ++inflight_;
        for (const TickItem& it : t.items) reqs_[it.req]->items += 1;
        return true;
      }
      const size_t keep = t.items.size() > 1 ? t.items.size() / 2 : 0;
      while (t.items.size() > keep) {
        const TickItem it = t.items.back();
        t.items.pop_back();
        Request& R = *reqs_[it.req];
        const bool follow_up = it.item == ITEM_CORRECT || (it.item == ITEM_FACTOR && R.refactors > 0);
        if (follow_up && !(keep == 0 && inflight_ == 0)) {
          ready_.push_front(it.req);  // it keeps its regions and waits for the next tick
          continue;
        }
        if (follow_up) {  // nothing else runs and even its tick does not fit
          complete(R, it.req, ST_REJECTED, 0, now);
          continue;
        }
        give_back(R);
        if (keep == 0 && inflight_ == 0 && ready_.empty()) {
          R.state = ST_REJECTED;  // cannot run even alone
          R.t_done = now;
          finished_.push_back(it.req);
        } else {
          R.state = ST_PENDING;
          pending_.push_front(it.req);
        }
      }
      if (keep == 0) break;
    }
    return false;
  }

  // ---- completion of a tick with the device's results (one per item, in order).
  void finish(const Tick& t, const std::vector<ItemResult>& res, int64_t now) {
    for (size_t q = 0; q < t.items.size(); ++q) {
      const int64_t id = t.items[q].req;
      Request& R = *reqs_[id];
      const ItemResult& r = res[q];
      R.eta = r.eta;
      if (t.items[q].item == ITEM_FACTOR && r.factor_err == 1) {
        complete(R, id, ST_NOT_SPD, r.factor_info, now);
      } else if ((t.items[q].item == ITEM_FACTOR && r.factor_err) || r.solve_err) {
        // a dependency wait ran out (the result is unspecified): the request
        // starts over once (a fresh solve, after a new factorization unless it
        // solves with a resident factor), then is reported as stalled
        if (R.stall_retries == 0) {
          R.stall_retries = 1;
          R.corrections = 0;
          R.next_item = R.kind == REQ_SOLVE ? ITEM_SOLVE : ITEM_FACTOR;
          ready_.push_back(id);
        } else if (t.items[q].item == ITEM_FACTOR && r.factor_err) {
          complete(R, id, ST_STALLED, r.factor_info > 0 ? r.factor_info : 1, now);
        } else {
          complete(R, id, ST_STALLED, -1, now);
        }
      } else if (!(r.eta > R.tol)) {
        complete(R, id, ST_DONE, 0, now);
      } else if (R.corrections < R.plan.max_corr) {
        R.corrections += 1;
        R.next_item = ITEM_CORRECT;
        ready_.push_back(id);
      } else if (R.kind == REQ_FACTOR_SOLVE && R.prec != PREC_FP64 && R.refactors == 0) {
        // the low-precision factor's corrections ran out: refactor in FP64
        R.refactors += 1;
        R.prec = PREC_FP64;
        R.plan.max_corr = 1;
        R.corrections = 0;
        R.next_item = ITEM_FACTOR;
        ready_.push_back(id);
      } else {
        complete(R, id, ST_DONE, 0, now);  // done, above its tolerance
      }
    }
    release_tick(t);
    --inflight_;
  }

  // Requests finished since the last call (their results are in place).
  std::vector<int64_t> take_finished() {
    std::vector<int64_t> f;
    f.swap(finished_);
    return f;
  }

  // Drop a resident factor (by its handle); false if it is in use or unknown.
  bool release_factor(int64_t fid) {
    auto it = factors_.find(fid);
    if (it == factors_.end() || !it->second.alive || it->second.refs > 0) return false;
    dev_.release(it->second.dev_off, it->second.dev_bytes);
    factors_.erase(it);
    return true;
  }

  // Tile side and precision of a FACTOR item of request R.
  int64_t tile_of(const Request& R) const { return sz_.tile(R.n, R.prec); }

 private:
  bool fits_or_evict(FirstFit& a, int64_t bytes, int64_t* off) {
    *off = a.alloc(bytes);
    while (*off < 0) {
      // evict the least recently used resident factor that no request holds
      Factor* lru = nullptr;
      for (auto& kv : factors_)
        if (kv.second.alive && kv.second.refs == 0 && (lru == nullptr || kv.second.last_use < lru->last_use))
          lru = &kv.second;
      if (lru == nullptr) return false;
      a.release(lru->dev_off, lru->dev_bytes);
      factors_.erase(lru->id);
      ++evictions_;
      *off = a.alloc(bytes);
    }
    return true;
  }

  // Regions of a newly admitted request; on failure nothing is held.  `alone`:
  // nothing else holds memory, so a failure means it can never fit.
  bool take_regions(Request& R, int64_t now, bool alone) {
    const bool own_factor = R.kind == REQ_FACTOR_SOLVE;
    R.fac_bytes = own_factor ? factor_bytes(R.n) : 0;
    R.work_bytes = work_bytes(R.n, R.nrhs);
    R.pin_bytes = pin_bytes(R.n, R.nrhs);
    int64_t foff = -1, woff = -1;
    if (own_factor && !fits_or_evict(dev_, R.fac_bytes, &foff)) {
      if (alone) reject(R, now);
      return false;
    }
    if (!fits_or_evict(dev_, R.work_bytes, &woff)) {
      if (foff >= 0) dev_.release(foff, R.fac_bytes);
      if (alone) reject(R, now);
      return false;
    }
    const int64_t poff = pin_.alloc(R.pin_bytes);
    if (poff < 0) {
      if (foff >= 0) dev_.release(foff, R.fac_bytes);
      dev_.release(woff, R.work_bytes);
      if (alone) reject(R, now);
      return false;
    }
    if (own_factor) {
      R.fac_off = foff;
      R.fac_owned = true;
    } else {
      const Factor& F = factors_.at(R.factor_id);
      R.fac_off = F.dev_off;
      R.fac_bytes = F.dev_bytes;
      R.fac_owned = false;
    }
    R.work_off = woff;
    R.pin_off = poff;
    return true;
  }
  void reject(Request& R, int64_t now) {
    R.state = ST_REJECTED;
    R.t_done = now;
    if (R.kind == REQ_SOLVE) unref(R.factor_id, now);
  }
  void give_back(Request& R) {
    if (R.fac_owned && R.fac_off >= 0) dev_.release(R.fac_off, R.fac_bytes);
    if (R.work_off >= 0) dev_.release(R.work_off, R.work_bytes);
    if (R.pin_off >= 0) pin_.release(R.pin_off, R.pin_bytes);
    R.fac_off = R.work_off = R.pin_off = -1;
    R.fac_owned = false;
  }
  void unref(int64_t fid, int64_t now) {
    auto it = factors_.find(fid);
    if (it != factors_.end()) {
      it->second.refs -= 1;
      it->second.last_use = now;
    }
  }
  void complete(Request& R, int64_t id, int state, int64_t info, int64_t now) {
    R.state = state;
    R.info = info;
    R.t_done = now;
    if (R.kind == REQ_FACTOR_SOLVE && R.keep && state == ST_DONE) {
      // the factor stays resident: its region moves to the factor table
      Factor F;
      F.id = next_factor_++;
      F.n = R.n;
      F.dev_off = R.fac_off;
      F.dev_bytes = R.fac_bytes;
      F.lengthscale = R.lengthscale;
      F.nugget = R.nugget;
      F.prec = R.prec;
      F.last_use = now;
      factors_[F.id] = F;
      R.factor_id = F.id;
      R.fac_owned = false;
      R.fac_off = -1;
    }
    if (R.kind == REQ_SOLVE) unref(R.factor_id, now);
    give_back(R);
    finished_.push_back(id);
  }
  bool tick_regions(Tick& t) {
    const int64_t m = (int64_t)t.items.size();
    std::vector<int64_t> n, T;
    std::vector<int32_t> p;
    for (const TickItem& it : t.items)
      if (it.item == ITEM_FACTOR) {
        const Request& R = *reqs_[it.req];
        n.push_back(R.n);
        T.push_back(tile_of(R));
        p.push_back(R.prec);
      }
    int64_t head = 0;
    if (!n.empty()) head = r256(mode_ == 0 ? sz_.batched(n, T, p) : sz_.fifo(n[0]));
    t.solve_off.assign(m, 0);
    int64_t off = head;
    for (int64_t q = 0; q < m; ++q) {
      const Request& R = *reqs_[t.items[q].req];
      t.solve_off[q] = off;
      off += r256(sz_.solve_ws(R.n, R.nrhs));
    }
    t.ws_bytes = off;
    t.meta_bytes = r256(sz_.desc * m);
    t.hdr_off = t.meta_bytes;
    t.pin_meta_bytes = t.hdr_off + r256(sz_.header * std::max<int64_t>(m, 1));
    if (!fits_or_evict(dev_, t.ws_bytes, &t.ws_off)) t.ws_off = -1;
    if (t.ws_off >= 0 && !fits_or_evict(dev_, t.meta_bytes, &t.meta_dev)) t.meta_dev = -1;
    t.meta_pin = t.meta_dev >= 0 ? pin_.alloc(t.pin_meta_bytes) : -1;
    if (t.meta_pin >= 0) return true;
    if (t.meta_dev >= 0) dev_.release(t.meta_dev, t.meta_bytes);
    if (t.ws_off >= 0) dev_.release(t.ws_off, t.ws_bytes);
    t.ws_off = t.meta_dev = t.meta_pin = -1;
    return false;
  }
  void release_tick(const Tick& t) {
    dev_.release(t.ws_off, t.ws_bytes);
    dev_.release(t.meta_dev, t.meta_bytes);
    pin_.release(t.meta_pin, t.pin_meta_bytes);
  }

  FirstFit dev_, pin_;
  int mode_;
  int64_t max_per_tick_;
  WsSizer sz_;
  PlanTable plans_;
  std::vector<std::unique_ptr<Request>> reqs_;
  std::deque<int64_t> pending_, ready_;
  std::vector<int64_t> finished_;
  std::map<int64_t, Factor> factors_;
  int64_t next_factor_ = 0, ticks_ = 0, evictions_ = 0;
  int inflight_ = 0, next_stream_ = 0;
};

}  // namespace tcs
