// serve.hip -- a factor + solve server with continuous batching.
//
// Requests (the paper's motivating use, Gaussian-process style SPD systems:
// a squared-exponential kernel matrix on n points plus a nugget, with one
// to a few right-hand sides and a target backward error) arrive at any
// time.  A worker thread admits pending requests in arrival order as long
// as their device footprint fits in the caller's arena (the HBM budget),
// and launches them as one tick:
//   1. inputs to the device (pinned staging, asynchronous copies);
//   2. kernel-matrix assembly on the device (lower triangle only);
//   3. ONE persistent launch factoring every matrix of the tick (the batched
//      kernel: per-matrix tile DAGs, tile side from the tuned table,
//      deterministic in n), then each request's solve as multi-workgroup
//      forward and backward sweeps;
//   4. a matrix-free residual (the kernel entries are recomputed from the
//      points, so the factor may overwrite the matrix) giving each request's
//      backward error ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf);
//   5. results back to pinned host memory, an event marks the tick done.
// Up to two ticks are in flight on two streams, so requests that arrive
// while a tick runs are admitted and launched while it is still on the
// device.  A request's result does not depend on what else was in its tick.
//
// The FIFO mode is the plain baseline: one request at a time, fork-join
// chol_factor with the default tile side, then chol_solve.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "launch.h"
#include "tuned_tiles.h"

#define SRV_THREADS 256
#define SRV_MAX_RHS 8
#define SRV_STATS (1 + 3 * SRV_MAX_RHS)  // anorm, rmax[8], xmax[8], bmax[8]

struct SrvDesc {
  double* A;          // n x n, row-major, lda = n
  const double* pts;  // n x 2
  const double* B;    // n x nrhs (the right-hand sides, kept)
  double* X;          // n x nrhs (solution)
  double* stats;      // SRV_STATS doubles, zeroed before the residual
  double* eta;        // one double: the request's worst column
  int64_t n, nrhs;
  double inv2l2, nugget;
};

__device__ __forceinline__ double srv_k(const double* p, int64_t i, int64_t j, double inv2l2, double nugget) {
  const double d0 = p[2 * i] - p[2 * j], d1 = p[2 * i + 1] - p[2 * j + 1];
  return exp(-(d0 * d0 + d1 * d1) * inv2l2) + (i == j ? nugget : 0.0);
}

// A_ij for j <= i; grid (row blocks of 8, requests).
__global__ __launch_bounds__(SRV_THREADS) void srv_assemble(const SrvDesc* __restrict__ reqs) {
  const SrvDesc d = reqs[blockIdx.y];
  const int64_t i0 = (int64_t)blockIdx.x * 8;
  for (int64_t i = i0; i < i0 + 8 && i < d.n; ++i)
    for (int64_t j = threadIdx.x; j <= i; j += SRV_THREADS) d.A[i * d.n + j] = srv_k(d.pts, i, j, d.inv2l2, d.nugget);
}

__device__ __forceinline__ void srv_atomic_max(double* p, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

// Matrix-free residual statistics; grid (row blocks of 64, requests).  Thread
// (row r, part p) sums columns j = p, p + 4, ... of row i = 64 block + r; the
// four parts are combined in a fixed order.
__global__ __launch_bounds__(SRV_THREADS) void srv_residual(const SrvDesc* __restrict__ reqs) {
  const SrvDesc d = reqs[blockIdx.y];
  const int r = threadIdx.x >> 2, p = threadIdx.x & 3;
  const int64_t i = (int64_t)blockIdx.x * 64 + r;
  const bool row = i < d.n;
  double rs = 0.0, acc[SRV_MAX_RHS];
#pragma unroll
  for (int c = 0; c < SRV_MAX_RHS; ++c) acc[c] = 0.0;
  if (row) {
    for (int64_t j = p; j < d.n; j += 4) {
      const double k = srv_k(d.pts, i, j, d.inv2l2, d.nugget);
      rs += fabs(k);
#pragma unroll
      for (int c = 0; c < SRV_MAX_RHS; ++c)
        if (c < d.nrhs) acc[c] += k * d.X[j * d.nrhs + c];
    }
  }
  rs += __shfl_xor(rs, 1);
  rs += __shfl_xor(rs, 2);
#pragma unroll
  for (int c = 0; c < SRV_MAX_RHS; ++c) {
    acc[c] += __shfl_xor(acc[c], 1);
    acc[c] += __shfl_xor(acc[c], 2);
  }
  if (row && p == 0) {
    srv_atomic_max(d.stats, rs);
    for (int c = 0; c < d.nrhs; ++c) {
      const double b = d.B[i * d.nrhs + c], x = d.X[i * d.nrhs + c];
      srv_atomic_max(d.stats + 1 + c, fabs(b - acc[c]));
      srv_atomic_max(d.stats + 1 + SRV_MAX_RHS + c, fabs(x));
      srv_atomic_max(d.stats + 1 + 2 * SRV_MAX_RHS + c, fabs(b));
    }
  }
}

__global__ void srv_eta(const SrvDesc* __restrict__ reqs, int64_t count) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= count) return;
  const SrvDesc d = reqs[q];
  double worst = 0.0;
  for (int c = 0; c < d.nrhs; ++c) {
    const double den = d.stats[0] * d.stats[1 + SRV_MAX_RHS + c] + d.stats[1 + 2 * SRV_MAX_RHS + c];
    const double e = den > 0.0 ? d.stats[1 + c] / den : 0.0;
    worst = e > worst || e != e ? e : worst;
  }
  d.eta[0] = worst;
}

__global__ void srv_zero(double* p, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// ------------------------------------------------------------ host runtime
namespace {
int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
int64_t r256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// First-fit allocator over [0, size) with 256-byte granularity.
class FirstFit {
 public:
  explicit FirstFit(int64_t size = 0) {
    if (size > 0) free_[0] = size;
  }
  int64_t alloc(int64_t bytes) {
    bytes = r256(bytes > 0 ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = r256(bytes > 0 ? bytes : 1);
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

 private:
  std::map<int64_t, int64_t> free_;
};

struct Request {
  int64_t n = 0, nrhs = 0;
  double lengthscale = 0, nugget = 0, tol = 0;
  std::vector<double> pts, B, X;
  double eta = 0;
  int64_t t_arrive = 0, t_done = 0, info = 0;
  // 0 pending, 1 running, 2 done, 3 failed (not SPD), 4 rejected (does not fit), 6 a dependency wait ran out
  int state = 0;
  int64_t dev_off = -1, dev_bytes = 0, pin_off = -1, pin_bytes = 0;
};

struct Tick {
  std::vector<int64_t> ids;
  std::vector<Request*> rq;  // taken under the lock at admission
  int stream = 0;
  hipEvent_t done = nullptr;
  int64_t ws_off = -1, ws_bytes = 0, solve_off = 0, meta_dev = -1, meta_bytes = 0, meta_pin = -1, pin_meta_bytes = 0;
  char* hdr_pin = nullptr;  // per-matrix status headers copied back
  char* sv_pin = nullptr;   // per-request solve workspaces (status words) copied back
};
}  // namespace

struct TcServer {
  int device = 0;
  char* arena = nullptr;
  int64_t arena_bytes = 0;
  char* pinned = nullptr;
  int64_t pinned_bytes = 0;
  int mode = 0;
  int64_t max_per_tick = 0;
  int64_t wait_ticks = 0;
  FirstFit dev, pin;
  hipStream_t st[2] = {nullptr, nullptr};
  std::mutex mu;
  std::condition_variable cv;
  std::deque<int64_t> pending;
  std::vector<std::unique_ptr<Request>> reqs;
  std::vector<Tick> inflight;
  std::thread worker;
  bool stop = false;
  int error = 0;
  int64_t ticks = 0;
  int next_stream = 0;
};

namespace {
// device bytes of one request: matrix, points, right-hand sides and
// solution, statistics and eta
int64_t dev_need(int64_t n, int64_t nrhs) {
  return r256(8 * n * n) + r256(16 * n) + 2 * r256(8 * n * nrhs) + r256(8 * (SRV_STATS + 1));
}
// pinned bytes: points and right-hand sides in, solution and eta out
int64_t pin_need(int64_t n, int64_t nrhs) { return r256(16 * n) + 2 * r256(8 * n * nrhs) + r256(8); }

// Launch one tick for the admitted requests `ids` (holding no lock; the
// requests' fields it reads are fixed while they run).
bool launch_tick(TcServer& S, Tick& t) {
  hipStream_t st = S.st[t.stream];
  const int64_t m = (int64_t)t.ids.size();
  std::vector<SrvDesc> desc(m);
  std::vector<double*> A(m), X(m);
  std::vector<int64_t> n(m), lda(m), T(m), nrhs(m), ldb(m);
  for (int64_t q = 0; q < m; ++q) {
    Request& R = *t.rq[q];
    char* d = S.arena + R.dev_off;
    char* h = S.pinned + R.pin_off;
    SrvDesc& D = desc[q];
    D.n = R.n;
    D.nrhs = R.nrhs;
    D.A = (double*)d;
    D.pts = (const double*)(d + r256(8 * R.n * R.n));
    D.B = (const double*)(d + r256(8 * R.n * R.n) + r256(16 * R.n));
    D.X = (double*)(d + r256(8 * R.n * R.n) + r256(16 * R.n) + r256(8 * R.n * R.nrhs));
    D.stats = (double*)(d + r256(8 * R.n * R.n) + r256(16 * R.n) + 2 * r256(8 * R.n * R.nrhs));
    D.eta = D.stats + SRV_STATS;
    D.inv2l2 = 1.0 / (2.0 * R.lengthscale * R.lengthscale);
    D.nugget = R.nugget;
    // inputs through pinned staging
    double* hp = (double*)h;
    double* hb = (double*)(h + r256(16 * R.n));
    memcpy(hp, R.pts.data(), 16 * R.n);
    memcpy(hb, R.B.data(), 8 * R.n * R.nrhs);
    if (hipMemcpyAsync((void*)D.pts, hp, 16 * R.n, hipMemcpyHostToDevice, st) != hipSuccess) return false;
    if (hipMemcpyAsync((void*)D.B, hb, 8 * R.n * R.nrhs, hipMemcpyHostToDevice, st) != hipSuccess) return false;
    if (hipMemcpyAsync(D.X, D.B, 8 * R.n * R.nrhs, hipMemcpyDeviceToDevice, st) != hipSuccess) return false;
    A[q] = D.A;
    X[q] = D.X;
    n[q] = R.n;
    lda[q] = R.n;
    nrhs[q] = R.nrhs;
    ldb[q] = R.nrhs;
    T[q] = S.mode == 0 ? tc_tuned_batched_tile(R.n) : tc_default_tile(R.n);
  }
  // descriptors: pinned -> device (meta region)
  SrvDesc* meta_h = (SrvDesc*)(S.pinned + t.meta_pin);
  memcpy(meta_h, desc.data(), sizeof(SrvDesc) * m);
  SrvDesc* meta_d = (SrvDesc*)(S.arena + t.meta_dev);
  if (hipMemcpyAsync(meta_d, meta_h, sizeof(SrvDesc) * m, hipMemcpyHostToDevice, st) != hipSuccess) return false;
  int64_t nmax = 0;
  for (int64_t q = 0; q < m; ++q) nmax = std::max(nmax, n[q]);
  hipLaunchKernelGGL(srv_assemble, dim3((unsigned)((nmax + 7) / 8), (unsigned)m), dim3(SRV_THREADS), 0, st, meta_d);
  if (S.mode == 0) {
    const int64_t grid = tc_batched_grid_size();
    const int64_t chunk = grid > 1 ? grid / 2 : 128;
    // one launch factors every matrix of the tick; the solves then run as
    // multi-workgroup sweeps per request (a one-workgroup solve unit would put
    // O(n^2 nrhs) serial work on one CU for the large orders)
    if (tc_launch_batched(A.data(), nullptr, n.data(), lda.data(), T.data(), m, S.arena + t.ws_off, st, grid,
                          S.wait_ticks, chunk) != 0)
      return false;
    // every request's solve has a workspace (and status word) of its own
    char* sws = S.arena + t.ws_off + t.solve_off;
    const int64_t sb = r256(tc_solve_ws_bytes());
    for (int64_t q = 0; q < m; ++q) {
      if (tc_solve_status_reset(sws + sb * q, st) != 0) return false;
      if (tc_launch_solve(A[q], n[q], n[q], T[q], X[q], nrhs[q], ldb[q], sws + sb * q, st, S.wait_ticks) != 0)
        return false;
    }
    if (hipMemcpyAsync(t.hdr_pin, S.arena + t.ws_off + 256, tc_ws_header_bytes() * m, hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return false;
    if (hipMemcpyAsync(t.sv_pin, sws, sb * m, hipMemcpyDeviceToHost, st) != hipSuccess) return false;
  } else {
    // one request: fork-join factor, then the solve
    char* sws = S.arena + t.ws_off + t.solve_off;
    if (tc_launch_factor(A[0], n[0], n[0], T[0], 0, S.arena + t.ws_off, st, 0, S.wait_ticks, 0) != 0) return false;
    if (tc_solve_status_reset(sws, st) != 0) return false;
    if (tc_launch_solve(A[0], n[0], n[0], T[0], X[0], nrhs[0], ldb[0], sws, st, S.wait_ticks) != 0) return false;
    if (hipMemcpyAsync(t.hdr_pin, S.arena + t.ws_off, tc_ws_header_bytes(), hipMemcpyDeviceToHost, st) != hipSuccess)
      return false;
    if (hipMemcpyAsync(t.sv_pin, sws, r256(tc_solve_ws_bytes()), hipMemcpyDeviceToHost, st) != hipSuccess)
      return false;
  }
  for (int64_t q = 0; q < m; ++q)
    hipLaunchKernelGGL(srv_zero, dim3(1), dim3(64), 0, st, desc[q].stats, (int64_t)(SRV_STATS + 1));
  hipLaunchKernelGGL(srv_residual, dim3((unsigned)((nmax + 63) / 64), (unsigned)m), dim3(SRV_THREADS), 0, st,
                     (const SrvDesc*)meta_d);
  hipLaunchKernelGGL(srv_eta, dim3((unsigned)((m + 63) / 64)), dim3(64), 0, st, (const SrvDesc*)meta_d, m);
  for (int64_t q = 0; q < m; ++q) {
    Request& R = *t.rq[q];
    char* h = S.pinned + R.pin_off;
    double* hx = (double*)(h + r256(16 * R.n) + r256(8 * R.n * R.nrhs));
    double* he = (double*)(h + r256(16 * R.n) + 2 * r256(8 * R.n * R.nrhs));
    if (hipMemcpyAsync(hx, desc[q].X, 8 * R.n * R.nrhs, hipMemcpyDeviceToHost, st) != hipSuccess) return false;
    if (hipMemcpyAsync(he, desc[q].eta, 8, hipMemcpyDeviceToHost, st) != hipSuccess) return false;
  }
  if (hipEventRecord(t.done, st) != hipSuccess) return false;
  return hipGetLastError() == hipSuccess;
}

// device bytes of the tick's own workspace: the batched counters and unit
// list (or the fork-join workspace), then one solve workspace per request
// from byte *solve_off on
int64_t tick_ws_bytes(TcServer& S, const std::vector<int64_t>& ids, int64_t* solve_off) {
  int64_t head = 0;
  if (S.mode == 0) {
    std::vector<int64_t> n, T;
    for (int64_t id : ids) {
      n.push_back(S.reqs[id]->n);
      T.push_back(tc_tuned_batched_tile(S.reqs[id]->n));
    }
    const int64_t grid = tc_batched_grid_size();
    head = r256(tc_batched_ws_bytes((int64_t)ids.size(), n.data(), T.data(), 0, grid > 1 ? grid / 2 : 128));
  } else {
    const int64_t n = S.reqs[ids[0]]->n;
    head = r256(tc_ws_bytes(n, tc_default_tile(n)));
  }
  *solve_off = head;
  return head + r256(tc_solve_ws_bytes()) * (int64_t)ids.size();
}

void finish_tick(TcServer& S, Tick& t) {
  const int64_t t_done = now_ns();
  const int64_t hb = tc_ws_header_bytes();
  for (size_t q = 0; q < t.ids.size(); ++q) {
    Request& R = *t.rq[q];
    char* h = S.pinned + R.pin_off;
    const double* hx = (const double*)(h + r256(16 * R.n) + r256(8 * R.n * R.nrhs));
    const double* he = (const double*)(h + r256(16 * R.n) + 2 * r256(8 * R.n * R.nrhs));
    R.X.assign(hx, hx + R.n * R.nrhs);
    R.eta = *he;
    int32_t err = 0, serr = 0;
    int64_t info = 0;
    tc_ws_header_read(t.hdr_pin + hb * q, &err, &info);
    memcpy(&serr, t.sv_pin + r256(tc_solve_ws_bytes()) * q + tc_solve_status_offset(), sizeof(serr));
    if (err == 1) {  // not positive definite: the failing column + 1
      R.info = info;
      R.state = 3;
    } else if (err) {  // the factorization's dependency wait ran out: 1 + its unit's ticket
      R.info = info > 0 ? info : 1;
      R.state = 6;
    } else if (serr) {  // a solve sweep's dependency wait ran out
      R.info = -1;
      R.state = 6;
    } else {
      R.info = 0;
      R.state = 2;
    }
    R.t_done = t_done;
    S.dev.release(R.dev_off, R.dev_bytes);
    S.pin.release(R.pin_off, R.pin_bytes);
    R.pts.clear();
    R.pts.shrink_to_fit();
    R.B.clear();
    R.B.shrink_to_fit();
  }
  S.dev.release(t.ws_off, t.ws_bytes);
  S.dev.release(t.meta_dev, t.meta_bytes);
  S.pin.release(t.meta_pin, t.pin_meta_bytes);
  (void)hipEventDestroy(t.done);
}

void worker_main(TcServer* Sp) {
  TcServer& S = *Sp;
  (void)hipSetDevice(S.device);
  const int max_inflight = S.mode == 0 ? 2 : 1;
  for (;;) {
    bool did = false;
    // completions
    {
      std::unique_lock<std::mutex> lk(S.mu);
      for (size_t k = 0; k < S.inflight.size();) {
        if (hipEventQuery(S.inflight[k].done) == hipSuccess) {
          finish_tick(S, S.inflight[k]);
          S.inflight.erase(S.inflight.begin() + k);
          did = true;
        } else {
          ++k;
        }
      }
      if (did) S.cv.notify_all();
      if (S.stop && S.pending.empty() && S.inflight.empty()) return;
    }
    // admission and launch
    Tick t;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      if ((int)S.inflight.size() < max_inflight && !S.pending.empty() && S.error == 0) {
        const int64_t cap = S.mode == 0 ? S.max_per_tick : 1;
        while (!S.pending.empty() && (int64_t)t.ids.size() < cap) {
          const int64_t id = S.pending.front();
          Request& R = *S.reqs[id];
          R.dev_bytes = dev_need(R.n, R.nrhs);
          R.pin_bytes = pin_need(R.n, R.nrhs);
          const int64_t doff = S.dev.alloc(R.dev_bytes);
          if (doff < 0) {
            if (t.ids.empty() && S.inflight.empty()) {  // can never fit
              R.state = 4;
              R.t_done = now_ns();
              S.pending.pop_front();
              S.cv.notify_all();
              continue;
            }
            break;  // wait for memory to free up (arrival order is kept)
          }
          const int64_t poff = S.pin.alloc(R.pin_bytes);
          if (poff < 0) {
            S.dev.release(doff, R.dev_bytes);
            if (t.ids.empty() && S.inflight.empty()) {
              R.state = 4;
              R.t_done = now_ns();
              S.pending.pop_front();
              S.cv.notify_all();
              continue;
            }
            break;
          }
          R.dev_off = doff;
          R.pin_off = poff;
          R.state = 1;
          S.pending.pop_front();
          t.ids.push_back(id);
          t.rq.push_back(&R);
        }
        // the tick's workspace and descriptors: if they do not fit, give the
        // last requests back (front of the queue, order kept) and retry with
        // fewer; a lone request that cannot get them with nothing in flight
        // is rejected
        while (!t.ids.empty()) {
          const int64_t m = (int64_t)t.ids.size();
          t.ws_bytes = tick_ws_bytes(S, t.ids, &t.solve_off);
          t.meta_bytes = r256((int64_t)sizeof(SrvDesc) * m);
          const int64_t hdr_bytes = r256(tc_ws_header_bytes() * m);
          t.pin_meta_bytes = t.meta_bytes + hdr_bytes + r256(tc_solve_ws_bytes()) * m;
          t.ws_off = S.dev.alloc(t.ws_bytes);
          t.meta_dev = t.ws_off >= 0 ? S.dev.alloc(t.meta_bytes) : -1;
          t.meta_pin = t.meta_dev >= 0 ? S.pin.alloc(t.pin_meta_bytes) : -1;
          if (t.meta_pin >= 0) {
            t.hdr_pin = S.pinned + t.meta_pin + t.meta_bytes;
            t.sv_pin = t.hdr_pin + hdr_bytes;
            t.stream = S.next_stream;
            S.next_stream ^= 1;
            break;
          }
          if (t.meta_dev >= 0) S.dev.release(t.meta_dev, t.meta_bytes);
          if (t.ws_off >= 0) S.dev.release(t.ws_off, t.ws_bytes);
          const size_t keep = t.ids.size() > 1 ? t.ids.size() / 2 : 0;
          while (t.ids.size() > keep) {
            Request& R = *t.rq.back();
            S.dev.release(R.dev_off, R.dev_bytes);
            S.pin.release(R.pin_off, R.pin_bytes);
            if (keep == 0 && S.inflight.empty()) {
              R.state = 4;  // cannot run even alone
              R.t_done = now_ns();
              S.cv.notify_all();
            } else {
              R.state = 0;
              S.pending.push_front(t.ids.back());
            }
            t.ids.pop_back();
            t.rq.pop_back();
          }
        }
      }
    }
    if (!t.ids.empty()) {
      if (hipEventCreateWithFlags(&t.done, hipEventDisableTiming) != hipSuccess || !launch_tick(S, t)) {
        std::unique_lock<std::mutex> lk(S.mu);
        S.error = 1;
        S.cv.notify_all();
        return;
      }
      std::unique_lock<std::mutex> lk(S.mu);
      S.inflight.push_back(t);
      ++S.ticks;
      did = true;
    }
    if (!did) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}
}  // namespace

// ---------------------------------------------------------------- entry points
int tc_server_create(void* arena, int64_t arena_bytes, int64_t pinned_bytes, int mode, int64_t max_per_tick,
                     int64_t wait_ticks, TcServer** out) {
  auto S = std::make_unique<TcServer>();
  if (hipGetDevice(&S->device) != hipSuccess) return TC_LAUNCH_EDEVICE;
  S->arena = (char*)arena;
  S->arena_bytes = arena_bytes;
  S->dev = FirstFit(arena_bytes & ~(int64_t)255);
  S->pinned_bytes = r256(pinned_bytes);
  void* p = nullptr;
  if (hipHostMalloc(&p, S->pinned_bytes, hipHostMallocDefault) != hipSuccess) return TC_LAUNCH_EDEVICE;
  S->pinned = (char*)p;
  S->pin = FirstFit(S->pinned_bytes);
  S->mode = mode;
  S->max_per_tick = max_per_tick;
  S->wait_ticks = wait_ticks;
  for (int k = 0; k < 2; ++k)
    if (hipStreamCreateWithFlags(&S->st[k], hipStreamNonBlocking) != hipSuccess) return TC_LAUNCH_EDEVICE;
  S->worker = std::thread(worker_main, S.get());
  *out = S.release();
  return 0;
}

int tc_server_submit(TcServer* S, const double* pts, int64_t n, double lengthscale, double nugget, const double* B,
                     int64_t nrhs, double tol, int64_t* id) {
  auto R = std::make_unique<Request>();
  R->n = n;
  R->nrhs = nrhs;
  R->lengthscale = lengthscale;
  R->nugget = nugget;
  R->tol = tol;
  R->pts.assign(pts, pts + 2 * n);
  R->B.assign(B, B + n * nrhs);
  R->t_arrive = now_ns();
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->error) return TC_LAUNCH_EDEVICE;
  *id = (int64_t)S->reqs.size();
  S->reqs.push_back(std::move(R));
  S->pending.push_back(*id);
  return 0;
}

// Returns the request state after waiting up to timeout_s (2 done within its
// tolerance, 5 done but above it, 3 not SPD, 4 rejected, 6 a dependency wait
// of its factorization (info = 1 + the unit's ticket) or of a solve sweep
// (info = -1) ran out, 0/1 still pending / running), or < 0 on a device
// error.
int tc_server_wait(TcServer* S, int64_t id, double timeout_s, double* X, double* eta, double* latency_s,
                   int64_t* info) {
  std::unique_lock<std::mutex> lk(S->mu);
  if (id < 0 || id >= (int64_t)S->reqs.size()) return TC_LAUNCH_EINVAL;
  Request& R = *S->reqs[id];
  S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return R.state >= 2 || S->error; });
  if (S->error && R.state < 2) return TC_LAUNCH_EDEVICE;
  if (R.state >= 2) {
    if (X && R.state == 2) memcpy(X, R.X.data(), 8 * R.n * R.nrhs);
    if (eta) *eta = R.eta;
    if (latency_s) *latency_s = (R.t_done - R.t_arrive) * 1e-9;
    if (info) *info = R.info;
    if (R.state == 2 && !(R.eta <= R.tol)) return 5;
  }
  return R.state;
}

int64_t tc_server_ticks(TcServer* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  return S->ticks;
}

int tc_server_destroy(TcServer* S) {
  {
    std::unique_lock<std::mutex> lk(S->mu);
    S->stop = true;
  }
  if (S->worker.joinable()) S->worker.join();
  int rc = S->error ? TC_LAUNCH_EDEVICE : 0;
  // after an error ticks may still be on the device: let them finish before
  // the pinned staging they copy into is freed
  for (int k = 0; k < 2; ++k)
    if (S->st[k] && hipStreamSynchronize(S->st[k]) != hipSuccess) rc = TC_LAUNCH_EDEVICE;
  for (Tick& t : S->inflight)
    if (t.done) (void)hipEventDestroy(t.done);
  for (int k = 0; k < 2; ++k)
    if (S->st[k]) (void)hipStreamDestroy(S->st[k]);
  if (S->pinned) (void)hipHostFree(S->pinned);
  delete S;
  return rc;
}
