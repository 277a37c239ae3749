// serve.hip -- a factor + solve server with continuous batching.
//
// Requests (the paper's motivating use, Gaussian-process style SPD systems:
// a squared-exponential kernel matrix on n points plus a nugget, with one
// to a few right-hand sides and a target backward error) arrive at any
// time, and so do solves against factors the server keeps resident.  The
// host-side bookkeeping (admission by device footprint in arrival order,
// the precision plan of each request, refinement and FP64 fallback steps,
// resident factors with LRU eviction) is serve_core.h; this file runs a
// worker thread around it and launches each tick:
//   1. inputs to the device (pinned staging, asynchronous copies);
//   2. kernel-matrix assembly for the tick's factorizations (lower
//      triangle only);
//   3. ONE persistent launch factoring every matrix of the tick (the batched
//      kernel: per-matrix tile DAGs, tile side from the tuned table for the
//      request's precision, FP32 or FP64 trailing products);
//   4. each item's solve as multi-workgroup forward and backward sweeps (of
//      B for a new solution, of the residual for a correction, then x += d);
//   5. a matrix-free residual r = b - A x (the kernel entries are recomputed
//      from the points, so the factor may overwrite the matrix and a
//      resident factor needs no copy of A) with each item's backward error
//      ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf);
//   6. results back to pinned host memory, an event marks the tick done.
// Up to two ticks are in flight on two streams, so requests that arrive
// while a tick runs are admitted and launched while it is still on the
// device.  A request's result does not depend on what else was in its tick:
// its plan depends on (n, tol) only and every step on its own data.
//
// The FIFO mode is the plain baseline: one request at a time, fork-join
// chol_factor in FP64 with the default tile side, then chol_solve.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <vector>

#include "gptr.h"
#include "launch.h"
#include "serve_core.h"
#include "tuned_tiles.h"

#define SRV_THREADS 256
#define SRV_MAX_RHS 8

// One work item of a tick (see serve_core.h).
struct SrvDesc {
  double* L;          // n x n, row-major, lda = n: the assembled matrix, then its factor
  const double* pts;  // n x 2
  const double* B;    // n x nrhs, the right-hand sides (kept)
  double* X;          // n x nrhs, the solution
  double* R;          // n x nrhs, residual / correction
  double* stats;      // ||A||_inf, then per column max|r|, max|x|, max|b|, then eta and the solve status
  const int32_t* serr;  // the status word of the item's solve workspace
  int64_t n, nrhs;
  double inv2l2, nugget;
  int32_t item;       // tcs::ITEM_*
  int32_t fresh;      // FACTOR or SOLVE item: X starts from B
};

// The descriptor of a workgroup's item with its addresses in the global
// address space (every lane reads the same descriptor).
__device__ __forceinline__ SrvDesc srv_global(SrvDesc d) {
  d.L = tc_global(d.L);
  d.pts = tc_global(d.pts);
  d.B = tc_global(d.B);
  d.X = tc_global(d.X);
  d.R = tc_global(d.R);
  d.stats = tc_global(d.stats);
  d.serr = tc_global(d.serr);
  return d;
}

__device__ __forceinline__ double srv_k(const double* p, int64_t i, int64_t j, double inv2l2, double nugget) {
  const double d0 = p[2 * i] - p[2 * j], d1 = p[2 * i + 1] - p[2 * j + 1];
  return exp(-(d0 * d0 + d1 * d1) * inv2l2) + (i == j ? nugget : 0.0);
}

// A_ij for j <= i of the FACTOR items; grid (row blocks of 8, items).
__global__ __launch_bounds__(SRV_THREADS) void srv_assemble(const SrvDesc* __restrict__ items) {
  const SrvDesc d = srv_global(items[blockIdx.y]);
  if (d.item != tcs::ITEM_FACTOR) return;
  const int64_t i0 = (int64_t)blockIdx.x * 8;
  for (int64_t i = i0; i < i0 + 8 && i < d.n; ++i)
    for (int64_t j = threadIdx.x; j <= i; j += SRV_THREADS) d.L[i * d.n + j] = srv_k(d.pts, i, j, d.inv2l2, d.nugget);
}

// Before the solves: X = B for items that start a solution; zero the
// statistics of every item.  Grid (row blocks of 256, items).
__global__ __launch_bounds__(SRV_THREADS) void srv_prepare(const SrvDesc* __restrict__ items) {
  const SrvDesc d = srv_global(items[blockIdx.y]);
  const int64_t e = (int64_t)blockIdx.x * SRV_THREADS + threadIdx.x;
  if (d.fresh && e < d.n * d.nrhs) d.X[e] = d.B[e];
  if (blockIdx.x == 0 && threadIdx.x < 3 * d.nrhs + 3) d.stats[threadIdx.x] = 0.0;  // tcs::stats_doubles
}

// After a correction's solve: X += R.  Grid (row blocks of 256, items).
__global__ __launch_bounds__(SRV_THREADS) void srv_apply(const SrvDesc* __restrict__ items) {
  const SrvDesc d = srv_global(items[blockIdx.y]);
  const int64_t e = (int64_t)blockIdx.x * SRV_THREADS + threadIdx.x;
  if (d.item == tcs::ITEM_CORRECT && e < d.n * d.nrhs) d.X[e] = d.X[e] + d.R[e];
}

__device__ __forceinline__ void srv_atomic_max(double* p, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

// Matrix-free residual R = B - A X and its statistics; grid (row blocks of
// 64, items).  Thread (row r, part p) sums columns j = p, p + 4, ... of row
// i = 64 block + r; the four parts are combined in a fixed order.
__global__ __launch_bounds__(SRV_THREADS) void srv_residual(const SrvDesc* __restrict__ items) {
  const SrvDesc d = srv_global(items[blockIdx.y]);
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
      const double b = d.B[i * d.nrhs + c], x = d.X[i * d.nrhs + c], ri = b - acc[c];
      d.R[i * d.nrhs + c] = ri;
      srv_atomic_max(d.stats + 1 + c, fabs(ri));
      srv_atomic_max(d.stats + 1 + d.nrhs + c, fabs(x));
      srv_atomic_max(d.stats + 1 + 2 * d.nrhs + c, fabs(b));
    }
  }
}

__global__ void srv_eta(const SrvDesc* __restrict__ items, int64_t count) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= count) return;
  const SrvDesc d = items[q];
  double worst = 0.0;
  for (int c = 0; c < d.nrhs; ++c) {
    const double den = d.stats[0] * d.stats[1 + d.nrhs + c] + d.stats[1 + 2 * d.nrhs + c];
    const double e = den > 0.0 ? d.stats[1 + c] / den : 0.0;
    worst = e > worst || e != e ? e : worst;
  }
  d.stats[1 + 3 * d.nrhs] = worst;
  d.stats[2 + 3 * d.nrhs] = (double)*d.serr;
}

// ------------------------------------------------------------ host runtime
namespace {
int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
using tcs::r256;

struct Flight {
  tcs::Tick t;
  std::vector<tcs::Request*> rq;   // the items' requests, taken under the lock at admission
  hipEvent_t done = nullptr;
  std::vector<int32_t> fac_index;  // item -> index in the batched launch (-1: no factorization)
};
}  // namespace

struct TcServer {
  int device = 0;
  char* arena = nullptr;
  char* pinned = nullptr;
  int mode = 0;
  int64_t wait_ticks = 0;
  std::unique_ptr<tcs::Core> core;
  hipStream_t st[2] = {nullptr, nullptr};
  std::mutex mu;
  std::condition_variable cv;
  std::vector<Flight> inflight;
  std::thread worker;
  bool stop = false;
  int error = 0;
  int64_t ticks = 0;
};

namespace {
// Launch one tick (holding no lock; the fields of its requests that it reads
// are fixed while they run).
bool launch_tick(TcServer& S, Flight& f) {
  const tcs::Tick& t = f.t;
  hipStream_t st = S.st[t.stream];
  const int64_t m = (int64_t)t.items.size();
  std::vector<SrvDesc> desc(m);
  std::vector<TcSolveJob> jobs(m);
  int64_t tickets = 0, max_entries = 0;
  std::vector<double*> A;
  std::vector<int64_t> n, T;
  std::vector<int32_t> prec;
  f.fac_index.assign(m, -1);
  int64_t nmax = 0, emax = 0;
  for (int64_t q = 0; q < m; ++q) {
    const tcs::TickItem& it = t.items[q];
    tcs::Request& R = *f.rq[q];
    char* fac = S.arena + R.fac_off;
    char* wk = S.arena + R.work_off;
    char* h = S.pinned + R.pin_off;
    SrvDesc& D = desc[q];
    D.n = R.n;
    D.nrhs = R.nrhs;
    D.L = (double*)fac;
    D.pts = (const double*)(fac + r256(8 * R.n * R.n));
    D.B = (const double*)wk;
    D.X = (double*)(wk + r256(8 * R.n * R.nrhs));
    D.R = (double*)(wk + 2 * r256(8 * R.n * R.nrhs));
    D.stats = (double*)(wk + 3 * r256(8 * R.n * R.nrhs));
    D.inv2l2 = 1.0 / (2.0 * R.lengthscale * R.lengthscale);
    D.nugget = R.nugget;
    D.item = it.item;
    D.fresh = it.item != tcs::ITEM_CORRECT;
    D.serr = (const int32_t*)(S.arena + t.ws_off + t.solve_off[q] + tc_solve_status_offset());
    // the item's solve, in the tick's one solve launch: of B (in X) for a
    // new solution, of the residual R for a correction
    TcSolveJob& J = jobs[q];
    J.L = D.L;
    J.B = D.fresh ? D.X : D.R;
    J.work = S.arena + t.ws_off + t.solve_off[q];
    J.n = J.lda = R.n;
    J.nrhs = J.ldb = R.nrhs;
    J.first = tickets;
    tickets += tc_solve_many_tickets(R.n, R.nrhs);
    max_entries = std::max(max_entries, ((R.n + 63) / 64) * 64 * 4 * ((R.nrhs + 3) / 4));
    nmax = std::max(nmax, R.n);
    emax = std::max(emax, R.n * R.nrhs);
    // inputs of a request's first item through its pinned staging
    if (R.items == 1) {
      double* hb = (double*)(h + r256(16 * R.n));
      memcpy(hb, R.B.data(), 8 * R.n * R.nrhs);
      if (hipMemcpyAsync((void*)D.B, hb, 8 * R.n * R.nrhs, hipMemcpyHostToDevice, st) != hipSuccess) return false;
      if (R.kind == tcs::REQ_FACTOR_SOLVE) {
        double* hp = (double*)h;
        memcpy(hp, R.pts.data(), 16 * R.n);
        if (hipMemcpyAsync((void*)D.pts, hp, 16 * R.n, hipMemcpyHostToDevice, st) != hipSuccess) return false;
      }
    }
    if (it.item == tcs::ITEM_FACTOR) {
      f.fac_index[q] = (int32_t)A.size();
      A.push_back(D.L);
      n.push_back(R.n);
      T.push_back(S.core->tile_of(R));
      prec.push_back(R.prec);
    }
  }
  // descriptors, then the solve jobs: pinned -> device; the solve launch's
  // two counters follow them
  SrvDesc* meta_h = (SrvDesc*)(S.pinned + t.meta_pin);
  memcpy(meta_h, desc.data(), sizeof(SrvDesc) * m);
  memcpy((char*)meta_h + sizeof(SrvDesc) * m, jobs.data(), sizeof(TcSolveJob) * m);
  SrvDesc* meta_d = (SrvDesc*)(S.arena + t.meta_dev);
  const TcSolveJob* jobs_d = (const TcSolveJob*)((char*)meta_d + sizeof(SrvDesc) * m);
  int32_t* solve_ctr = (int32_t*)((char*)meta_d + (sizeof(SrvDesc) + sizeof(TcSolveJob)) * m);
  if (hipMemcpyAsync(meta_d, meta_h, (sizeof(SrvDesc) + sizeof(TcSolveJob)) * m, hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return false;
  char* ws = S.arena + t.ws_off;
  if (!A.empty()) {
    hipLaunchKernelGGL(srv_assemble, dim3((unsigned)((nmax + 7) / 8), (unsigned)m), dim3(SRV_THREADS), 0, st, meta_d);
    if (S.mode == 0) {
      // one launch factors every matrix of the tick
      const int64_t grid = tc_batched_grid_size();
      const int64_t chunk = grid > 1 ? grid / 2 : 128;
      TcBatchMixed mx;
      mx.prec = prec.data();
      if (tc_launch_batched(A.data(), nullptr, n.data(), n.data(), T.data(), (int64_t)A.size(), ws, st, grid,
                            S.wait_ticks, chunk, nullptr, nullptr, &mx) != 0)
        return false;
    } else if (tc_launch_factor(A[0], n[0], n[0], T[0], 0, ws, st, 0, S.wait_ticks, 0) != 0) {
      return false;
    }
  }
  hipLaunchKernelGGL(srv_prepare, dim3((unsigned)((emax + SRV_THREADS - 1) / SRV_THREADS), (unsigned)m),
                     dim3(SRV_THREADS), 0, st, meta_d);
  // every item's solve in one launch pair, each with a solve workspace (and
  // status word) of its own
  if (tc_launch_solve_many(jobs_d, m, tickets, max_entries, solve_ctr, st, S.wait_ticks) != 0) return false;
  hipLaunchKernelGGL(srv_apply, dim3((unsigned)((emax + SRV_THREADS - 1) / SRV_THREADS), (unsigned)m),
                     dim3(SRV_THREADS), 0, st, (const SrvDesc*)meta_d);
  hipLaunchKernelGGL(srv_residual, dim3((unsigned)((nmax + 63) / 64), (unsigned)m), dim3(SRV_THREADS), 0, st,
                     (const SrvDesc*)meta_d);
  hipLaunchKernelGGL(srv_eta, dim3((unsigned)((m + 63) / 64)), dim3(64), 0, st, (const SrvDesc*)meta_d, m);
  // results: status headers of the factorizations, X, eta and the solve status
  char* hdr_pin = S.pinned + t.meta_pin + t.hdr_off;
  if (!A.empty()) {
    const char* hdr_dev = S.mode == 0 ? ws + 256 : ws;  // batched: per-matrix headers after the ticket
    if (hipMemcpyAsync(hdr_pin, hdr_dev, tc_ws_header_bytes() * (int64_t)A.size(), hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return false;
  }
  for (int64_t q = 0; q < m; ++q) {
    const tcs::Request& R = *f.rq[q];
    char* h = S.pinned + R.pin_off;
    double* hx = (double*)(h + r256(16 * R.n) + r256(8 * R.n * R.nrhs));
    double* he = (double*)(h + r256(16 * R.n) + 2 * r256(8 * R.n * R.nrhs));
    if (hipMemcpyAsync(hx, desc[q].X, 8 * R.n * R.nrhs, hipMemcpyDeviceToHost, st) != hipSuccess) return false;
    if (hipMemcpyAsync(he, desc[q].stats + 1 + 3 * R.nrhs, 16, hipMemcpyDeviceToHost, st) != hipSuccess) return false;
  }
  if (hipEventRecord(f.done, st) != hipSuccess) return false;
  return hipGetLastError() == hipSuccess;
}

void finish_tick(TcServer& S, Flight& f) {
  const tcs::Tick& t = f.t;
  const int64_t hb = tc_ws_header_bytes(), m = (int64_t)t.items.size();
  std::vector<tcs::ItemResult> res(m);
  for (int64_t q = 0; q < m; ++q) {
    tcs::Request& R = S.core->req(t.items[q].req);
    const char* h = S.pinned + R.pin_off;
    const double* hx = (const double*)(h + r256(16 * R.n) + r256(8 * R.n * R.nrhs));
    const double* he = (const double*)(h + r256(16 * R.n) + 2 * r256(8 * R.n * R.nrhs));
    res[q].eta = he[0];
    res[q].solve_err = (int32_t)he[1];
    R.X.assign(hx, hx + R.n * R.nrhs);
    if (f.fac_index[q] >= 0)
      tc_ws_header_read(S.pinned + t.meta_pin + t.hdr_off + hb * f.fac_index[q], &res[q].factor_err,
                        &res[q].factor_info);
  }
  S.core->finish(t, res, now_ns());
  for (int64_t id : S.core->take_finished()) {
    tcs::Request& R = S.core->req(id);
    R.pts.clear();
    R.pts.shrink_to_fit();
    R.B.clear();
    R.B.shrink_to_fit();
  }
  (void)hipEventDestroy(f.done);
}

tcs::WsSizer make_sizer() {
  tcs::WsSizer z;
  z.batched = [](const std::vector<int64_t>& n, const std::vector<int64_t>& T, const std::vector<int32_t>& p) {
    const int64_t grid = tc_batched_grid_size();
    return tc_batched_ws_bytes((int64_t)n.size(), n.data(), T.data(), 0, grid > 1 ? grid / 2 : 128, p.data());
  };
  z.fifo = [](int64_t n) { return tc_ws_bytes(n, tc_default_tile(n)); };
  z.tile = [](int64_t n, int prec) { return tc_tuned_batched_tile_prec(n, prec); };
  z.solve_ws = [](int64_t n, int64_t nrhs) { return tc_solve_many_ws_bytes(n, nrhs); };
  z.header = tc_ws_header_bytes();
  // an item's descriptor and solve job, and room for the solve launch's two
  // counters after the last job
  z.desc = (int64_t)(sizeof(SrvDesc) + sizeof(TcSolveJob) + 16);
  return z;
}

void worker_main(TcServer* Sp) {
  TcServer& S = *Sp;
  (void)hipSetDevice(S.device);
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
      if (S.stop && S.core->idle()) return;
    }
    // admission and launch (at most two ticks in flight, one in FIFO mode)
    Flight f;
    bool have = false;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      const int max_inflight = S.mode == 0 ? 2 : 1;
      if ((int)S.inflight.size() < max_inflight && S.error == 0) {
        have = S.core->admit(f.t, now_ns());
        if (have)
          for (const tcs::TickItem& it : f.t.items) f.rq.push_back(&S.core->req(it.req));
        (void)S.core->take_finished();  // requests rejected at admission are final
        S.cv.notify_all();
      }
    }
    if (have) {
      if (hipEventCreateWithFlags(&f.done, hipEventDisableTiming) != hipSuccess || !launch_tick(S, f)) {
        std::unique_lock<std::mutex> lk(S.mu);
        S.error = 1;
        S.cv.notify_all();
        return;
      }
      std::unique_lock<std::mutex> lk(S.mu);
      S.inflight.push_back(f);
      ++S.ticks;
      did = true;
    }
    if (!did) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}
}  // namespace

// The precision plan of served requests (tuning/batched_tiles.json, "serve").
static tcs::PlanTable tc_serve_plan_table() {
  tcs::PlanTable t;
  t.fp32_min_n_loose = TC_SERVE_FP32_MIN_N_LOOSE;
  t.fp32_min_n_strict = TC_SERVE_FP32_MIN_N_STRICT;
  t.loose_tol = TC_SERVE_LOOSE_TOL;
  t.fp32_corr = TC_SERVE_FP32_CORRECTIONS;
  return t;
}

// ---------------------------------------------------------------- entry points
int tc_server_create(void* arena, int64_t arena_bytes, int64_t pinned_bytes, int mode, int64_t max_per_tick,
                     int64_t wait_ticks, TcServer** out) {
  auto S = std::make_unique<TcServer>();
  if (hipGetDevice(&S->device) != hipSuccess) return TC_LAUNCH_EDEVICE;
  S->arena = (char*)arena;
  void* p = nullptr;
  if (hipHostMalloc(&p, r256(pinned_bytes), hipHostMallocDefault) != hipSuccess) return TC_LAUNCH_EDEVICE;
  S->pinned = (char*)p;
  S->mode = mode;
  S->wait_ticks = wait_ticks;
  S->core = std::make_unique<tcs::Core>(arena_bytes, r256(pinned_bytes), mode, max_per_tick, make_sizer(),
                                        tc_serve_plan_table());
  for (int k = 0; k < 2; ++k)
    if (hipStreamCreateWithFlags(&S->st[k], hipStreamNonBlocking) != hipSuccess) return TC_LAUNCH_EDEVICE;
  S->worker = std::thread(worker_main, S.get());
  *out = S.release();
  return 0;
}

int tc_server_submit(TcServer* S, const double* pts, int64_t n, double lengthscale, double nugget, const double* B,
                     int64_t nrhs, double tol, int keep, int64_t* id) {
  std::vector<double> P(pts, pts + 2 * n), Bv(B, B + n * nrhs);
  const int64_t t = now_ns();
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->error) return TC_LAUNCH_EDEVICE;
  *id = S->core->submit_factor(std::move(P), n, lengthscale, nugget, std::move(Bv), nrhs, tol, keep != 0, t);
  return 0;
}

int tc_server_submit_solve(TcServer* S, int64_t factor, const double* B, int64_t n, int64_t nrhs, double tol,
                           int64_t* id) {
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->error) return TC_LAUNCH_EDEVICE;
  auto it = S->core->factors().find(factor);
  if (it == S->core->factors().end()) return TC_LAUNCH_ENOFACTOR;
  if (it->second.n != n) return TC_LAUNCH_EINVAL;
  std::vector<double> Bv(B, B + n * nrhs);
  const int64_t r = S->core->submit_solve(factor, std::move(Bv), nrhs, tol, now_ns());
  if (r < 0) return TC_LAUNCH_ENOFACTOR;
  *id = r;
  return 0;
}

// Returns the request state after waiting up to timeout_s (tcs::ST_*: 2
// done within its tolerance, 5 done but above it, 3 not SPD, 4 rejected, 6 a
// dependency wait of its factorization (info = 1 + the unit's ticket) or of
// a solve sweep (info = -1) ran out, 0/1 still pending / running), or < 0
// on a device error.
int tc_server_wait(TcServer* S, int64_t id, double timeout_s, double* X, double* eta, double* latency_s,
                   int64_t* info) {
  std::unique_lock<std::mutex> lk(S->mu);
  if (id < 0 || id >= S->core->num_requests()) return TC_LAUNCH_EINVAL;
  tcs::Request& R = S->core->req(id);
  S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return R.state >= 2 || S->error; });
  if (S->error && R.state < 2) return TC_LAUNCH_EDEVICE;
  if (R.state >= 2) {
    if (X && R.state == tcs::ST_DONE) memcpy(X, R.X.data(), 8 * R.n * R.nrhs);
    if (eta) *eta = R.eta;
    if (latency_s) *latency_s = (R.t_done - R.t_arrive) * 1e-9;
    if (info) *info = R.info;
    if (R.state == tcs::ST_DONE && !(R.eta <= R.tol)) return 5;
  }
  return R.state;
}

int tc_server_request_info(TcServer* S, int64_t id, int64_t* factor, int* prec, int* corrections, int* refactors) {
  std::unique_lock<std::mutex> lk(S->mu);
  if (id < 0 || id >= S->core->num_requests()) return TC_LAUNCH_EINVAL;
  const tcs::Request& R = S->core->req(id);
  if (factor) *factor = R.state == tcs::ST_DONE ? R.factor_id : -1;
  if (prec) *prec = R.prec;
  if (corrections) *corrections = R.corrections;
  if (refactors) *refactors = R.refactors;
  return R.state;
}

int tc_server_release_factor(TcServer* S, int64_t factor) {
  std::unique_lock<std::mutex> lk(S->mu);
  return S->core->release_factor(factor) ? 0 : TC_LAUNCH_ENOFACTOR;
}

int tc_server_set_plan(TcServer* S, int64_t fp32_min_n_loose, int64_t fp32_min_n_strict) {
  std::unique_lock<std::mutex> lk(S->mu);
  tcs::PlanTable p = S->core->plans();
  p.fp32_min_n_loose = fp32_min_n_loose;
  p.fp32_min_n_strict = fp32_min_n_strict;
  S->core->set_plans(p);
  return 0;
}

int64_t tc_server_ticks(TcServer* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  return S->ticks;
}

int64_t tc_server_evictions(TcServer* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  return S->core->evictions();
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
  for (Flight& f : S->inflight)
    if (f.done) (void)hipEventDestroy(f.done);
  for (int k = 0; k < 2; ++k)
    if (S->st[k]) (void)hipStreamDestroy(S->st[k]);
  if (S->pinned) (void)hipHostFree(S->pinned);
  delete S;
  return rc;
}
