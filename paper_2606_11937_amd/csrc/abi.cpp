// abi.cpp -- the extern "C" entry points declared in include/tilechol.h:
// argument validation, workspace sizing and dispatch to the launchers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <new>
#include <vector>

#include "../../include/tilechol.h"
#include "dag.h"
#include "launch.h"
#include "tuned_tiles.h"

#define TC_PREC_FP64 0
#define TC_PREC_FP32 1
#define TC_PREC_BF16 2

static_assert(CHOL_PREC_FP64 == TC_PREC_FP64 && CHOL_PREC_FP32 == TC_PREC_FP32 && CHOL_PREC_BF16 == TC_PREC_BF16,
              "precision codes of the ABI and the kernels differ");
static_assert(CHOL_BLOCK == TC_BLK, "sub-block size of the ABI and the kernels differ");
static_assert(CHOL_NOALLOC_WORKSPACE == TC_SCRATCH_BYTES, "no-allocation workspace sizes of the ABI and the library differ");
static_assert(CHOL_UNIT_POTRF == TC_UNIT_POTRF && CHOL_UNIT_TRSM == TC_UNIT_TRSM &&
                  CHOL_UNIT_UPDATE == TC_UNIT_UPDATE && CHOL_UNIT_PANEL == TC_UNIT_PANEL,
              "unit kinds of the ABI and the kernels differ");
static_assert(CHOL_SCHED_FORK_JOIN == 0 && CHOL_SCHED_ASYNC_DAG == 1 && CHOL_SCHED_FORK_JOIN_NAIVE == 2 &&
                  CHOL_SCHED_TASK_SYNC == 3 && CHOL_SCHED_FORK_JOIN_LOOKAHEAD == 4 && CHOL_SCHED_GRAPH_DAG == 5 &&
                  CHOL_SCHED_NOOP == TC_SCHED_NOOP,
              "schedule codes of the ABI and the launcher differ");
static_assert(TC_TIMING_KINDS == CHOL_TIMING_KINDS && TC_TIMING_PERSISTENT == 4 && TC_TIMING_REST == 5,
              "timing kinds of the ABI and the launcher differ");

namespace {
thread_local int g_bad_arg = 0;
std::atomic<double> g_wait_limit_s{10.0};
std::atomic<int64_t> g_lookahead{-1};

int bad(int idx, int code = CHOL_EINVAL) {
  g_bad_arg = idx;
  return code;
}
inline int64_t max1(int64_t x) { return x > 1 ? x : 1; }
// Largest order / leading dimension: the staging loads address one
// 128-row block with 32-bit byte offsets.
const int64_t kMaxN = (int64_t)1 << 20;

int64_t wait_ticks() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
  const double t = g_wait_limit_s.load() * 1e3 * (double)khz;
  return t > 9e18 ? (int64_t)9e18 : (int64_t)t;
}

int status_from(int32_t err, int64_t dinfo, int64_t* info) {
  // err 1: dinfo is the failing column + 1; err 2: 1 + the ticket of the
  // unit whose dependency wait ran out (persistent schedules), else 0
  if (info) *info = (err == 1 || err == 2) ? dinfo : 0;
  if (err == 1) return CHOL_NOT_SPD;
  if (err == 2) return CHOL_ETIMEOUT;
  return CHOL_OK;
}

bool sched_valid(int sched) {
  const int base = sched & 0xff, flags = sched & ~0xff;
  return base >= CHOL_SCHED_FORK_JOIN && base <= CHOL_SCHED_GRAPH_DAG && (flags & ~CHOL_SCHED_NOOP) == 0;
}

int check_factor_args(double* A, int64_t n, int64_t lda, int64_t T, int sched) {
  if (n < 0 || n > kMaxN) return bad(2);
  if (lda < max1(n) || lda > kMaxN) return bad(3);
  if (T < 1) return bad(4);
  if (!sched_valid(sched)) return bad(5);
  if ((sched & 0xff) == CHOL_SCHED_ASYNC_DAG && n > 0 && tc_cdiv(n, T) > CHOL_ASYNC_MAX_TILES) return bad(4);
  if (n > 0 && A == nullptr) return bad(1);
  return CHOL_OK;
}
}  // namespace

extern "C" {

int chol_last_bad_arg(void) { return g_bad_arg; }

const char* chol_status_str(int status) {
  switch (status) {
    case CHOL_OK: return "success";
    case CHOL_NOT_SPD: return "matrix is not positive definite (see info)";
    case CHOL_EINVAL: return "invalid argument (see chol_last_bad_arg)";
    case CHOL_EDEVICE: return "HIP runtime error";
    case CHOL_EWORKSPACE: return "workspace too small";
    case CHOL_ETIMEOUT: return "dependency wait exceeded the wait limit";
    case CHOL_ESTALLED: return "a served request's dependency wait exceeded the wait limit (see info)";
    case CHOL_ENOFACTOR: return "no such resident factor (never kept, released or evicted)";
    case CHOL_NOT_CONVERGED: return "refinement did not reach the tolerance within max_iter";
    default: return "unknown status";
  }
}

double chol_set_wait_limit(double seconds) {
  if (!(seconds >= 0.0)) return -1.0;
  return g_wait_limit_s.exchange(seconds);
}

int64_t chol_set_lookahead(int64_t units) { return g_lookahead.exchange(units < 0 ? -1 : units); }

int64_t chol_default_tile(int64_t n) { return tc_default_tile(n); }

int64_t chol_factor_workspace_size(int64_t n, int64_t T, int sched) {
  g_bad_arg = 0;
  if (n < 0 || n > kMaxN) return bad(1);
  if (T < 1) return bad(2);
  if (!sched_valid(sched)) return bad(3);
  return tc_ws_bytes(n > 0 ? n : 1, T);
}

int chol_factor(double* A, int64_t n, int64_t lda, int64_t T, int sched, void* work, int64_t work_bytes,
                void* stream, int64_t* info) {
  g_bad_arg = 0;
  if (int e = check_factor_args(A, n, lda, T, sched)) return e;
  if (n == 0) {
    if (info) *info = 0;
    return CHOL_OK;
  }
  if (work == nullptr) return bad(6);
  if (work_bytes < tc_ws_bytes(n, T)) return bad(7, CHOL_EWORKSPACE);
  hipStream_t st = (hipStream_t)stream;
  int64_t grid = 0;
  if ((sched & 0xff) == CHOL_SCHED_ASYNC_DAG || (sched & 0xff) == CHOL_SCHED_TASK_SYNC) {
    grid = (sched & 0xff) == CHOL_SCHED_ASYNC_DAG ? tc_async_grid_size() : tc_sync_grid_size();
    if (grid <= 0) return CHOL_EDEVICE;
  }
  if (tc_launch_factor(A, n, lda, T, sched, work, st, grid, wait_ticks(), tc_lookahead_chunk(grid, g_lookahead.load())) != 0)
    return CHOL_EDEVICE;
  if (info == nullptr) return CHOL_OK;
  int32_t err = 0;
  int64_t dinfo = 0;
  if (tc_read_status(work, st, &err, &dinfo) != 0) return CHOL_EDEVICE;
  return status_from(err, dinfo, info);
}

int chol_factor_noalloc(double* A, int64_t n, int64_t lda, int64_t T, int sched, void* stream, int64_t* info) {
  g_bad_arg = 0;
  if (int e = check_factor_args(A, n, lda, T, sched)) return e;
  const int base = sched & 0xff;
  if (base != CHOL_SCHED_FORK_JOIN && base != CHOL_SCHED_ASYNC_DAG) return bad(5);
  if (n == 0) {
    if (info) *info = 0;
    return CHOL_OK;
  }
  if (tc_ws_bytes(n, T) > tc_scratch_bytes()) return bad(2, CHOL_EWORKSPACE);
  void* work = tc_scratch_ptr();
  if (work == nullptr) return CHOL_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  int64_t grid = 0;
  if (base == CHOL_SCHED_ASYNC_DAG) {
    grid = tc_async_grid_size();
    if (grid <= 0) return CHOL_EDEVICE;
  }
  if (tc_launch_factor(A, n, lda, T, sched, work, st, grid, wait_ticks(), tc_lookahead_chunk(grid, g_lookahead.load())) != 0)
    return CHOL_EDEVICE;
  if (info == nullptr) return CHOL_OK;
  int32_t err = 0;
  int64_t dinfo = 0;
  if (tc_read_status(work, st, &err, &dinfo) != 0) return CHOL_EDEVICE;
  return status_from(err, dinfo, info);
}

int chol_factor_info(const void* work, void* stream, int64_t* info) {
  g_bad_arg = 0;
  if (work == nullptr) return bad(1);
  if (info == nullptr) return bad(3);
  int32_t err = 0;
  int64_t dinfo = 0;
  if (tc_read_status(work, (hipStream_t)stream, &err, &dinfo) != 0) return CHOL_EDEVICE;
  return status_from(err, dinfo, info);
}

int64_t chol_solve_workspace_size(int64_t n, int64_t T, int64_t nrhs) {
  g_bad_arg = 0;
  if (n < 0 || n > kMaxN) return bad(1);
  if (T < 1) return bad(2);
  if (nrhs < 0) return bad(3);
  return tc_solve_ws_bytes(n, nrhs, false);
}

int chol_solve(const double* L, int64_t n, int64_t lda, int64_t T, double* B, int64_t nrhs, int64_t ldb, void* work,
               int64_t work_bytes, void* stream) {
  g_bad_arg = 0;
  if (n < 0 || n > kMaxN) return bad(2);
  if (lda < max1(n) || lda > kMaxN) return bad(3);
  if (T < 1) return bad(4);
  if (nrhs < 0) return bad(6);
  if (ldb < max1(nrhs)) return bad(7);
  if (n == 0 || nrhs == 0) return CHOL_OK;
  if (L == nullptr) return bad(1);
  if (B == nullptr) return bad(5);
  if (work == nullptr) return bad(8);
  if (work_bytes < tc_solve_ws_bytes(n, nrhs, false)) return bad(9, CHOL_EWORKSPACE);
  hipStream_t st = (hipStream_t)stream;
  if (tc_solve_status_reset(work, st) != 0) return CHOL_EDEVICE;
  return tc_launch_solve(L, n, lda, T, B, nrhs, ldb, work, st, wait_ticks()) == 0 ? CHOL_OK : CHOL_EDEVICE;
}

int chol_solve_info(const void* work, void* stream) {
  g_bad_arg = 0;
  if (work == nullptr) return bad(1);
  int32_t err = 0;
  if (tc_solve_status((void*)work, (hipStream_t)stream, &err) != 0) return CHOL_EDEVICE;
  return err ? CHOL_ETIMEOUT : CHOL_OK;
}

int64_t chol_factor_mixed_workspace_size(int64_t n, int64_t T, int prec) {
  g_bad_arg = 0;
  if (n < 0 || n > kMaxN) return bad(1);
  if (T < 1) return bad(2);
  if (prec < CHOL_PREC_FP64 || prec > CHOL_PREC_BF16) return bad(3);
  return tc_ws_mixed_bytes(n > 0 ? n : 1, T, prec);
}

int chol_factor_mixed(double* A, int64_t n, int64_t lda, int64_t T, int prec, int flags, double shift, void* work,
                      int64_t work_bytes, void* stream, int64_t* info) {
  g_bad_arg = 0;
  if (int e = check_factor_args(A, n, lda, T, CHOL_SCHED_FORK_JOIN)) return e;
  if (prec < CHOL_PREC_FP64 || prec > CHOL_PREC_BF16) return bad(5);
  if ((flags & ~CHOL_MIXED_SCALE) != 0) return bad(6);
  if (!(shift >= 0.0) || shift > 1e300) return bad(7);
  if (n == 0) {
    if (info) *info = 0;
    return CHOL_OK;
  }
  if (work == nullptr) return bad(8);
  if (work_bytes < tc_ws_mixed_bytes(n, T, prec)) return bad(9, CHOL_EWORKSPACE);
  hipStream_t st = (hipStream_t)stream;
  if (tc_launch_factor_mixed(A, n, lda, T, prec, (flags & CHOL_MIXED_SCALE) ? 1 : 0, shift, work, st) != 0)
    return CHOL_EDEVICE;
  if (info == nullptr) return CHOL_OK;
  int32_t err = 0;
  int64_t dinfo = 0;
  if (tc_read_status(work, st, &err, &dinfo) != 0) return CHOL_EDEVICE;
  return status_from(err, dinfo, info);
}

int64_t chol_refine_workspace_size(int64_t n, int64_t T, int64_t nrhs) {
  g_bad_arg = 0;
  if (n < 0 || n > kMaxN) return bad(1);
  if (T < 1) return bad(2);
  if (nrhs < 0) return bad(3);
  return tc_refine_ws_bytes(n > 0 ? n : 1, nrhs > 0 ? nrhs : 1);
}

int chol_solve_refine(const double* A, int64_t lda, const double* L, int64_t ldl, int64_t n, int64_t T,
                      const double* B, int64_t ldb, double* X, int64_t ldx, int64_t nrhs, int method, double tol,
                      int64_t max_iter, void* work, int64_t work_bytes, void* stream, int64_t* iters, double* eta) {
  g_bad_arg = 0;
  if (n < 0 || n > kMaxN) return bad(5);
  if (lda < max1(n) || lda > kMaxN) return bad(2);
  if (ldl < max1(n) || ldl > kMaxN) return bad(4);
  if (T < 1) return bad(6);
  if (nrhs < 0) return bad(11);
  if (ldb < max1(nrhs)) return bad(8);
  if (ldx < max1(nrhs)) return bad(10);
  if (method != CHOL_REFINE_IR && method != CHOL_REFINE_PCG) return bad(12);
  if (!(tol > 0.0)) return bad(13);
  if (max_iter < 0) return bad(14);
  if (iters) *iters = 0;
  if (n == 0 || nrhs == 0) return CHOL_OK;
  if (A == nullptr) return bad(1);
  if (L == nullptr) return bad(3);
  if (B == nullptr) return bad(7);
  if (X == nullptr) return bad(9);
  if (work == nullptr) return bad(15);
  if (work_bytes < tc_refine_ws_bytes(n, nrhs)) return bad(16, CHOL_EWORKSPACE);
  const int r = tc_refine(A, lda, L, ldl, n, T, B, ldb, X, ldx, nrhs, method, tol, max_iter, work,
                          (hipStream_t)stream, wait_ticks(), iters, eta);
  if (r == TC_LAUNCH_ETIMEOUT) return CHOL_ETIMEOUT;
  if (r < 0) return CHOL_EDEVICE;
  return r == 0 ? CHOL_OK : CHOL_NOT_CONVERGED;
}

int64_t chol_batched_tile(int64_t n, int prec) {
  g_bad_arg = 0;
  if (prec != CHOL_PREC_FP64 && prec != CHOL_PREC_FP32) return bad(2);
  if (n < 0) return bad(1);
  return tc_tuned_batched_tile_prec(n, prec);
}

namespace {
// tile sides of a batch (given, or the tuned choice per n)
bool batch_tiles(int64_t batch, const int64_t* n, const int64_t* T, std::vector<int64_t>& t) {
  t.resize(batch);
  for (int64_t i = 0; i < batch; ++i) {
    t[i] = T ? T[i] : tc_tuned_batched_tile(n[i] > 0 ? n[i] : 1);
    if (t[i] < 1) return false;
  }
  return true;
}
int64_t batch_chunk() {
  const int64_t grid = tc_batched_grid_size();
  return tc_lookahead_chunk(grid > 0 ? grid : 1, g_lookahead.load());
}
int64_t batched_ws(int64_t batch, const int64_t* n, const int64_t* T, int solve) {
  g_bad_arg = 0;
  if (batch < 0) return bad(1);
  if (batch > 0 && n == nullptr) return bad(2);
  for (int64_t i = 0; i < batch; ++i)
    if (n[i] < 0 || n[i] > kMaxN) return bad(2);
  std::vector<int64_t> t;
  if (!batch_tiles(batch, n, T, t)) return bad(3);
  for (int64_t i = 0; i < batch; ++i)
    if (n[i] > 0 && tc_cdiv(n[i], t[i]) > CHOL_ASYNC_MAX_TILES) return bad(3);
  return tc_batched_ws_bytes(batch, n, t.data(), solve, batch_chunk());
}
int batched_run(double* const* A, double* const* B, const int64_t* n, const int64_t* lda, int64_t batch,
                const int64_t* T, void* work, int64_t work_bytes, void* stream, int64_t* info, int iA, int iB,
                int in, int ilda, int ibatch, int iT, int iwork, int iwb) {
  g_bad_arg = 0;
  if (batch < 0) return bad(ibatch);
  if (batch == 0) return CHOL_OK;
  if (A == nullptr) return bad(iA);
  if (n == nullptr) return bad(in);
  if (lda == nullptr) return bad(ilda);
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] < 0 || n[i] > kMaxN) return bad(in);
    if (lda[i] < max1(n[i]) || lda[i] > kMaxN) return bad(ilda);
    if (n[i] > 0 && A[i] == nullptr) return bad(iA);
    if (B != nullptr && n[i] > 0 && B[i] == nullptr) return bad(iB);
  }
  std::vector<int64_t> t;
  if (!batch_tiles(batch, n, T, t)) return bad(iT);
  for (int64_t i = 0; i < batch; ++i)
    if (n[i] > 0 && tc_cdiv(n[i], t[i]) > CHOL_ASYNC_MAX_TILES) return bad(iT);
  const int64_t chunk = batch_chunk();
  const int64_t need = tc_batched_ws_bytes(batch, n, t.data(), B != nullptr, chunk);
  if (work == nullptr) return bad(iwork);
  if (work_bytes < need) return bad(iwb, CHOL_EWORKSPACE);
  const int64_t grid = tc_batched_grid_size();
  if (grid <= 0) return CHOL_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (tc_launch_batched(A, B, n, lda, t.data(), batch, work, st, grid, wait_ticks(), chunk) != 0)
    return CHOL_EDEVICE;
  if (info == nullptr) return CHOL_OK;
  std::vector<int32_t> err(batch);
  std::vector<int64_t> dinfo(batch);
  if (tc_read_batched_status(work, batch, st, err.data(), dinfo.data()) != 0) return CHOL_EDEVICE;
  int worst = CHOL_OK;
  for (int64_t i = 0; i < batch; ++i) {
    const int s = status_from(err[i], dinfo[i], &info[i]);
    if (n[i] <= 0) info[i] = 0;
    if (s == CHOL_ETIMEOUT) worst = CHOL_ETIMEOUT;
    else if (s != CHOL_OK && worst == CHOL_OK) worst = s;
  }
  return worst;
}
}  // namespace

int64_t chol_factor_batched_workspace_size(int64_t batch, const int64_t* n, const int64_t* T) {
  return batched_ws(batch, n, T, 0);
}

int chol_factor_batched(double* const* A, const int64_t* n, const int64_t* lda, int64_t batch, const int64_t* T,
                        void* work, int64_t work_bytes, void* stream, int64_t* info) {
  return batched_run(A, nullptr, n, lda, batch, T, work, work_bytes, stream, info, 1, 0, 2, 3, 4, 5, 6, 7);
}

int64_t chol_factor_solve_batched_workspace_size(int64_t batch, const int64_t* n, const int64_t* T) {
  return batched_ws(batch, n, T, 1);
}

int chol_factor_solve_batched(double* const* A, double* const* B, const int64_t* n, const int64_t* lda,
                              int64_t batch, const int64_t* T, void* work, int64_t work_bytes, void* stream,
                              int64_t* info) {
  if (B == nullptr) {
    g_bad_arg = 2;
    return CHOL_EINVAL;
  }
  return batched_run(A, B, n, lda, batch, T, work, work_bytes, stream, info, 1, 2, 3, 4, 5, 6, 7, 8);
}

namespace {
// per-matrix precision and tile side of a mixed batched call (given, or the
// tuned choice per (n, precision))
bool mixed_plan(int64_t batch, const int64_t* n, const int64_t* T, const int* prec, std::vector<int32_t>& p,
                std::vector<int64_t>& t) {
  p.resize(batch);
  t.resize(batch);
  for (int64_t i = 0; i < batch; ++i) {
    p[i] = prec ? prec[i] : CHOL_PREC_FP64;
    if (p[i] != CHOL_PREC_FP64 && p[i] != CHOL_PREC_FP32) return false;
    t[i] = T ? T[i] : tc_tuned_batched_tile_prec(n[i] > 0 ? n[i] : 1, p[i]);
  }
  return true;
}
bool mixed_tiles_ok(int64_t batch, const int64_t* n, const std::vector<int32_t>& p, const std::vector<int64_t>& t) {
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] <= 0) continue;
    if (t[i] < 1 || tc_cdiv(n[i], t[i]) > CHOL_ASYNC_MAX_TILES) return false;
    // the FP32 panel copy is read in 16-byte pieces from column J T on
    if (p[i] == CHOL_PREC_FP32 && t[i] < n[i] && t[i] % 4 != 0) return false;
  }
  return true;
}
}  // namespace

int64_t chol_factor_solve_batched_mixed_workspace_size(int64_t batch, const int64_t* n, const int64_t* T,
                                                       const int* prec) {
  g_bad_arg = 0;
  if (batch < 0) return bad(1);
  if (batch > 0 && n == nullptr) return bad(2);
  for (int64_t i = 0; i < batch; ++i)
    if (n[i] < 0 || n[i] > kMaxN) return bad(2);
  std::vector<int32_t> p;
  std::vector<int64_t> t;
  if (!mixed_plan(batch, n, T, prec, p, t)) return bad(4);
  if (!mixed_tiles_ok(batch, n, p, t)) return bad(3);
  return tc_batched_ws_bytes(batch, n, t.data(), 1, batch_chunk(), p.data(), true);
}

int chol_factor_solve_batched_mixed(const double* const* A, double* const* L, const double* const* B,
                                    double* const* X, const int64_t* n, const int64_t* lda, const int64_t* ldl,
                                    int64_t batch, const int64_t* T, const int* prec, double tol, int64_t max_iter,
                                    void* work, int64_t work_bytes, void* stream, int64_t* info, int64_t* iters,
                                    double* eta) {
  g_bad_arg = 0;
  if (batch < 0) return bad(8);
  if (!(tol > 0.0)) return bad(11);
  if (max_iter < 0) return bad(12);
  if (batch == 0) return CHOL_OK;
  if (A == nullptr) return bad(1);
  if (L == nullptr) return bad(2);
  if (B == nullptr) return bad(3);
  if (X == nullptr) return bad(4);
  if (n == nullptr) return bad(5);
  if (lda == nullptr) return bad(6);
  if (ldl == nullptr) return bad(7);
  for (int64_t i = 0; i < batch; ++i) {
    if (n[i] < 0 || n[i] > kMaxN) return bad(5);
    if (lda[i] < max1(n[i]) || lda[i] > kMaxN) return bad(6);
    if (ldl[i] < max1(n[i]) || ldl[i] > kMaxN) return bad(7);
    if (n[i] == 0) continue;
    if (A[i] == nullptr) return bad(1);
    if (L[i] == nullptr || (const double*)L[i] == A[i]) return bad(2);  // the original stays for the residuals
    if (B[i] == nullptr) return bad(3);
    if (X[i] == nullptr) return bad(4);
  }
  std::vector<int32_t> p;
  std::vector<int64_t> t;
  if (!mixed_plan(batch, n, T, prec, p, t)) return bad(10);
  if (!mixed_tiles_ok(batch, n, p, t)) return bad(9);
  const int64_t chunk = batch_chunk();
  const int64_t need = tc_batched_ws_bytes(batch, n, t.data(), 1, chunk, p.data(), true);
  if (work == nullptr) return bad(13);
  if (work_bytes < need) return bad(14, CHOL_EWORKSPACE);
  const int64_t grid = tc_batched_grid_size();
  if (grid <= 0) return CHOL_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  TcBatchMixed mx;
  mx.prec = p.data();
  mx.A0 = A;
  mx.lda0 = lda;
  mx.b0 = B;
  mx.tol = tol;
  mx.max_iter = max_iter;
  if (tc_launch_batched(L, X, n, ldl, t.data(), batch, work, st, grid, wait_ticks(), chunk, nullptr, nullptr, &mx) != 0)
    return CHOL_EDEVICE;
  if (info == nullptr) return CHOL_OK;
  std::vector<int32_t> err(batch);
  std::vector<int64_t> dinfo(batch);
  if (tc_read_batched_status(work, batch, st, err.data(), dinfo.data()) != 0) return CHOL_EDEVICE;
  std::vector<double> e(batch);
  std::vector<int64_t> it(batch);
  if (tc_read_batched_stats(work, batch, n, t.data(), chunk, p.data(), st, e.data(), it.data()) != 0)
    return CHOL_EDEVICE;
  int worst = CHOL_OK;
  for (int64_t i = 0; i < batch; ++i) {
    const int s = status_from(err[i], dinfo[i], &info[i]);
    if (n[i] <= 0) info[i] = 0;
    const bool solved = n[i] <= 0 || s == CHOL_OK;
    if (iters) iters[i] = n[i] > 0 && solved ? it[i] : 0;
    if (eta) eta[i] = n[i] > 0 && solved ? e[i] : 0.0;
    if (s == CHOL_ETIMEOUT) worst = CHOL_ETIMEOUT;
    else if (s != CHOL_OK && worst == CHOL_OK) worst = s;
    else if (s == CHOL_OK && worst == CHOL_OK && n[i] > 0 && !(e[i] <= tol)) worst = CHOL_NOT_CONVERGED;
  }
  return worst;
}

// ---------------------------------------------------------------- serving
struct chol_server {
  TcServer* s;
};

int chol_server_create(void* arena, int64_t arena_bytes, int64_t pinned_bytes, int mode, int64_t max_per_tick,
                       chol_server** server) {
  g_bad_arg = 0;
  if (arena == nullptr) return bad(1);
  if (arena_bytes < 4096) return bad(2);
  if (pinned_bytes < 4096) return bad(3);
  if (mode != CHOL_SERVE_CONTINUOUS && mode != CHOL_SERVE_FIFO) return bad(4);
  if (max_per_tick < 1 || max_per_tick > 65536) return bad(5);
  if (server == nullptr) return bad(6);
  TcServer* s = nullptr;
  if (tc_server_create(arena, arena_bytes, pinned_bytes, mode, max_per_tick, wait_ticks(), &s) != 0)
    return CHOL_EDEVICE;
  *server = new (std::nothrow) chol_server{s};
  if (*server == nullptr) {
    tc_server_destroy(s);
    return CHOL_EDEVICE;
  }
  return CHOL_OK;
}

int chol_server_submit(chol_server* server, const double* points, int64_t n, double lengthscale, double nugget,
                       const double* B, int64_t nrhs, double tol, int flags, int64_t* id) {
  g_bad_arg = 0;
  if (server == nullptr) return bad(1);
  if (points == nullptr) return bad(2);
  if (n < 1 || n > 65536) return bad(3);
  if (!(lengthscale > 0.0) || lengthscale > 1e300) return bad(4);
  if (!(nugget >= 0.0) || nugget > 1e300) return bad(5);
  if (B == nullptr) return bad(6);
  if (nrhs < 1 || nrhs > CHOL_SERVE_MAX_RHS) return bad(7);
  if (!(tol > 0.0)) return bad(8);
  if ((flags & ~CHOL_SERVE_KEEP) != 0) return bad(9);
  if (id == nullptr) return bad(10);
  return tc_server_submit(server->s, points, n, lengthscale, nugget, B, nrhs, tol, flags & CHOL_SERVE_KEEP, id) == 0
             ? CHOL_OK
             : CHOL_EDEVICE;
}

int chol_server_submit_solve(chol_server* server, int64_t factor, const double* B, int64_t n, int64_t nrhs,
                             double tol, int64_t* id) {
  g_bad_arg = 0;
  if (server == nullptr) return bad(1);
  if (B == nullptr) return bad(3);
  if (n < 1 || n > 65536) return bad(4);
  if (nrhs < 1 || nrhs > CHOL_SERVE_MAX_RHS) return bad(5);
  if (!(tol > 0.0)) return bad(6);
  if (id == nullptr) return bad(7);
  const int r = tc_server_submit_solve(server->s, factor, B, n, nrhs, tol, id);
  if (r == TC_LAUNCH_ENOFACTOR) return CHOL_ENOFACTOR;
  if (r == TC_LAUNCH_EINVAL) return bad(4);
  return r == 0 ? CHOL_OK : CHOL_EDEVICE;
}

int chol_server_request_info(chol_server* server, int64_t id, int64_t* factor, int* prec, int* corrections,
                             int* refactors) {
  g_bad_arg = 0;
  if (server == nullptr) return bad(1);
  const int st = tc_server_request_info(server->s, id, factor, prec, corrections, refactors);
  return st == TC_LAUNCH_EINVAL ? bad(2) : CHOL_OK;
}


int chol_server_release_factor(chol_server* server, int64_t factor) {
  g_bad_arg = 0;
  if (server == nullptr) return bad(1);
  return tc_server_release_factor(server->s, factor) == 0 ? CHOL_OK : CHOL_ENOFACTOR;
}

int chol_server_set_plan(chol_server* server, int64_t fp32_min_n_loose, int64_t fp32_min_n_strict) {
  g_bad_arg = 0;
  if (server == nullptr) return bad(1);
  if (fp32_min_n_loose < 1) return bad(2);
  if (fp32_min_n_strict < 1) return bad(3);
  return tc_server_set_plan(server->s, fp32_min_n_loose, fp32_min_n_strict) == 0 ? CHOL_OK : CHOL_EDEVICE;
}

int64_t chol_server_evictions(chol_server* server) {
  if (server == nullptr) return bad(1);
  return tc_server_evictions(server->s);
}

int chol_server_wait(chol_server* server, int64_t id, double timeout_s, double* X, double* eta, double* latency_s,
                     int64_t* info) {
  g_bad_arg = 0;
  if (server == nullptr) return bad(1);
  if (!(timeout_s >= 0.0)) return bad(3);
  const int st = tc_server_wait(server->s, id, timeout_s, X, eta, latency_s, info);
  switch (st) {
    case 2: return CHOL_OK;
    case 5: return CHOL_NOT_CONVERGED;
    case 3: return CHOL_NOT_SPD;
    case 4: return CHOL_EWORKSPACE;
    case 6: return CHOL_ESTALLED;
    case 0:
    case 1: return CHOL_ETIMEOUT;
    case TC_LAUNCH_EINVAL: return bad(2);
    default: return CHOL_EDEVICE;
  }
}

int64_t chol_server_ticks(chol_server* server) {
  if (server == nullptr) return bad(1);
  return tc_server_ticks(server->s);
}

int chol_server_destroy(chol_server* server) {
  if (server == nullptr) return CHOL_OK;
  const int rc = tc_server_destroy(server->s);
  delete server;
  return rc == 0 ? CHOL_OK : CHOL_EDEVICE;
}

int chol_dag_counts(int64_t n, int64_t T, int64_t counts[5]) {
  g_bad_arg = 0;
  if (n < 1 || n > kMaxN) return bad(1);
  if (T < 1) return bad(2);
  if (counts == nullptr) return bad(3);
  TcGeom g = tc_geom(n, T, 0);
  tc_task_counts(g, counts);
  int64_t total = 0;
  for (int32_t P = 0; P < g.M; ++P) total += tc_phase_size(g, P);
  counts[4] = total;
  return CHOL_OK;
}

int64_t chol_dag_enumerate(int64_t n, int64_t T, int64_t grid, int32_t* out, int64_t cap) {
  g_bad_arg = 0;
  if (n < 1 || n > kMaxN) return bad(1);
  if (T < 1) return bad(2);
  if (grid < 1) return bad(3);
  if (cap < 0) return bad(5);
  if (cap > 0 && out == nullptr) return bad(4);
  TcGeom g = tc_geom(n, T, tc_lookahead_chunk(grid, g_lookahead.load()));
  int64_t k = 0;
  for (int32_t P = 0; P < g.M; ++P) {
    const int64_t sz = tc_phase_size(g, P);
    for (int64_t r = 0; r < sz; ++r, ++k) {
      if (k < cap) {
        TcUnit u = tc_decode_in_phase(g, P, r);
        int32_t* o = out + 6 * k;
        o[0] = u.kind; o[1] = u.J; o[2] = u.I; o[3] = u.a; o[4] = u.K; o[5] = u.b;
      }
    }
  }
  return k;
}

int64_t chol_dag_forkjoin_update(int64_t n, int64_t T, int64_t J, int32_t* out, int64_t cap) {
  g_bad_arg = 0;
  if (n < 1 || n > kMaxN) return bad(1);
  if (T < 1) return bad(2);
  const TcGeom g = tc_geom(n, T, 0);
  if (J < 0 || J >= g.M) return bad(3);
  if (cap < 0) return bad(5);
  if (cap > 0 && out == nullptr) return bad(4);
  const int64_t total = tc_trailing_units(g, (int32_t)J);
  for (int64_t k = 0; k < total && k < cap; ++k) {
    const TcUnit u = tc_decode_trailing(g, (int32_t)J, (int32_t)J, k);
    int32_t* o = out + 6 * k;
    o[0] = u.kind; o[1] = u.J; o[2] = u.I; o[3] = u.a; o[4] = u.K; o[5] = u.b;
  }
  return total;
}

int chol_timing_enable(int kinds) { return tc_timing_enable(kinds); }

int chol_timing_read(void* stream, double ms[CHOL_TIMING_KINDS], int64_t launches[CHOL_TIMING_KINDS]) {
  g_bad_arg = 0;
  if (ms == nullptr) return bad(2);
  if (launches == nullptr) return bad(3);
  return tc_timing_read((hipStream_t)stream, ms, launches) == 0 ? CHOL_OK : CHOL_EDEVICE;
}

int64_t chol_async_grid(void) {
  const int64_t g = tc_async_grid_size();
  return g > 0 ? g : CHOL_EDEVICE;
}

}  // extern "C"
