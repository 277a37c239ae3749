// launch.h -- internal interface between the C ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TC_LAUNCH_EDEVICE (-2)
#define TC_LAUNCH_ETIMEOUT (-4)
#define TC_LAUNCH_ENOFACTOR (-6)

// Tile side of the plain factorization when the caller gives none (measured
// on MI355X, fork-join: small orders are launch-bound and prefer short
// panels, large ones deep updates).
inline int64_t tc_default_tile(int64_t n) { return n <= 8192 ? 128 : 1024; }
#define TC_LAUNCH_EINVAL (-1)

// Workspace bytes chol_factor needs (every schedule uses one layout).
int64_t tc_ws_bytes(int64_t n, int64_t T);
// The device-resident factorization workspace of chol_factor_noalloc: its
// size, and its address on the current device (looked up once per device;
// nullptr on a runtime error).
#define TC_SCRATCH_BYTES ((4 << 20) + (64 << 10))
int64_t tc_scratch_bytes();
void* tc_scratch_ptr();
// Enqueue one factorization.  sched_flags: schedule 0 fork-join, 1 async
// DAG, 2 naive fork-join, 3 synchronous tasking, 4 fork-join with lookahead,
// 5 HIP-graph DAG, optionally ORed with
// TC_SCHED_NOOP (empty unit bodies, for measuring the schedule's own cost).
// grid: persistent workgroups (1 and 3); wait_ticks: wait limit in
// wall-clock ticks (1 and 3); chunk: bulk units after each panel-chain link
// in the ticket order (1).
#define TC_SCHED_NOOP 0x100
int tc_launch_factor(double* A, int64_t n, int64_t lda, int64_t T, int sched_flags, void* work, hipStream_t st,
                     int64_t grid, int64_t wait_ticks, int64_t chunk);
// Per-launch timing of tc_launch_factor on the calling thread (measurement
// aid): enable takes a mask of the kinds to time (bit k for kind k) and
// returns the previous mask; read synchronises `st`, sums the
// recorded launch times per kind (POTRF, TRSM, UPDATE, PANEL unit launches,
// then the persistent launch, then the lookahead schedule's second-stream
// trailing updates) and clears.
#define TC_TIMING_KINDS 6
#define TC_TIMING_PERSISTENT 4
#define TC_TIMING_REST 5
int tc_timing_enable(int mask);
int tc_timing_read(hipStream_t st, double ms[TC_TIMING_KINDS], int64_t cnt[TC_TIMING_KINDS]);
// Mixed precision (fork-join): prec 0 FP64, 1 FP32, 2 BF16 trailing
// products; scale: symmetric diagonal scaling around the factorization;
// shift added to the (scaled) diagonal first.  Workspace: tc_ws_mixed_bytes.
int64_t tc_ws_mixed_bytes(int64_t n, int64_t T, int prec);
int64_t tc_lp_ld(int64_t T);
int tc_launch_factor_mixed(double* A, int64_t n, int64_t lda, int64_t T, int prec, int scale, double shift,
                           void* work, hipStream_t st);
// Synchronise the stream and read the error flag / info of a workspace.
int tc_read_status(const void* work, hipStream_t st, int32_t* error, int64_t* info);
// Co-resident workgroups of the persistent kernels on the current device.
int64_t tc_async_grid_size();
int64_t tc_sync_grid_size();
// Workspace bytes of the solve of nrhs right-hand sides of order n: block
// tickets, done counters and a status word, then the two sweeps' payloads
// (inv: the sweeps with inverted diagonal blocks).
int64_t tc_solve_ws_bytes(int64_t n, int64_t nrhs, bool inv);
// The status word: cleared by tc_solve_status_reset (enqueued), set when a
// sweep's dependency wait runs out, kept by the launches below (which clear
// only their counters) until the next reset; tc_solve_status synchronises
// `st` and reads it; tc_solve_status_offset is its byte offset.
int tc_solve_status_reset(void* work, hipStream_t st);
int tc_solve_status(const void* work, hipStream_t st, int32_t* error);
int64_t tc_solve_status_offset();
// Enqueue forward + backward substitution (64-row blocks).
int tc_launch_solve(const double* L, int64_t n, int64_t lda, int64_t T, double* B, int64_t nrhs, int64_t ldb,
                    void* work, hipStream_t st, int64_t wait_ticks);
// Several independent solves in one launch pair (a serving tick's items):
// job j's sweeps take the tickets [first, first + tc_solve_many_tickets(n,
// nrhs)) of the launch, in passes of four; `work` is the job's own workspace
// of tc_solve_many_ws_bytes(n, nrhs) bytes (its status word where
// tc_solve_status_offset says).  B is n x nrhs row-major with leading
// dimension ldb; L has leading dimension lda.
struct TcSolveJob {
  const double* L;
  double* B;
  void* work;
  int64_t n, lda, nrhs, ldb;
  int64_t first;
};
int64_t tc_solve_many_ws_bytes(int64_t n, int64_t nrhs);
int64_t tc_solve_many_tickets(int64_t n, int64_t nrhs);
// jobs: device array of `count` jobs in ticket order; tickets: their total;
// max_entries: the largest job's forward payload entries (the fill's
// width); ctr: two int32 of device memory for the launch's counters.
int tc_launch_solve_many(const TcSolveJob* jobs, int64_t count, int64_t tickets, int64_t max_entries, int32_t* ctr,
                         hipStream_t st, int64_t wait_ticks);
// Repeated solves with one factor: invert the 64 x 64 diagonal blocks and
// form the coupling blocks of neighbouring block rows once
// (tc_solve_inv_bytes of storage), then sweep with one matrix-core product
// per block step on the chain.
int64_t tc_solve_inv_bytes(int64_t n);
int tc_launch_invert_diag(const double* L, int64_t n, int64_t lda, double* Dinv, hipStream_t st);
int tc_launch_solve_inv(const double* L, int64_t n, int64_t lda, const double* Dinv, double* B, int64_t nrhs,
                        int64_t ldb, void* work, hipStream_t st, int64_t wait_ticks);
// Refinement of A X = B with a (low-precision) factor: method 0 iterative
// refinement, 1 preconditioned CG.  Synchronises `st` once per iteration.
// Returns 0 converged, 1 not converged, TC_LAUNCH_ETIMEOUT when a sweep's
// dependency wait ran out (X unspecified), other < 0 device errors.
int64_t tc_refine_ws_bytes(int64_t n, int64_t nrhs);
int tc_refine(const double* A, int64_t lda, const double* L, int64_t ldl, int64_t n, int64_t T, const double* B,
              int64_t ldb, double* X, int64_t ldx, int64_t nrhs, int method, double tol, int64_t max_iter, void* work,
              hipStream_t st, int64_t wait_ticks, int64_t* iters, double* eta_out);
// Batched: many matrices in one persistent launch (b null: factor only,
// else one right-hand side per matrix, solved in place after its factor).
// Matrices with n <= 0 are skipped.  chunk: ticket-order lookahead of each
// matrix (as for the asynchronous schedule).
// Mixed precision and refinement of a batched launch (all optional):
//   prec      per-matrix trailing-product precision (TC_PREC_FP64 / FP32),
//             null = FP64;
//   A0, lda0  originals: with them the launch first copies each lower
//             triangle A0 -> A (A is then the factor's storage) and b0 -> b,
//             and every solve unit refines against A0 and b0 to tol (at most
//             max_iter corrections).
struct TcBatchMixed {
  const int32_t* prec = nullptr;
  const double* const* A0 = nullptr;
  const int64_t* lda0 = nullptr;
  const double* const* b0 = nullptr;
  double tol = 0.0;
  int64_t max_iter = 0;
};
int64_t tc_batched_ws_bytes(int64_t batch, const int64_t* n, const int64_t* T, int solve, int64_t chunk,
                            const int32_t* prec = nullptr, bool refine = false);
// nrhs / ldb: right-hand sides per matrix (n x nrhs row-major, leading
// dimension ldb); null means one right-hand side, contiguous.
int tc_launch_batched(double* const* A, double* const* b, const int64_t* n, const int64_t* lda, const int64_t* T,
                      int64_t batch, void* work, hipStream_t st, int64_t grid, int64_t wait_ticks, int64_t chunk,
                      const int64_t* nrhs = nullptr, const int64_t* ldb = nullptr, const TcBatchMixed* mx = nullptr);
// Refinement statistics {eta, corrections} of every matrix (synchronises).
int tc_read_batched_stats(const void* work, int64_t batch, const int64_t* n, const int64_t* T, int64_t chunk,
                          const int32_t* prec, hipStream_t st, double* eta, int64_t* iters);
int tc_read_batched_status(const void* work, int64_t batch, hipStream_t st, int32_t* error, int64_t* info);
int64_t tc_batched_grid_size();
// Status header of a factorization workspace: its size, and decoding a host
// copy of it.
int64_t tc_ws_header_bytes();
void tc_ws_header_read(const void* hdr, int32_t* error, int64_t* info);
// Serving with continuous batching (serve.hip; bookkeeping in serve_core.h).
// mode 0 continuous batching, 1 one request at a time.
struct TcServer;
int tc_server_create(void* arena, int64_t arena_bytes, int64_t pinned_bytes, int mode, int64_t max_per_tick,
                     int64_t wait_ticks, TcServer** out);
int tc_server_submit(TcServer* S, const double* pts, int64_t n, double lengthscale, double nugget, const double* B,
                     int64_t nrhs, double tol, int keep, int64_t* id);
int tc_server_submit_solve(TcServer* S, int64_t factor, const double* B, int64_t n, int64_t nrhs, double tol,
                           int64_t* id);
int tc_server_wait(TcServer* S, int64_t id, double timeout_s, double* X, double* eta, double* latency_s,
                   int64_t* info);
int tc_server_request_info(TcServer* S, int64_t id, int64_t* factor, int* prec, int* corrections, int* refactors);
int tc_server_release_factor(TcServer* S, int64_t factor);
int tc_server_set_plan(TcServer* S, int64_t fp32_min_n_loose, int64_t fp32_min_n_strict);
int64_t tc_server_ticks(TcServer* S);
int64_t tc_server_evictions(TcServer* S);
int tc_server_destroy(TcServer* S);
