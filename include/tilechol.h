/*
 * tilechol.h -- C ABI of the MI355X (gfx950) tiled Cholesky library.
 *
 * Operation (Methods, "Tiled Cholesky Decomposition"): the symmetric
 * positive-definite matrix A is partitioned into square tiles A_{I,J} of
 * side T; only the diagonal and strictly lower tiles are used, and the
 * right-looking algorithm (Fig. 1) overwrites them in place with the lower
 * Cholesky factor L, A = L L^T, through four tile operations:
 *   POTRF  A_JJ <- chol(A_JJ)
 *   TRSM   A_IJ <- A_IJ A_JJ^{-T}             (I > J)
 *   SYRK   A_II <- A_II - A_IJ A_IJ^T         (I > J)
 *   GEMM   A_IK <- A_IK - A_IJ A_KJ^T         (J < K < I)
 * The tile operations are ordered by their data dependencies (Methods,
 * "Implementations": the task graph of Fig. 3).  Two schedules are offered,
 * the GPU analogues of the paper's collapsed fork-join variant and of its
 * asynchronous task variant with explicit dependencies.
 *
 * Conventions shared by every entry point
 *   Storage   row-major: element (i, j) of A lives at A[i * lda + j],
 *             lda >= max(1, n).  Only the lower triangle including the
 *             diagonal is read or written; the strict upper triangle is
 *             never touched.  (A column-major caller holding a symmetric A
 *             finds L^T in its upper triangle.)
 *   Tiles     M = ceil(n / T) tiles per dimension; the last tile row and
 *             column are ragged with side n - (M - 1) T.  T > n is allowed
 *             (one tile).  All sizes and offsets are 64-bit; n and lda are
 *             at most CHOL_MAX_N (a 2^20-order FP64 matrix is 8 TB, far
 *             beyond one device, and the limit lets 128-row staging loads
 *             use 32-bit offsets).
 *   Memory    A, B and the workspace are device pointers owned by the
 *             caller; the library never allocates, frees or retains device
 *             memory.  `stream` is a hipStream_t passed as void* (NULL is
 *             the default stream); all work is enqueued on it.
 *   Errors    argument checks happen before anything is enqueued, so a
 *             call that returns CHOL_EINVAL or CHOL_EWORKSPACE has written
 *             nothing.  chol_last_bad_arg() names the offending argument.
 *             No C++ exception crosses this interface.
 *   Threads   calls are thread-safe; calls that share a workspace or a
 *             matrix must be ordered by the caller (same stream, or events).
 */
#ifndef TILECHOL_H
#define TILECHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHOL_MAX_N 1048576

/* Status codes.  > 0: numerical outcome; < 0: caller or runtime error. */
enum {
  CHOL_OK = 0,
  CHOL_NOT_SPD = 1,     /* a leading minor is not positive definite; see *info */
  CHOL_EINVAL = -1,     /* invalid argument (chol_last_bad_arg gives which)     */
  CHOL_EDEVICE = -2,    /* a HIP runtime call failed                             */
  CHOL_EWORKSPACE = -3, /* work_bytes smaller than the *_workspace_size result   */
  CHOL_ETIMEOUT = -4,   /* a dependency wait of the asynchronous schedule
                           exceeded chol_set_wait_limit; factor unspecified     */
  CHOL_ESTALLED = -5,   /* chol_server_wait: a dependency wait of the request's
                           factorization or solve exceeded the wait limit       */
  CHOL_ENOFACTOR = -6   /* serving: no such resident factor (never kept,
                           released, or evicted to make room)                    */
};

/* Schedules (Methods, "Implementations", the fork-join collapsed and task
 * asynchronous variants). */
enum {
  /* One launch per phase of each step J: POTRF(J), the TRSM panel of column
   * J, and the collapsed SYRK+GEMM trailing update of step J; stream order is
   * the barrier between phases. */
  CHOL_SCHED_FORK_JOIN = 0,
  /* One persistent launch.  Workgroups take work units in a fixed
   * topological order from an atomic ticket, wait on per-block dependency
   * counters in the workspace, run the unit, and publish its completion. */
  CHOL_SCHED_ASYNC_DAG = 1,
  /* The paper's naive fork-join variant: like CHOL_SCHED_FORK_JOIN, but the
   * trailing update is parallel over tile rows only (one workgroup walks a
   * whole tile row) and every POTRF has its own launch. */
  CHOL_SCHED_FORK_JOIN_NAIVE = 2,
  /* The paper's synchronous tasking variant: one persistent launch that
   * walks the phases of the blocked program order (each POTRF, TRSM column,
   * panel update and trailing update) with a grid-wide barrier after each
   * phase.  It needs all its workgroups co-resident (it launches exactly
   * the co-resident capacity); a barrier wait beyond chol_set_wait_limit
   * ends the call with CHOL_ETIMEOUT instead of hanging. */
  CHOL_SCHED_TASK_SYNC = 3,
  /* Fork-join with a one-step lookahead: the trailing update of step J is
   * split into the update of tile column J+1 (on the caller's stream) and
   * the rest (on a second stream the library keeps per host thread and
   * device), so the panel of step J+1 is factored while the rest of step J's
   * update runs.  Events keep every block's updates in step order; the
   * factor is bit-identical to the other schedules.  The call stays ordered
   * on the caller's stream. */
  CHOL_SCHED_FORK_JOIN_LOOKAHEAD = 4,
  /* The tile DAG as a HIP graph (the runtime-managed analogue of the
   * paper's task dependencies): the fork-join launches are graph nodes, the
   * trailing update of step J is one node per tile column, and the edges
   * are the dependencies between them, so the runtime overlaps later
   * columns' updates with the following panels as far as they allow.  The
   * instantiated graph is cached per (A, lda, n, T, work) and replayed on
   * `stream`; bit-identical to the other schedules. */
  CHOL_SCHED_GRAPH_DAG = 5
};

/* Flag ORed into `sched` to run the schedule with empty tile-operation
 * bodies (launches, tickets, waits, barriers and counters only), to measure
 * the schedule's own per-task cost.  A is left unchanged; the result is not
 * a factorization. */
#define CHOL_SCHED_NOOP 0x100

/* Bytes of device workspace chol_factor needs for (n, T, sched); < 0 on
 * invalid arguments.  The workspace holds the dependency counters, the work
 * ticket, an error flag and the device copy of info; its contents need not
 * be initialised by the caller. */
int64_t chol_factor_workspace_size(int64_t n, int64_t T, int sched);

/* Largest tile count per dimension the asynchronous schedule accepts
 * (ceil(n / T) above it returns CHOL_EINVAL naming T). */
#define CHOL_ASYNC_MAX_TILES 1024

/* Factor A = L L^T in place (Methods, Fig. 1, right-looking tiled order).
 *   A          device pointer, n x n row-major with leading dimension lda.
 *   T          tile side, T >= 1.
 *   sched      one of the CHOL_SCHED_* schedules, optionally ORed with
 *              CHOL_SCHED_NOOP.  All schedules run the same work units
 *              with the same bodies in the same per-block update order, so
 *              they return bit-identical factors.
 *   work       device workspace of at least chol_factor_workspace_size bytes
 *              (may be NULL only when n == 0).
 *   stream     hipStream_t as void*.
 *   info       host pointer or NULL.  If non-NULL the call synchronises the
 *              stream and stores 0 on success or k > 0 when the leading
 *              minor of order k is not positive definite (a pivot <= 0 or
 *              NaN at global column k - 1, LAPACK potrf convention); the
 *              lower triangle is then unspecified (the factorization stops
 *              inside the 128-column block that holds column k - 1).  With
 *              CHOL_ETIMEOUT it stores 1 + the ticket of the work unit whose
 *              dependency wait ran out (asynchronous schedule), or 0.  If
 *              NULL the call is fully asynchronous and its outcome is only
 *              visible through chol_factor_info().
 * Returns CHOL_OK, CHOL_NOT_SPD (only when info != NULL), CHOL_ETIMEOUT
 * (only when info != NULL) or a negative error code. */
int chol_factor(double* A, int64_t n, int64_t lda, int64_t T, int sched,
                void* work, int64_t work_bytes, void* stream, int64_t* info);

/* chol_factor for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same factorization, bit for bit, with the workspace taken from a
 * fixed array that the library keeps in each device's memory
 * (CHOL_NOALLOC_WORKSPACE bytes per device, held until the process ends)
 * instead of a caller's buffer.  The call allocates and frees nothing.
 *   A, n, lda, T, stream, info   as for chol_factor.
 *   sched      CHOL_SCHED_FORK_JOIN or CHOL_SCHED_ASYNC_DAG, optionally ORed
 *              with CHOL_SCHED_NOOP; other schedules give CHOL_EINVAL
 *              naming sched.
 * A problem whose workspace (chol_factor_workspace_size) exceeds
 * CHOL_NOALLOC_WORKSPACE returns CHOL_EWORKSPACE naming n (argument 2)
 * before anything is enqueued; with T >= 128 every n up to 131072 fits.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (concurrent streams or threads) race and must be ordered by
 * the caller.  The array's contents are cleared on the stream at the start
 * of each call.  With info == NULL the call is fully stream-ordered and its
 * outcome is not reported. */
#define CHOL_NOALLOC_WORKSPACE ((4 << 20) + (64 << 10))
int chol_factor_noalloc(double* A, int64_t n, int64_t lda, int64_t T, int sched, void* stream, int64_t* info);

/* Read the outcome of the last chol_factor enqueued with this workspace:
 * synchronises `stream`, stores info as above, and returns CHOL_OK,
 * CHOL_NOT_SPD or CHOL_ETIMEOUT. */
int chol_factor_info(const void* work, void* stream, int64_t* info);

/* Bytes of device workspace chol_solve needs: a 256-byte header (block
 * tickets and the status word), then two payload areas of
 * ceil(n / 64) * 64 rows of 2 (nrhs <= 2) or 4 x min(16, ceil(nrhs / 4))
 * (nrhs > 2) doubles each,
 * every part rounded up to 256 bytes; < 0 on invalid arguments. */
int64_t chol_solve_workspace_size(int64_t n, int64_t T, int64_t nrhs);

/* Solve A X = B with the factor from chol_factor (the paper's motivating
 * use, SPD linear systems via the Cholesky decomposition): forward
 * substitution L Y = B, then backward substitution L^T X = Y, each one
 * launch over 64-row blocks (one per workgroup).  A solved block reaches
 * the workgroups of later blocks through the workspace's payload areas
 * (device-scope atomic stores read until no sentinel remains), so no
 * counter or cache flush sits between two blocks of the chain.  One or two
 * right-hand sides take one pass; more take passes of four, up to 16 passes
 * (64 columns) sharing one launch pair, further columns further launch
 * pairs.  A column's result is the same bit for bit however many others
 * share its call.
 *   L      device pointer to the factor (lower triangle read only).
 *   B      device pointer, n x nrhs row-major, leading dimension
 *          ldb >= max(1, nrhs); overwritten by X.
 *   T      tile side of the factor (validated, T >= 1; the sweeps use their
 *          own 64-row blocks, so any T gives the same X).
 *   work   device workspace of chol_solve_workspace_size bytes (contents
 *          need not be initialised; calls sharing it must be ordered).
 * Returns CHOL_OK or a negative error code.  Stream-ordered; no host sync.
 * A sweep whose dependency wait exceeds chol_set_wait_limit stops early and
 * leaves B unspecified instead of hanging; the workspace then records the
 * timeout until the next chol_solve with it (chol_solve_info reads it). */
int chol_solve(const double* L, int64_t n, int64_t lda, int64_t T,
               double* B, int64_t nrhs, int64_t ldb,
               void* work, int64_t work_bytes, void* stream);

/* Outcome of the last chol_solve enqueued with this workspace: synchronises
 * `stream` and returns CHOL_OK, or CHOL_ETIMEOUT when a dependency wait of
 * one of its sweeps ran out (B is then unspecified), or CHOL_EDEVICE. */
int chol_solve_info(const void* work, void* stream);

/* ---- mixed precision ----------------------------------------------------
 * The trailing SYRK/GEMM products, which carry almost all of the flops, are
 * formed from panel entries rounded once to a lower precision and summed in
 * FP32 on the matrix cores, then subtracted from FP64 storage; POTRF and
 * TRSM stay in FP64.  Around the factorization the matrix may be scaled
 * symmetrically to unit diagonal and shifted, and the solve recovers FP64
 * accuracy by refinement against the original A.  (The paper's algorithm is
 * FP64 throughout; this is an extension of its tile loop, Fig. 1.) */
enum {
  CHOL_PREC_FP64 = 0,  /* the plain FP64 trailing update                        */
  CHOL_PREC_FP32 = 1,  /* panel rounded to FP32 (nearest even), FP32 sums       */
  CHOL_PREC_BF16 = 2   /* panel rounded to BF16 (nearest even, no double
                          rounding), FP32 sums                                  */
};
/* Flags of chol_factor_mixed. */
#define CHOL_MIXED_SCALE 1 /* factor D^-1 A D^-1 with D = diag(A)^(1/2), return D L^ */

/* Bytes of device workspace chol_factor_mixed needs: the fork-join
 * workspace plus n doubles (D) plus two rounded panel copies (each n rows
 * of ceil(T / 64) * 64 elements of the chosen precision).  < 0 on invalid
 * arguments. */
int64_t chol_factor_mixed_workspace_size(int64_t n, int64_t T, int prec);

/* Factor in place with low-precision trailing products.  CHOL_PREC_FP32 and
 * CHOL_PREC_BF16 run the fork-join schedule with a one-step lookahead on a
 * second stream (panel J+1 is factored, and rounded into the second panel
 * copy, while the bulk of step J's update runs; the factor is the same bit
 * for bit as with plain fork-join); CHOL_PREC_FP64 runs plain fork-join.
 *   A, n, lda, T, work, stream, info   as for chol_factor.
 *   prec    one of CHOL_PREC_*.
 *   flags   0 or CHOL_MIXED_SCALE.
 *   shift   >= 0, added to the diagonal of the (scaled) matrix before the
 *           factorization: the result factors A + shift D^2 with scaling, or
 *           A + shift I without.  A low-precision factorization of an
 *           ill-conditioned matrix can meet a non-positive pivot; a shift
 *           restores positive definiteness at the cost of a worse
 *           preconditioner (refine with CHOL_REFINE_PCG then).
 * On return the lower triangle holds L (FP64 storage).  A non-positive
 * diagonal entry of A itself, or a failed pivot, returns CHOL_NOT_SPD with
 * *info as for chol_factor; the lower triangle is then unspecified.
 * prec = CHOL_PREC_FP64 with flags = 0 and shift = 0 is chol_factor with the
 * fork-join schedule, bit for bit. */
int chol_factor_mixed(double* A, int64_t n, int64_t lda, int64_t T, int prec, int flags, double shift,
                      void* work, int64_t work_bytes, void* stream, int64_t* info);

/* Refinement methods of chol_solve_refine. */
enum {
  CHOL_REFINE_IR = 0,  /* classical iterative refinement (FP64 residuals)        */
  CHOL_REFINE_PCG = 1  /* conjugate gradients preconditioned by L L^T            */
};
/* Status of chol_solve_refine when max_iter is reached first. */
#define CHOL_NOT_CONVERGED 2

/* Bytes of device workspace chol_solve_refine needs: the solve's header and
 * 16-column payloads, three arrays of ceil(n / 64) 64 x 64 blocks (the
 * inverted diagonal blocks of L and the coupling blocks of neighbouring
 * block rows), four n x nrhs FP64 blocks, n doubles and a few per-column
 * scalars.  < 0 on invalid arguments. */
int64_t chol_refine_workspace_size(int64_t n, int64_t T, int64_t nrhs);

/* Solve A X = B in FP64 to backward error <= tol per column, with a factor
 * L L^T of A (or of a shifted A) from chol_factor_mixed or chol_factor.
 * The backward error of column c is ||b - A x||_inf / (||A||_inf ||x||_inf
 * + ||b||_inf).  The solves with L L^T use the 64 x 64 diagonal blocks of L
 * inverted once per call and the products D_b L_{b,b-1} of neighbouring
 * block rows, so one matrix-core product per block sits on the sweeps'
 * chain; their rounding (about kappa(L_bb) u) is corrected by the
 * refinement like the factor's own error.
 *   A       device, the original SPD matrix (lower triangle read; lda).
 *   L       device, the factor (lower triangle read; ldl).
 *   B       device, n x nrhs row-major (ldb >= nrhs), read only.
 *   X       device, n x nrhs row-major (ldx >= nrhs), the solution.
 *   method  CHOL_REFINE_IR or CHOL_REFINE_PCG.
 *   tol     target backward error (> 0); max_iter >= 0 corrections
 *           (IR) or iterations (PCG).
 *   iters   host, or NULL: corrections applied (IR) / iterations of the
 *           slowest column (PCG).
 *   eta     host array of nrhs, or NULL: the final backward errors.
 * The call synchronises `stream` once per iteration (the stopping test).
 * Returns CHOL_OK, CHOL_NOT_CONVERGED (X holds the last iterate),
 * CHOL_ETIMEOUT (a dependency wait of a solve sweep exceeded
 * chol_set_wait_limit; X unspecified) or a negative error code. */
int chol_solve_refine(const double* A, int64_t lda, const double* L, int64_t ldl, int64_t n, int64_t T,
                      const double* B, int64_t ldb, double* X, int64_t ldx, int64_t nrhs, int method,
                      double tol, int64_t max_iter, void* work, int64_t work_bytes, void* stream,
                      int64_t* iters, double* eta);

/* ---- batched: many independent SPD matrices of uneven sizes in ONE
 * persistent launch.  Every matrix keeps its own tile DAG (the asynchronous
 * schedule's units and ticket order); the launch interleaves the matrices
 * phase by phase, largest first, so the grid always holds ready units.  A
 * matrix that is not positive definite is skipped from then on without
 * disturbing the others.
 *   A      host array of `batch` device pointers (row-major, lda[i]).
 *   n, lda host arrays of `batch` orders / leading dimensions (n[i] = 0 is
 *          allowed and skipped).
 *   T      host array of `batch` tile sides, or NULL for the tuned choice
 *          chol_batched_tile(n[i], CHOL_PREC_FP64).  ceil(n / T) must not
 *          exceed CHOL_ASYNC_MAX_TILES.
 *   work   device workspace of the *_workspace_size bytes (it holds the
 *          per-matrix counters and status, the descriptors and the unit
 *          list the host writes before the launch).
 *   info   host array of `batch` results or NULL (as for chol_factor).
 * Returns CHOL_OK, CHOL_NOT_SPD if any matrix failed (info says which),
 * CHOL_ETIMEOUT, or a negative error code. */
int64_t chol_factor_batched_workspace_size(int64_t batch, const int64_t* n, const int64_t* T);
int chol_factor_batched(double* const* A, const int64_t* n, const int64_t* lda, int64_t batch,
                        const int64_t* T, void* work, int64_t work_bytes, void* stream,
                        int64_t* info);

/* The same launch also solving A_i x_i = b_i for one right-hand side per
 * matrix: B is a host array of `batch` device pointers to n[i] contiguous
 * doubles, overwritten by x_i.  Each solve is one unit, run by one
 * workgroup (forward and backward substitution over 64-row blocks) as soon
 * as its factor is complete. */
int64_t chol_factor_solve_batched_workspace_size(int64_t batch, const int64_t* n, const int64_t* T);
int chol_factor_solve_batched(double* const* A, double* const* B, const int64_t* n, const int64_t* lda,
                              int64_t batch, const int64_t* T, void* work, int64_t work_bytes,
                              void* stream, int64_t* info);

/* The same launch with a per-matrix precision of the trailing products and
 * a refined solve (the mixed-precision extension of the tile loop, Fig. 1,
 * applied to a batch): matrix i is factored into L[i] from its original
 * A[i], which stays untouched, with its SYRK/GEMM products formed from panel
 * entries rounded once to FP32 and summed in FP32 (prec[i] =
 * CHOL_PREC_FP32; POTRF and TRSM stay FP64) or in FP64 (CHOL_PREC_FP64),
 * and its solve unit then computes x_i = (L L^T)^-1 b_i and refines it,
 * x_i += (L L^T)^-1 (b_i - A_i x_i) in FP64, until the backward error
 * ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf) is <= tol or max_iter
 * corrections were applied.
 *   A, B    host arrays of device pointers: the originals (lower triangle of
 *           A[i] read, lda[i]; b_i of n[i] contiguous doubles), read only.
 *   L, X    host arrays of device pointers: the factor (lower triangle of
 *           L[i] written, ldl[i]; L[i] must differ from A[i]) and x_i (n[i]
 *           contiguous doubles).
 *   T       host array of tile sides or NULL (chol_batched_tile(n, prec));
 *           an FP32 matrix of more than one tile needs T % 4 == 0.
 *   prec    host array of CHOL_PREC_FP64 / CHOL_PREC_FP32, or NULL (FP64).
 *   info    host array or NULL as for chol_factor_batched; iters, eta: host
 *           arrays (or NULL) of the corrections applied and the final
 *           backward error per matrix, filled only when info != NULL.
 * Returns CHOL_OK, CHOL_NOT_SPD, CHOL_ETIMEOUT, CHOL_NOT_CONVERGED (a
 * matrix ended above tol), or a negative error code. */
int64_t chol_factor_solve_batched_mixed_workspace_size(int64_t batch, const int64_t* n, const int64_t* T,
                                                       const int* prec);
int chol_factor_solve_batched_mixed(const double* const* A, double* const* L, const double* const* B,
                                    double* const* X, const int64_t* n, const int64_t* lda, const int64_t* ldl,
                                    int64_t batch, const int64_t* T, const int* prec, double tol, int64_t max_iter,
                                    void* work, int64_t work_bytes, void* stream, int64_t* info, int64_t* iters,
                                    double* eta);

/* Tile side a batched call uses for a matrix of order n when the caller
 * passes none: tables measured by an offline sweep over n-buckets for each
 * precision of the trailing products (paper_2606_11937_amd/tune_batched.py),
 * deterministic in (n, prec); prec is CHOL_PREC_FP64 or CHOL_PREC_FP32; < 0
 * on invalid arguments. */
int64_t chol_batched_tile(int64_t n, int prec);

/* ---- serving with continuous batching ----------------------------------
 * A server takes factor + solve requests at any time and answers each with
 * X = A^-1 B and its backward error.  A request is a Gaussian-process style
 * system: A = k(x_i, x_j) + nugget I with the squared-exponential kernel
 * k(x, y) = exp(-|x - y|^2 / (2 lengthscale^2)) on n points in the plane,
 * 1 <= nrhs <= CHOL_SERVE_MAX_RHS right-hand sides, and a target backward
 * error tol.  It may ask for its factor to stay resident (CHOL_SERVE_KEEP);
 * later solves against a resident factor (chol_server_submit_solve) skip
 * the factorization.
 * A worker thread admits pending requests in arrival order while their
 * device footprint fits in the caller's arena (8 n^2 + 16 n bytes for the
 * factor and the points, 24 n nrhs + 8 (3 nrhs + 2) for right-hand sides,
 * solution, residual and statistics, plus a per-tick workspace), evicting
 * resident factors that no request is using, least recently used first,
 * when the arena is short.  Each admitted group is one tick: matrix assembly
 * on the device, ONE persistent batched factorization launch, the solves as
 * multi-workgroup sweeps (as chol_solve), and a matrix-free residual giving
 * every request's backward error.  Up to two ticks are in flight on two
 * streams, so requests that arrive while a tick runs are admitted and
 * launched meanwhile.
 * Precision per request, from (n, tol) only: FP32 trailing products
 * (CHOL_PREC_FP32, tile side chol_batched_tile(n, CHOL_PREC_FP32)) from an
 * order on that depends on the tolerance class (tol >= 1e-8 or below, a
 * table measured offline), FP64 otherwise.  A request whose backward error
 * after its solve exceeds tol gets FP64 refinement corrections in later
 * ticks, x += (L L^T)^-1 (b - A x) with the residual formed matrix-free in
 * FP64; an FP32 factor whose corrections run out is refactored in FP64.
 * A request's result does not depend on which other requests shared its
 * ticks (bit for bit).
 *   CHOL_SERVE_FIFO is the plain baseline: one request at a time, chol_factor
 *   (fork-join, chol_default_tile) in FP64 then chol_solve.
 * Memory: the device arena (arena_bytes) belongs to the caller and is the
 * server's HBM budget; the server allocates no device memory.  It allocates
 * pinned_bytes of pinned host memory for staging (inputs and results of the
 * requests in flight) and frees it in chol_server_destroy.
 * Threads: every call may come from any thread.  destroy lets the admitted
 * and pending requests finish, then stops the worker. */
typedef struct chol_server chol_server;
enum { CHOL_SERVE_CONTINUOUS = 0, CHOL_SERVE_FIFO = 1 };
#define CHOL_SERVE_MAX_RHS 8
#define CHOL_SERVE_KEEP 1 /* flag of chol_server_submit: keep the factor resident */

/* max_per_tick: work items launched together at most (1 .. 65536). */
int chol_server_create(void* arena, int64_t arena_bytes, int64_t pinned_bytes, int mode,
                       int64_t max_per_tick, chol_server** server);
/* points: host, n x 2 row-major (copied); B: host, n x nrhs row-major
 * (copied); 1 <= n <= 65536; flags 0 or CHOL_SERVE_KEEP.  *id receives the
 * request's handle; the arrival time is taken here. */
int chol_server_submit(chol_server* server, const double* points, int64_t n, double lengthscale,
                       double nugget, const double* B, int64_t nrhs, double tol, int flags, int64_t* id);
/* A solve with resident factor `factor` (from chol_server_request_info of a
 * request submitted with CHOL_SERVE_KEEP): B host, n x nrhs row-major
 * (copied), n must be the factor's order.  The factor cannot be evicted
 * while such a request is pending or running.  Returns CHOL_ENOFACTOR if
 * the factor is not resident (never kept, released, or evicted). */
int chol_server_submit_solve(chol_server* server, int64_t factor, const double* B, int64_t n, int64_t nrhs,
                             double tol, int64_t* id);
/* Wait up to timeout_s seconds for request id.  When it is done: X (host,
 * n x nrhs, or NULL) receives the solution, *eta the worst column's backward
 * error, *latency_s the time from submission to the result being in host
 * memory.  Returns CHOL_OK (eta <= tol), CHOL_NOT_CONVERGED (done, eta >
 * tol), CHOL_NOT_SPD (*info as for chol_factor), CHOL_ESTALLED (a dependency
 * wait exceeded chol_set_wait_limit, in the request's first run and again
 * in the one restart it is given, and X is unspecified: *info = 1 + the
 * ticket, within its tick's launch, of the factorization unit that waited,
 * or -1 when a solve sweep's wait ran out), CHOL_EWORKSPACE (the request can
 * never fit in the arena), CHOL_ETIMEOUT (not done yet), or a negative error
 * code. */
int chol_server_wait(chol_server* server, int64_t id, double timeout_s, double* X, double* eta,
                     double* latency_s, int64_t* info);
/* How request id was served (any argument but server may be NULL): *factor
 * the handle of its resident factor (CHOL_SERVE_KEEP, once done; -1
 * otherwise, and for a solve request the factor it used), *prec the
 * precision of the factor that produced the result (CHOL_PREC_*),
 * *corrections the refinement corrections of that factor, *refactors 1 if
 * an FP32 factor was replaced by an FP64 one.  Returns CHOL_OK or
 * CHOL_EINVAL (unknown id). */
int chol_server_request_info(chol_server* server, int64_t id, int64_t* factor, int* prec, int* corrections,
                             int* refactors);
/* The precision plan of requests submitted from now on: FP32 trailing
 * products for orders n >= fp32_min_n_loose when tol >= 1e-8, and for
 * n >= fp32_min_n_strict below; FP64 otherwise (a value above 65536 turns
 * FP32 off for that class).  The default is the measured table the library
 * compiles in; this call is for measuring other plans. */
int chol_server_set_plan(chol_server* server, int64_t fp32_min_n_loose, int64_t fp32_min_n_strict);
/* Drop a resident factor; CHOL_ENOFACTOR if it is not resident or a pending
 * or running request still uses it. */
int chol_server_release_factor(chol_server* server, int64_t factor);
/* Ticks launched so far, and resident factors evicted so far (< 0 on invalid
 * arguments). */
int64_t chol_server_ticks(chol_server* server);
int64_t chol_server_evictions(chol_server* server);
int chol_server_destroy(chol_server* server);

/* Tile side the library picks for order n when the caller passes none
 * (deterministic in n; from measured factor times). */
int64_t chol_default_tile(int64_t n);

/* ---- introspection of the tile DAG (host only; no device is touched) ----
 * Work units are the pieces the schedules launch.  Blocks are CHOL_BLOCK
 * rows (and columns) inside a tile; sub-block a of tile I is global block
 * I * ceil(min(T, n) / CHOL_BLOCK) + a.  The panel of tile column J (its
 * POTRF and TRSM tasks) is factored one CHOL_BLOCK-wide sub-column at a
 * time, the blocked form of the same operations; the SYRK/GEMM trailing
 * update of step J keeps K-depth T.  Each unit is 6 int32 {kind, J, I, a,
 * K, b}:
 *   POTRF   {0, J, J, s, -1, -1}   diagonal block s of tile J;
 *   TRSM    {1, J, I, a,  s, -1}   block (I, a) below it against that block;
 *   UPDATE  {2, J, I, a,  K,  b}   output block (a, b) of tile (I, K) at
 *                                  step J (SYRK when I == K, only b <= a);
 *   PANEL   {3, J, I, a,  s, s2}   block (I, a) of panel sub-column s2 of
 *                                  tile J minus the product of the finished
 *                                  sub-column s < s2 (rows at or below s2). */
#define CHOL_BLOCK 128

/* Work-unit kinds as encoded by chol_dag_enumerate. */
enum { CHOL_UNIT_POTRF = 0, CHOL_UNIT_TRSM = 1, CHOL_UNIT_UPDATE = 2, CHOL_UNIT_PANEL = 3 };

/* Tile-task counts for (n, T) (Results, "Problem Size Scaling": M POTRF,
 * M(M-1)/2 TRSM and SYRK each, M(M-1)(M-2)/6 GEMM): counts[0..3] =
 * POTRF, TRSM, SYRK, GEMM tasks; counts[4] = work units of the asynchronous
 * schedule.  Returns CHOL_OK or CHOL_EINVAL. */
int chol_dag_counts(int64_t n, int64_t T, int64_t counts[5]);

/* Write the asynchronous schedule's work units in dispatch (ticket) order,
 * 6 int32 each as above.
 * `grid` is the number of persistent workgroups the order is tuned for
 * (it sets how far the panel of step J+1 runs ahead of step J's bulk
 * update).  Writes min(cap, total) units; returns the total, or a negative
 * error code. */
int64_t chol_dag_enumerate(int64_t n, int64_t T, int64_t grid, int32_t* out, int64_t cap);

/* Write the units of the fork-join schedule's trailing-update launch of step
 * J (the collapsed SYRK + GEMM launch, Methods, fork-join) in launch order,
 * one workgroup per unit, 6 int32 each as above.  Writes min(cap, total)
 * units; returns the total or a negative error code. */
int64_t chol_dag_forkjoin_update(int64_t n, int64_t T, int64_t J, int32_t* out, int64_t cap);

/* Number of persistent workgroups the asynchronous schedule launches on the
 * current device (co-resident capacity); < 0 on error.  Touches the device. */
int64_t chol_async_grid(void);

/* ---- measurement aid ----
 * Per-launch device time of chol_factor.  `kinds` is a bit mask: bit k
 * (k = CHOL_UNIT_POTRF, CHOL_UNIT_TRSM, CHOL_UNIT_UPDATE, CHOL_UNIT_PANEL)
 * times the fork-join launches of that unit kind, bit 4 the persistent
 * launch of the asynchronous schedule, bit 5 the bulk trailing update of
 * each step of CHOL_SCHED_FORK_JOIN_LOOKAHEAD (the columns beyond J+1: one
 * interval per step, from its launch on the second stream to the later of
 * that launch's end and the end of its tail launch on the call's stream,
 * which shares its unit counter; its column-(J+1) launches count under bit
 * CHOL_UNIT_UPDATE); 0 turns timing off.  While enabled on
 * the calling thread, each selected launch chol_factor enqueues is
 * bracketed by a pair of HIP events on the call's stream (events are
 * created on first use and reused; no device memory is allocated; each pair
 * adds a few microseconds to the stream, so time only what is needed).
 * chol_timing_read synchronises `stream`, writes the summed milliseconds and
 * the launch counts per kind (same indices) recorded since the previous
 * read, and clears them.  The workspace-clearing launch is never timed.
 * chol_timing_enable returns the previous mask; chol_timing_read returns
 * CHOL_OK, CHOL_EINVAL (NULL output) or CHOL_EDEVICE. */
#define CHOL_TIMING_KINDS 6
int chol_timing_enable(int kinds);
int chol_timing_read(void* stream, double ms[CHOL_TIMING_KINDS], int64_t launches[CHOL_TIMING_KINDS]);

/* Dispatch-order knob of the asynchronous schedule (the paper's task
 * priorities, here a property of the ticket order): the number of bulk
 * trailing-update units placed after each link of a panel chain.  Negative
 * restores the default (half the persistent grid); 0 puts each panel's
 * whole chain ahead of the previous step's bulk update; a value at least
 * that bulk's size puts the bulk first (no lookahead).  Process-wide; also
 * used by chol_dag_enumerate.  Returns the previous setting. */
int64_t chol_set_lookahead(int64_t units);

/* Upper bound in seconds on any single dependency wait of the asynchronous
 * schedule (default 10).  A wait that exceeds it ends the factorization
 * with CHOL_ETIMEOUT instead of a hang.  Process-wide; values < 0 are
 * rejected.  Returns the previous value. */
double chol_set_wait_limit(double seconds);

/* 1-based index of the argument that made the last call on this thread
 * return CHOL_EINVAL or CHOL_EWORKSPACE; 0 if none. */
int chol_last_bad_arg(void);

/* Static description of a status code. */
const char* chol_status_str(int status);

#ifdef __cplusplus
}
#endif
#endif /* TILECHOL_H */
