// refine.hip -- solving A X = B in FP64 with a factor L L^T of A (or of a
// shifted A) computed with low-precision trailing products.
//
// Every solve with L L^T here runs the sweeps with inverted diagonal blocks
// (solve.hip): the blocks are inverted once per call, and the small error of
// the inverses is corrected by the refinement like the factor's own.
//
//   iterative refinement   x_0 = (L L^T)^-1 b;  r = b - A x,
//                          x <- x + (L L^T)^-1 r  until the backward error
//                          of every column is <= tol;
//   preconditioned CG      conjugate gradients on A with M = L L^T, every
//                          column with its own step lengths; a column stops
//                          when its recurrence residual meets tol and the
//                          true residual b - A x confirms it (if not, the
//                          true residual replaces the recurrence one and the
//                          column restarts its search direction).
//
// The backward error of a column is ||r||_inf / (||A||_inf ||x||_inf +
// ||b||_inf).  A is the original symmetric matrix, of which only the lower
// triangle is read.
//
// Products with A: one launch; every wave owns 16 output rows and 16
// columns of X and contracts on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64), reading the lower triangle straight from HBM
// (rows of A left of the diagonal, columns below it).  The sums of each
// output entry run in a fixed order, so results are reproducible.  Column reductions (maxima, dot products) are one workgroup
// per column with a fixed partition and a fixed tree.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "launch.h"

#define RF_THREADS 256
#define RF_RC 16  // right-hand sides per pass of a product kernel
#define RF_CH 2   // 16-wide k chunks per step of the product kernel (and in flight)

typedef double rf_v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ rf_v4d rf_mfma(double a, double b, rf_v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------ A times X
// Y = B - A X (Y = -A X when B is null) for symmetric A stored as its lower
// triangle, and, when rowabs is not null, rowabs[i] = sum_k |A_ik| (the row
// sums of |A|, from the same reads).  One workgroup per 64 rows; wave w owns rows
// 64 blockIdx + 16 w .. +15 and walks k = 0 .. n - 1 in 16-wide chunks,
// reading A_ik from row i for k <= i and as A_ki from column i for k > i (so
// every stored entry is read twice in all, once for each of its rows).
// The row sums of |A| add, per lane, the entries it brings to the products
// (chunks in ascending k), then the lanes of a row in the fixed order
// (g0 + g1) + (g2 + g3).
// MFMA operand layout (measured on gfx950): A-operand lane l holds row
// l % 16 at k group l / 16, B-operand lane l holds column l % 16 at k group
// l / 16, output item q of lane l is row 4 q + l / 16, column l % 16.  In a
// chunk, lane (r, g) brings k = 4 g + m to MFMA m for both operands.  Each
// output entry sums its chunks in ascending k, so results are reproducible.
// Loads are branch-free: indices are clamped into the stored triangle and
// masked entries are selected away; the next chunk is loaded while the
// current one is multiplied.
__global__ __launch_bounds__(RF_THREADS, 2) void rf_symv(const double* __restrict__ A, int64_t lda, int64_t n,
                                                         const double* __restrict__ X, int64_t ldx,
                                                         const double* __restrict__ B, int64_t ldb,
                                                         double* __restrict__ Y, int64_t ldy, int64_t nrhs,
                                                         double* __restrict__ rowabs) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, g4 = (lane >> 4) * 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + 16 * w;  // first output row of this wave
  if (row0 >= n) return;
  const int64_t myrow = row0 + r16;
  const bool rowok = myrow < n;
  const int64_t rowc = rowok ? myrow : n - 1;
  const int64_t nch = (n + 15) / 16;
  for (int64_t c0 = 0; c0 < nrhs; c0 += RF_RC) {
    const int64_t col = c0 + r16;
    const bool colok = col < nrhs;
    const int64_t colc = colok ? col : nrhs - 1;
    auto load = [&](int64_t ch, double* a, double* x) {
      const int64_t k0 = 16 * ch;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int64_t k = k0 + g4 + m;
        const bool kin = k < n;
        const int64_t kc = kin ? k : n - 1;
        // k <= row: A[row][k] (row part); k > row: A[k][row] (column part)
        const bool low = kc <= rowc;
        const double v = low ? A[rowc * lda + kc] : A[kc * lda + rowc];
        a[m] = (rowok && kin) ? v : 0.0;
        const double xv = X[kc * ldx + colc];
        x[m] = (colok && kin) ? xv : 0.0;
      }
    };
    // chunks in groups of RF_CH, the next group in flight while this one is
    // multiplied (a chunk index past the end re-reads the last chunk and is
    // not used)
    rf_v4d acc = {0.0, 0.0, 0.0, 0.0};
    // with rowabs, the first pass also sums |A_ik| over this lane's k
    const bool absum_on = rowabs != nullptr && c0 == 0;
    double absum = 0.0;
    double a[4 * RF_CH], x[4 * RF_CH];
#pragma unroll
    for (int h = 0; h < RF_CH; ++h) load(h < nch ? h : nch - 1, a + 4 * h, x + 4 * h);
    for (int64_t ch = 0; ch < nch; ch += RF_CH) {
      double an[4 * RF_CH], xn[4 * RF_CH];
#pragma unroll
      for (int h = 0; h < RF_CH; ++h) load(ch + RF_CH + h < nch ? ch + RF_CH + h : nch - 1, an + 4 * h, xn + 4 * h);
#pragma unroll
      for (int h = 0; h < RF_CH; ++h) {
        if (ch + h < nch) {
#pragma unroll
          for (int m = 0; m < 4; ++m) acc = rf_mfma(a[4 * h + m], x[4 * h + m], acc);
          if (absum_on) {
#pragma unroll
            for (int m = 0; m < 4; ++m) absum += fabs(a[4 * h + m]);
          }
        }
      }
#pragma unroll
      for (int m = 0; m < 4 * RF_CH; ++m) {
        a[m] = an[m];
        x[m] = xn[m];
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = row0 + 4 * q + (lane >> 4);
      const int64_t c = c0 + (lane & 15);
      if (r < n && c < nrhs) Y[r * ldy + c] = (B != nullptr ? B[r * ldb + c] : 0.0) - acc[q];
    }
    if (absum_on) {
      // the four k groups of row r16: (g0 + g1) + (g2 + g3)
      absum += __shfl_xor(absum, 16, 64);
      absum += __shfl_xor(absum, 32, 64);
      if (lane < 16 && rowok) rowabs[myrow] = absum;
    }
  }
}

// ------------------------------------------------------- column reductions
// Fixed-order tree over the 256 threads of the workgroup.
__device__ __forceinline__ double rf_block_reduce(double v, bool take_max) {
  __shared__ double red[RF_THREADS];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = RF_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double o = red[threadIdx.x + s];
      red[threadIdx.x] = take_max ? fmax(red[threadIdx.x], o) : red[threadIdx.x] + o;
    }
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// out[c] = max_i |U[i][c]| (one workgroup per column c).
__global__ __launch_bounds__(RF_THREADS) void rf_colmax(const double* U, int64_t ldu, int64_t n, double* out) {
  const int64_t c = blockIdx.x;
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += RF_THREADS) m = fmax(m, fabs(U[i * ldu + c]));
  m = rf_block_reduce(m, true);
  if (threadIdx.x == 0) out[c] = m;
}

// out[c] = sum_i U[i][c] V[i][c]: thread t sums rows t, t + 256, ... in
// order, then the fixed tree.
__global__ __launch_bounds__(RF_THREADS) void rf_coldot(const double* U, int64_t ldu, const double* V, int64_t ldv,
                                                        int64_t n, double* out) {
  const int64_t c = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += RF_THREADS) s = fma(U[i * ldu + c], V[i * ldv + c], s);
  s = rf_block_reduce(s, false);
  if (threadIdx.x == 0) out[c] = s;
}

// eta[c] = rmax[c] / (anorm xmax[c] + bmax[c]) (0 when the denominator is 0).
__global__ void rf_eta(const double* rmax, const double* xmax, const double* bmax, const double* anorm, int64_t nrhs,
                       double* eta) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const double den = anorm[0] * xmax[c] + bmax[c];
  eta[c] = den > 0.0 ? rmax[c] / den : 0.0;
}

// ------------------------------------------------------- elementwise steps
// Y[i][c] += f[c] X[i][c] with f = alpha (sign +1) or -alpha (sign -1); f = 1
// when alpha is null.
__global__ void rf_axpy(double* Y, int64_t ldy, const double* X, int64_t ldx, const double* alpha, double sign,
                        int64_t n, int64_t nrhs) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * nrhs) return;
  const int64_t i = idx / nrhs, c = idx - i * nrhs;
  const double f = alpha != nullptr ? sign * alpha[c] : sign;
  Y[i * ldy + c] = Y[i * ldy + c] + f * X[i * ldx + c];
}

// P[i][c] = Z[i][c] + beta[c] P[i][c].
__global__ void rf_xpby(double* P, int64_t ldp, const double* Z, int64_t ldz, const double* beta, int64_t n,
                        int64_t nrhs) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * nrhs) return;
  const int64_t i = idx / nrhs, c = idx - i * nrhs;
  P[i * ldp + c] = Z[i * ldz + c] + beta[c] * P[i * ldp + c];
}

// Y[i][c] = X[i][c], for columns with mask[c] != 0 (all columns when mask is null).
__global__ void rf_copy(double* Y, int64_t ldy, const double* X, int64_t ldx, const int32_t* mask, int64_t n,
                        int64_t nrhs) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * nrhs) return;
  const int64_t i = idx / nrhs, c = idx - i * nrhs;
  if (mask == nullptr || mask[c]) Y[i * ldy + c] = X[i * ldx + c];
}

// PCG step lengths.  The product kernel returns Q' = -A p, so p.q = -pq'.
//   alpha[c] = rz[c] / (p.q)                 (0 for finished columns)
//   beta[c]  = rz_new[c] / rz[c]             (0 for finished or restarted)
__global__ void rf_alpha(const double* rz, const double* pqn, const int32_t* done, int64_t nrhs, double* alpha) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const double pq = -pqn[c];
  alpha[c] = (done[c] || pq == 0.0) ? 0.0 : rz[c] / pq;
}
__global__ void rf_beta(double* rz, const double* rz_new, const int32_t* zero, int64_t nrhs, double* beta) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  beta[c] = (zero[c] || rz[c] == 0.0) ? 0.0 : rz_new[c] / rz[c];
  rz[c] = rz_new[c];
}

// ------------------------------------------------------------ host driver
namespace {
inline unsigned rf_blocks(int64_t count, int per) { return (unsigned)((count + per - 1) / per); }
inline int64_t rf_r256(int64_t x) { return (x + 255) & ~(int64_t)255; }

struct RfWs {
  void* solve_ws;
  double* dinv;                   // inverted 64 x 64 diagonal blocks of L
  double *R, *Z, *P, *Q;          // n x nrhs each, leading dimension nrhs
  double* rowsum;                 // n: the row sums of |A|
  double *anorm, *rmax, *xmax, *bmax, *eta, *rz, *rzn, *pq, *alpha, *beta;  // nrhs each (anorm: 1)
  int32_t *done, *zero, *mask;    // nrhs each
};

RfWs rf_map(void* work, int64_t n, int64_t nrhs) {
  RfWs w;
  char* p = (char*)work;
  w.solve_ws = p;
  p += rf_r256(tc_solve_ws_bytes(n, nrhs, true));
  w.dinv = (double*)p;
  p += rf_r256(tc_solve_inv_bytes(n));
  const int64_t mat = rf_r256(8 * n * nrhs);
  w.R = (double*)p; p += mat;
  w.Z = (double*)p; p += mat;
  w.P = (double*)p; p += mat;
  w.Q = (double*)p; p += mat;
  w.rowsum = (double*)p; p += rf_r256(8 * n);
  double** vecs[] = {&w.anorm, &w.rmax, &w.xmax, &w.bmax, &w.eta, &w.rz, &w.rzn, &w.pq, &w.alpha, &w.beta};
  for (double** v : vecs) {
    *v = (double*)p;
    p += rf_r256(8 * nrhs);
  }
  int32_t** flags[] = {&w.done, &w.zero, &w.mask};
  for (int32_t** f : flags) {
    *f = (int32_t*)p;
    p += rf_r256(4 * nrhs);
  }
  return w;
}

// Y = B - A X  (B null: Y = -A X); rowabs (optional): the row sums of |A|
void rf_residual(const double* A, int64_t lda, int64_t n, const double* X, int64_t ldx, const double* B, int64_t ldb,
                 double* Y, int64_t ldy, int64_t nrhs, hipStream_t st, double* rowabs = nullptr) {
  hipLaunchKernelGGL(rf_symv, dim3(rf_blocks(n, 64)), dim3(RF_THREADS), 0, st, A, lda, n, X, ldx, B, ldb, Y, ldy, nrhs,
                     rowabs);
}

// eta of every column of (R, X, B) into w.eta, copied to host `eta`
int rf_eta_host(const RfWs& w, const double* R, const double* X, int64_t ldx, int64_t n, int64_t nrhs,
                std::vector<double>& eta, hipStream_t st) {
  hipLaunchKernelGGL(rf_colmax, dim3((unsigned)nrhs), dim3(RF_THREADS), 0, st, R, nrhs, n, w.rmax);
  hipLaunchKernelGGL(rf_colmax, dim3((unsigned)nrhs), dim3(RF_THREADS), 0, st, X, ldx, n, w.xmax);
  hipLaunchKernelGGL(rf_eta, dim3(rf_blocks(nrhs, 64)), dim3(64), 0, st, w.rmax, w.xmax, w.bmax, w.anorm, nrhs, w.eta);
  if (hipMemcpyAsync(eta.data(), w.eta, 8 * nrhs, hipMemcpyDeviceToHost, st) != hipSuccess) return -1;
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  return 0;
}

double rf_max(const std::vector<double>& v) {
  double m = 0.0;
  for (double x : v) m = x > m || x != x ? x : m;
  return m;
}
}  // namespace

int64_t tc_refine_ws_bytes(int64_t n, int64_t nrhs) {
  return rf_r256(tc_solve_ws_bytes(n, nrhs, true)) + rf_r256(tc_solve_inv_bytes(n)) + 4 * rf_r256(8 * n * nrhs) + rf_r256(8 * n) + 10 * rf_r256(8 * nrhs) +
         3 * rf_r256(4 * nrhs);
}

// Returns 0 converged, 1 not converged within max_iter, < 0 device error.
int tc_refine(const double* A, int64_t lda, const double* L, int64_t ldl, int64_t n, int64_t T, const double* B,
              int64_t ldb, double* X, int64_t ldx, int64_t nrhs, int method, double tol, int64_t max_iter, void* work,
              hipStream_t st, int64_t wait_ticks, int64_t* iters, double* eta_out) {
  const RfWs w = rf_map(work, n, nrhs);
  const unsigned eb = rf_blocks(n * nrhs, 256);
  std::vector<double> eta(nrhs, 0.0), eta_true(nrhs, 0.0);
  // host flag arrays stay alive until the function returns; every host
  // update of them follows a stream synchronisation
  std::vector<int32_t> done(nrhs, 0), zero(nrhs, 0), mask(nrhs, 0);
  auto fail = [&]() { return TC_LAUNCH_EDEVICE; };
  (void)T;
  auto solve = [&](double* Y, int64_t ldy) {
    return tc_launch_solve_inv(L, n, ldl, w.dinv, Y, nrhs, ldy, w.solve_ws, st, wait_ticks);
  };
  if (tc_launch_invert_diag(L, n, ldl, w.dinv, st) != 0) return fail();
  // one status word for every sweep of the call
  if (tc_solve_status_reset(w.solve_ws, st) != 0) return fail();
  // ||b||_inf per column (||A||_inf comes with the first residual)
  hipLaunchKernelGGL(rf_colmax, dim3((unsigned)nrhs), dim3(RF_THREADS), 0, st, B, ldb, n, w.bmax);
  // x0 = (L L^T)^-1 b
  hipLaunchKernelGGL(rf_copy, dim3(eb), dim3(256), 0, st, X, ldx, B, ldb, (const int32_t*)nullptr, n, nrhs);
  if (solve(X, ldx) != 0) return fail();
  // the first residual also gives the row sums of |A|: ||A||_inf is their maximum
  rf_residual(A, lda, n, X, ldx, B, ldb, w.R, nrhs, nrhs, st, w.rowsum);
  hipLaunchKernelGGL(rf_colmax, dim3(1), dim3(RF_THREADS), 0, st, (const double*)w.rowsum, (int64_t)1, n, w.anorm);
  if (rf_eta_host(w, w.R, X, ldx, n, nrhs, eta, st) != 0) return fail();
  int64_t it = 0;
  int status = 1;
  if (method == 0) {  // iterative refinement
    while (true) {
      if (rf_max(eta) <= tol) {
        status = 0;
        break;
      }
      if (it == max_iter) break;
      if (solve(w.R, nrhs) != 0) return fail();
      hipLaunchKernelGGL(rf_axpy, dim3(eb), dim3(256), 0, st, X, ldx, (const double*)w.R, nrhs,
                         (const double*)nullptr, 1.0, n, nrhs);
      ++it;
      rf_residual(A, lda, n, X, ldx, B, ldb, w.R, nrhs, nrhs, st);
      if (rf_eta_host(w, w.R, X, ldx, n, nrhs, eta, st) != 0) return fail();
    }
  } else {  // preconditioned conjugate gradients
    for (int64_t c = 0; c < nrhs; ++c) done[c] = eta[c] <= tol;
    if (hipMemcpyAsync(w.done, done.data(), 4 * nrhs, hipMemcpyHostToDevice, st) != hipSuccess) return fail();
    hipLaunchKernelGGL(rf_copy, dim3(eb), dim3(256), 0, st, w.Z, nrhs, (const double*)w.R, nrhs,
                       (const int32_t*)nullptr, n, nrhs);
    if (solve(w.Z, nrhs) != 0) return fail();
    hipLaunchKernelGGL(rf_copy, dim3(eb), dim3(256), 0, st, w.P, nrhs, (const double*)w.Z, nrhs,
                       (const int32_t*)nullptr, n, nrhs);
    hipLaunchKernelGGL(rf_coldot, dim3((unsigned)nrhs), dim3(RF_THREADS), 0, st, (const double*)w.R, nrhs,
                       (const double*)w.Z, nrhs, n, w.rz);
    auto all_done = [&]() {
      for (int64_t c = 0; c < nrhs; ++c)
        if (!done[c]) return false;
      return true;
    };
    eta_true = eta;
    while (!all_done() && it < max_iter) {
      ++it;
      rf_residual(A, lda, n, w.P, nrhs, nullptr, 0, w.Q, nrhs, nrhs, st);  // Q = -A P
      hipLaunchKernelGGL(rf_coldot, dim3((unsigned)nrhs), dim3(RF_THREADS), 0, st, (const double*)w.P, nrhs,
                         (const double*)w.Q, nrhs, n, w.pq);
      hipLaunchKernelGGL(rf_alpha, dim3(rf_blocks(nrhs, 64)), dim3(64), 0, st, (const double*)w.rz,
                         (const double*)w.pq, (const int32_t*)w.done, nrhs, w.alpha);
      hipLaunchKernelGGL(rf_axpy, dim3(eb), dim3(256), 0, st, X, ldx, (const double*)w.P, nrhs,
                         (const double*)w.alpha, 1.0, n, nrhs);
      hipLaunchKernelGGL(rf_axpy, dim3(eb), dim3(256), 0, st, w.R, nrhs, (const double*)w.Q, nrhs,
                         (const double*)w.alpha, 1.0, n, nrhs);  // r -= alpha q  (Q holds -A p)
      if (rf_eta_host(w, w.R, X, ldx, n, nrhs, eta, st) != 0) return fail();
      bool check = false;
      for (int64_t c = 0; c < nrhs; ++c) check = check || (!done[c] && eta[c] <= tol);
      for (int64_t c = 0; c < nrhs; ++c) zero[c] = done[c];
      if (check) {
        // confirm with the true residual b - A x (into Z, reused as scratch)
        rf_residual(A, lda, n, X, ldx, B, ldb, w.Z, nrhs, nrhs, st);
        if (rf_eta_host(w, w.Z, X, ldx, n, nrhs, eta_true, st) != 0) return fail();
        for (int64_t c = 0; c < nrhs; ++c) mask[c] = 0;
        for (int64_t c = 0; c < nrhs; ++c) {
          if (done[c] || eta[c] > tol) continue;
          if (eta_true[c] <= tol) {
            done[c] = 1;
          } else {
            mask[c] = 1;  // replace the recurrence residual, restart the direction
          }
          zero[c] = 1;
        }
        if (hipMemcpyAsync(w.mask, mask.data(), 4 * nrhs, hipMemcpyHostToDevice, st) != hipSuccess) return fail();
        hipLaunchKernelGGL(rf_copy, dim3(eb), dim3(256), 0, st, w.R, nrhs, (const double*)w.Z, nrhs,
                           (const int32_t*)w.mask, n, nrhs);
        if (hipMemcpyAsync(w.done, done.data(), 4 * nrhs, hipMemcpyHostToDevice, st) != hipSuccess) return fail();
      }
      if (all_done()) break;
      if (hipMemcpyAsync(w.zero, zero.data(), 4 * nrhs, hipMemcpyHostToDevice, st) != hipSuccess) return fail();
      hipLaunchKernelGGL(rf_copy, dim3(eb), dim3(256), 0, st, w.Z, nrhs, (const double*)w.R, nrhs,
                         (const int32_t*)nullptr, n, nrhs);
      if (solve(w.Z, nrhs) != 0) return fail();
      hipLaunchKernelGGL(rf_coldot, dim3((unsigned)nrhs), dim3(RF_THREADS), 0, st, (const double*)w.R, nrhs,
                         (const double*)w.Z, nrhs, n, w.rzn);
      hipLaunchKernelGGL(rf_beta, dim3(rf_blocks(nrhs, 64)), dim3(64), 0, st, w.rz, (const double*)w.rzn,
                         (const int32_t*)w.zero, nrhs, w.beta);
      hipLaunchKernelGGL(rf_xpby, dim3(eb), dim3(256), 0, st, w.P, nrhs, (const double*)w.Z, nrhs,
                         (const double*)w.beta, n, nrhs);
    }
    // final true backward error of every column
    rf_residual(A, lda, n, X, ldx, B, ldb, w.R, nrhs, nrhs, st);
    if (rf_eta_host(w, w.R, X, ldx, n, nrhs, eta, st) != 0) return fail();
    status = rf_max(eta) <= tol ? 0 : 1;
  }
  if (hipGetLastError() != hipSuccess) return fail();
  int32_t stalled = 0;
  if (tc_solve_status(w.solve_ws, st, &stalled) != 0) return fail();
  if (iters) *iters = it;
  if (stalled) return TC_LAUNCH_ETIMEOUT;
  if (eta_out)
    for (int64_t c = 0; c < nrhs; ++c) eta_out[c] = eta[c];
  return status;
}
