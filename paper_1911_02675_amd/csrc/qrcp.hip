// Column-pivoted QR preconditioner (the factor step of Section 1.2 with a rank-revealing QR): S A P = Q R
// by Householder reflections, choosing at each step the remaining column of largest norm.  The leading
// r x r block R11 (r: the diagonal entries above rtol |R_00|) gives
//     W = P [R11^{-1}; 0]  (dense d x d, zero outside the kept columns),  W W^T = H_S^{-1} at full rank,
// and for a rank-deficient A PCG from x_0 = 0 then solves the least-squares problem on the kept columns
// (the basic solution: the dropped coordinates stay zero).
//
// The m x d sketch is copied to X (d x m, one row per column of S A) so that a column is contiguous.  Step
// k: one workgroup picks the pivot and swaps two rows of X (which carries the computed parts of R along),
// one workgroup forms the reflector of column k, and one wavefront per trailing column applies it and
// recomputes that column's remaining norm exactly (no downdating).
#include "internal.h"

namespace lsq {

constexpr int QP_NT = 1024;

__global__ __launch_bounds__(256) void k_qrcp_init(const double* __restrict__ SA, int64_t m, int64_t d, int64_t lds,
                                                   double* __restrict__ X) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * d) return;
  const int64_t i = idx / d, j = idx % d;  // coalesced reads of SA
  X[j * m + i] = SA[i * lds + j];
}

// norms[j] = ||X[j][from..m)||^2, one wavefront per column
__global__ __launch_bounds__(256) void k_qrcp_norms(const double* __restrict__ X, int64_t m, int64_t d,
                                                    double* __restrict__ norms, int* __restrict__ perm) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= d) return;
  double s = 0.0;
  for (int64_t i = lane; i < m; i += 64) s = fma(X[j * m + i], X[j * m + i], s);
  s = wave_sum(s);
  if (lane == 0) {
    norms[j] = s;
    perm[j] = (int)j;
  }
}

// Pivot of step k: the largest remaining norm (first such j on ties); swap rows k and p of X.
__global__ __launch_bounds__(QP_NT) void k_qrcp_pivot(double* __restrict__ X, int64_t m, int64_t d, int64_t k,
                                                      double* __restrict__ norms, int* __restrict__ perm) {
  __shared__ double sv[QP_NT / 64];
  __shared__ int si[QP_NT / 64];
  __shared__ int sp;
  double best = -1.0;
  int bi = (int)k;
  for (int64_t j = k + threadIdx.x; j < d; j += QP_NT) {
    const double v = norms[j];
    if (v > best) {
      best = v;
      bi = (int)j;
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ov > best || (ov == best && oi < bi)) {
      best = ov;
      bi = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = best;
    si[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = sv[0];
    int p = si[0];
    for (int w = 1; w < QP_NT / 64; ++w)
      if (sv[w] > b || (sv[w] == b && si[w] < p)) {
        b = sv[w];
        p = si[w];
      }
    sp = p;
    if (p != k) {
      const double t = norms[k];
      norms[k] = norms[p];
      norms[p] = t;
      const int q = perm[k];
      perm[k] = perm[p];
      perm[p] = q;
    }
  }
  __syncthreads();
  const int64_t p = sp;
  if (p == k) return;
  for (int64_t i = threadIdx.x; i < m; i += QP_NT) {
    const double a = X[k * m + i];
    X[k * m + i] = X[p * m + i];
    X[p * m + i] = a;
  }
}

// Reflector of column k: x = X[k][k..m); beta = -sign(x_k) ||x||, v = (1, x_{k+1..} / (x_k - beta)),
// tau = (beta - x_k) / beta; X[k][k] = beta (R_kk), X[k][k+1..] = v.  A zero column gives tau = 0.
__global__ __launch_bounds__(QP_NT) void k_qrcp_house(double* __restrict__ X, int64_t m, int64_t k,
                                                      double* __restrict__ tau) {
  __shared__ double scr[QP_NT / 64 + 1];
  double* x = X + k * m;
  const double alpha = x[k];  // read before the barriers of the sum: thread 0 rewrites x[k] below
  double s[1] = {0.0};
  for (int64_t i = k + 1 + threadIdx.x; i < m; i += QP_NT) s[0] = fma(x[i], x[i], s[0]);
  block_sum<QP_NT, 1>(s, scr);
  const double nrm = sqrt(fma(alpha, alpha, s[0]));
  if (nrm == 0.0) {
    if (threadIdx.x == 0) tau[k] = 0.0;
    return;
  }
  const double beta = alpha >= 0.0 ? -nrm : nrm;
  const double scale = 1.0 / (alpha - beta);
  for (int64_t i = k + 1 + threadIdx.x; i < m; i += QP_NT) x[i] *= scale;
  if (threadIdx.x == 0) {
    tau[k] = (beta - alpha) / beta;
    x[k] = beta;
  }
}

// Columns j > k: w = v^T a_j, a_j -= tau w v, norms[j] = ||a_j[k+1..m)||^2.  One wavefront per column.
__global__ __launch_bounds__(256) void k_qrcp_apply(double* __restrict__ X, int64_t m, int64_t d, int64_t k,
                                                    const double* __restrict__ tau, double* __restrict__ norms) {
  const int lane = threadIdx.x & 63;
  const int64_t j = k + 1 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= d) return;
  const double* v = X + k * m;
  double* a = X + j * m;
  const double t = tau[k];
  double w = 0.0;
  for (int64_t i = k + 1 + lane; i < m; i += 64) w = fma(v[i], a[i], w);
  w = wave_sum(w) + a[k];
  const double tw = t * w;
  double s = 0.0;
  for (int64_t i = k + 1 + lane; i < m; i += 64) {
    const double ai = fma(-tw, v[i], a[i]);
    a[i] = ai;
    s = fma(ai, ai, s);
  }
  s = wave_sum(s);
  if (lane == 0) {
    a[k] -= tw;
    norms[j] = s;
  }
}

// Rank r (first k with |R_kk| <= rtol |R_00|), R11 (r x r, ld r) compact, and the permutation.
__global__ __launch_bounds__(256) void k_qrcp_r11(const double* __restrict__ X, int64_t m, int64_t d, double rtol,
                                                  double* __restrict__ R11, int* __restrict__ rank) {
  __shared__ int sr;
  if (threadIdx.x == 0) {
    const double r00 = fabs(X[0]);
    int r = 0;
    while (r < d && fabs(X[(int64_t)r * m + r]) > rtol * r00) ++r;
    sr = r;
    if (blockIdx.x == 0) *rank = r;
  }
  __syncthreads();
  const int64_t r = sr;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < r * r;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / r, j = idx % r;
    R11[idx] = i <= j ? X[j * m + i] : 0.0;  // R[i][j] = column j at row i
  }
}

// W[perm[i]][j] = Winv[i][j] (i, j < r), WT = W^T; R[i][perm[j]] = R[i][j] for rows i < r; zero elsewhere.
__global__ __launch_bounds__(256) void k_qrcp_out(const double* __restrict__ X, int64_t m, int64_t d,
                                                  const int* __restrict__ rank, const int* __restrict__ perm,
                                                  const double* __restrict__ Winv, double* __restrict__ R,
                                                  double* __restrict__ W, double* __restrict__ WT) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int64_t r = *rank;
  const int64_t i = idx / d, j = idx % d;
  const int64_t pj = perm[j];
  R[i * d + pj] = (i < r && i <= j) ? X[j * m + i] : 0.0;
  const int64_t pi = perm[i];
  const double w = (i < r && j < r) ? Winv[i * r + j] : 0.0;
  W[pi * d + j] = w;
  WT[j * d + pi] = w;
}

// X (m d), norms and tau (d each), R11, Winv, WTinv (d^2 each), perm (d ints, given d doubles)
size_t qrcp_scratch_len(int64_t m, int64_t d) { return (size_t)m * d + 3 * (size_t)d * d + 3 * (size_t)d + 8; }

int qrcp_precond(hipStream_t st, const double* SA, int64_t m, int64_t d, int64_t lds, double rtol, double* scratch,
                 double* trinv_scratch, double* R, double* W, double* WT, int* flags, int* hflags) {
  double* X = scratch;
  double* norms = X + m * d;
  double* tau = norms + d;
  double* R11 = tau + d;
  double* Winv = R11 + d * d;
  double* WTinv = Winv + d * d;
  int* perm = (int*)(WTinv + d * d);
  hipLaunchKernelGGL(k_qrcp_init, dim3((unsigned)((m * d + 255) / 256)), dim3(256), 0, st, SA, m, d, lds, X);
  hipLaunchKernelGGL(k_qrcp_norms, dim3((unsigned)((d + 3) / 4)), dim3(256), 0, st, X, m, d, norms, perm);
  const int64_t steps = d < m ? d : m;
  for (int64_t k = 0; k < steps; ++k) {
    hipLaunchKernelGGL(k_qrcp_pivot, dim3(1), dim3(QP_NT), 0, st, X, m, d, k, norms, perm);
    hipLaunchKernelGGL(k_qrcp_house, dim3(1), dim3(QP_NT), 0, st, X, m, k, tau);
    if (k + 1 < d)
      hipLaunchKernelGGL(k_qrcp_apply, dim3((unsigned)((d - k - 1 + 3) / 4)), dim3(256), 0, st, X, m, d, k, tau,
                         norms);
  }
  hipLaunchKernelGGL(k_qrcp_r11, dim3(64), dim3(256), 0, st, X, m, d, rtol, R11, flags);
  hipMemcpyAsync(hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  const int r = hflags[0];
  if (r < 1) return 0;
  tri_inverse(st, R11, r, Winv, WTinv, trinv_scratch);
  hipLaunchKernelGGL(k_qrcp_out, dim3((unsigned)((d * d + 255) / 256)), dim3(256), 0, st, X, m, d, flags, perm, Winv,
                     R, W, WT);
  return r;
}

}  // namespace lsq
