// SVD preconditioner (the factor step of Section 1.2 in the LSRN form): with S A = Q R, the right singular
// vectors and singular values of S A are those of the d x d R.  One-sided Jacobi (Hestenes) rotates pairs
// of columns of R until all are mutually orthogonal, R V = U Sigma; then
//     P = V Sigma^+ (singular values below rtol * sigma_max dropped),  P P^T = H_S^+,
// replaces R^{-1} in PCG (the preconditioner becomes two dense GEMVs), and R is returned as Sigma V^T
// (R^T R = H_S on the kept subspace).  For a rank-deficient A the iterates from x_0 = 0 stay in the row
// space, so PCG converges to the minimum-norm solution.
//
// Columns are kept as rows of C = R^T (and of V^T), so a column pair is two contiguous rows.  Each sweep
// visits every pair once in the round-robin (circle) order: d2 - 1 rounds of d2 / 2 disjoint pairs
// (d2 = d rounded up to even; a pair with the padding index is idle), one wavefront per pair and one
// launch per round.  A sweep without a rotation ends the iteration.
#include "internal.h"

namespace lsq {

__global__ __launch_bounds__(256) void k_jac_init(const double* __restrict__ R, int64_t d, double* __restrict__ C,
                                                  double* __restrict__ VT) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int64_t i = idx / d, j = idx % d;
  C[idx] = R[j * d + i];
  VT[idx] = i == j ? 1.0 : 0.0;
}

__global__ __launch_bounds__(256) void k_jac_round(double* __restrict__ C, double* __restrict__ VT, int64_t d,
                                                   int64_t d2, int64_t k, double tol, int* __restrict__ rotated) {
  const int lane = threadIdx.x & 63;
  const int64_t pr = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (pr >= d2 / 2) return;  // whole wavefronts
  const int64_t M = d2 - 1;
  const int64_t p = pr == 0 ? M : (k + pr) % M;
  const int64_t q = pr == 0 ? k : (k - pr + M) % M;
  if (p >= d || q >= d) return;
  double* cp = C + p * d;
  double* cq = C + q * d;
  double a = 0.0, b = 0.0, g = 0.0;
  for (int64_t i = lane; i < d; i += 64) {
    const double x = cp[i], y = cq[i];
    a = fma(x, x, a);
    b = fma(y, y, b);
    g = fma(x, y, g);
  }
  a = wave_sum(a);
  b = wave_sum(b);
  g = wave_sum(g);
  if (!(fabs(g) > tol * sqrt(a * b))) return;  // orthogonal to working accuracy (or a zero column)
  // x' = c x - s y, y' = s x + c y with x'.y' = 0: t = s / c solves t^2 + 2 zeta t - 1 = 0, smaller root
  const double zeta = (b - a) / (2.0 * g);
  const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
  for (int64_t i = lane; i < d; i += 64) {
    const double x = cp[i], y = cq[i];
    cp[i] = c * x - s * y;
    cq[i] = s * x + c * y;
  }
  double* vp = VT + p * d;
  double* vq = VT + q * d;
  for (int64_t i = lane; i < d; i += 64) {
    const double x = vp[i], y = vq[i];
    vp[i] = c * x - s * y;
    vq[i] = s * x + c * y;
  }
  if (lane == 0) *rotated = 1;
}

// sigma[p] = ||row p of C||, one wavefront per row.
__global__ __launch_bounds__(256) void k_jac_norms(const double* __restrict__ C, int64_t d, double* __restrict__ sigma) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= d) return;
  double s = 0.0;
  for (int64_t i = lane; i < d; i += 64) s = fma(C[p * d + i], C[p * d + i], s);
  s = wave_sum(s);
  if (lane == 0) sigma[p] = sqrt(s);
}

// W[i][p] = V[i][p] / sigma_p, WT = W^T, R[p][j] = sigma_p V[j][p] for kept p (sigma_p > rtol sigma_max),
// zero otherwise; *rank = number kept.  One block of 1024 threads finds sigma_max; the grid writes.
__global__ __launch_bounds__(256) void k_jac_out(const double* __restrict__ VT, const double* __restrict__ sigma,
                                                 int64_t d, double rtol, double* __restrict__ R, double* __restrict__ W,
                                                 double* __restrict__ WT, int* __restrict__ rank) {
  __shared__ double smax[4];
  __shared__ int scnt[4];
  double mx = 0.0;
  for (int64_t p = threadIdx.x; p < d; p += 256) mx = fmax(mx, sigma[p]);
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
  const double cut = rtol * mx;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0) {
    int cnt = 0;
    for (int64_t p = threadIdx.x; p < d; p += 256) cnt += sigma[p] > cut ? 1 : 0;
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if ((threadIdx.x & 63) == 0) scnt[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) *rank = scnt[0] + scnt[1] + scnt[2] + scnt[3];
  }
  if (idx >= d * d) return;
  const int64_t p = idx / d, j = idx % d;  // row p of V^T, entry j = V[j][p]
  const double sp = sigma[p];
  const bool keep = sp > cut;
  const double v = VT[idx];
  R[p * d + j] = keep ? sp * v : 0.0;
  W[j * d + p] = keep ? v / sp : 0.0;
  WT[p * d + j] = keep ? v / sp : 0.0;
}

// xout = M xin (dense d x d, row-major), one wavefront per row; with DOT also the per-block partials of
// xout . rdot (the layout precond_apply leaves for the PCG update).
template <bool DOT>
__global__ __launch_bounds__(256) void k_gemv_dense(const double* __restrict__ M, int64_t d,
                                                    const double* __restrict__ xin, double* __restrict__ xout,
                                                    const double* __restrict__ rdot, double* __restrict__ dotpart,
                                                    const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  double prod = 0.0;
  if (i < d) {
    const double* row = M + i * d;
    double s = 0.0;
    for (int64_t k = lane; k < d; k += 64) s = fma(row[k], xin[k], s);
    s = wave_sum(s);
    if (lane == 0) xout[i] = s;
    if (DOT) prod = s * rdot[i];
  }
  if (DOT) {
    if (lane == 0) sh[wv] = prod;
    __syncthreads();
    if (threadIdx.x == 0) dotpart[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
  }
}

void precond_apply_any(hipStream_t st, const double* W, const double* WT, int64_t d, const double* r, double* u,
                       double* rhat, double* dotpart, int* ndot, const int* done, int dense) {
  if (!dense) {
    precond_apply(st, W, WT, d, r, u, rhat, dotpart, ndot, done);
    return;
  }
  const unsigned nb = (unsigned)((d + 3) / 4);
  hipLaunchKernelGGL(k_gemv_dense<false>, dim3(nb), dim3(256), 0, st, WT, d, r, u, nullptr, nullptr, done);
  hipLaunchKernelGGL(k_gemv_dense<true>, dim3(nb), dim3(256), 0, st, W, d, u, rhat, r, dotpart, done);
  *ndot = (int)nb;
}

size_t svd_scratch_len(int64_t d) { return 2 * (size_t)d * d + (size_t)d; }

int svd_precond(hipStream_t st, double* R, int64_t d, double rtol, double* scratch, double* W, double* WT,
                int* flags, int* hflags, int* sweeps_out) {
  double* C = scratch;
  double* VT = C + d * d;
  double* sigma = VT + d * d;
  const int64_t d2 = (d + 1) / 2 * 2;
  const unsigned nb = (unsigned)((d * d + 255) / 256);
  hipLaunchKernelGGL(k_jac_init, dim3(nb), dim3(256), 0, st, R, d, C, VT);
  const double tol = 4.0 * (double)d * 2.220446049250313e-16;
  const unsigned rb = (unsigned)((d2 / 2 + 3) / 4);
  int sweeps = 0;
  for (; sweeps < SVD_MAX_SWEEPS; ++sweeps) {
    hipMemsetAsync(flags, 0, sizeof(int), st);
    for (int64_t k = 0; k < d2 - 1; ++k)
      hipLaunchKernelGGL(k_jac_round, dim3(rb), dim3(256), 0, st, C, VT, d, d2, k, tol, flags);
    hipMemcpyAsync(hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    if (!hflags[0]) break;
  }
  *sweeps_out = sweeps + 1;
  hipLaunchKernelGGL(k_jac_norms, dim3((unsigned)((d + 3) / 4)), dim3(256), 0, st, C, d, sigma);
  hipLaunchKernelGGL(k_jac_out, dim3(nb), dim3(256), 0, st, VT, sigma, d, rtol, R, W, WT, flags + 1);
  hipMemcpyAsync(hflags + 1, flags + 1, sizeof(int), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  return hflags[1];
}

}  // namespace lsq
