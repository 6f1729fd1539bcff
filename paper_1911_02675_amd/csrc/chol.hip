// Factor step through the Gram matrix (the paper's alternative to QR of S A: a Cholesky factor of
// H_S = (S A)^T (S A), Section 1.2 and Section 6).  With X = S A (m x d), R1 = chol(X^T X) is the factor
// itself; its error (about u kappa(X)^2 relative) only matters to the preconditioner once kappa(X)^2 u is
// no longer small, so a second pass, CholeskyQR2,
//     Q1 = X R1^{-1},  R2 = chol(Q1^T Q1),  R = R2 R1,
// runs only when the spread of diag(R1) exceeds CHOLQR_ONE_PASS_SPREAD (or when asked for); when the
// first factorization breaks down, the shifted form with a third pass
// (R1 = chol(X^T X + s I), s = 11 (m d + d (d + 1)) u ||X||_F^2).  Every product runs on the FP64
// matrix cores (v_mfma_f64_16x16x4); the Cholesky is blocked by 64 columns (one wavefront factors the
// diagonal block in registers and inverts it, then the block row and the trailing matrix are updated
// in parallel).
// All matrices are row-major and padded to dp = 64 ceil(d / 64) columns, with the identity on the
// padding of every Gram matrix so that the padded factors are diag(R, I).
#include "internal.h"

namespace lsq {

typedef double lsq_c_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ lsq_c_d4 mfma_d(double a, double b, lsq_c_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int CQ_T = 64;   // tile edge
constexpr int CQ_KS = 16;  // rows of X per LDS stage
constexpr int CQ_LP = 65;  // padded LDS row (doubles)

// --------------------------------------------------------------------------------------------------
// Gram partials: part[s] = X[rows of split s]^T X[rows of split s] on the upper 64 x 64 tiles.
// Grid (upper tile pairs, S).  Four wavefronts, each a 32 x 32 quarter of the tile (2 x 2 blocks of
// 16 x 16).  Stages of 32 rows of both 64-column slices pass through LDS; the next stage is loaded into
// registers while the MFMAs consume the current one.  Columns at or past d read as zero.  VEC: d and
// ldx even and X 16-byte aligned (16-byte loads of column pairs).
// --------------------------------------------------------------------------------------------------
constexpr int GR_KS = 32;  // rows of X per stage

template <bool VEC>
__global__ __launch_bounds__(256) void k_gram_part(const double* __restrict__ X, int64_t m, int64_t d,
                                                   int64_t ldx, int64_t dp, double* __restrict__ part) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  __shared__ double As[GR_KS][CQ_LP];
  __shared__ double Bs[GR_KS][CQ_LP];
  const int nt = (int)(dp / CQ_T);
  // tile pair p -> (bi, bj), bi <= bj, row-major over the upper triangle
  int p = blockIdx.x, bi = 0;
  while (p >= nt - bi) {
    p -= nt - bi;
    ++bi;
  }
  const int bj = bi + p;
  const int S = gridDim.y, s = blockIdx.y;
  const int64_t r0 = m * s / S, r1 = m * (s + 1) / S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = wv >> 1, wj = wv & 1;
  const int lr = tid >> 5, lc = (tid & 31) * 2;  // loader: rows lr + 8 i, columns lc, lc + 1 of both slices
  const int64_t i0 = (int64_t)bi * CQ_T, j0 = (int64_t)bj * CQ_T;
  d2 ra[4], rb[4];
  // loads are unconditional (addresses clamped into the matrix) and the values are masked when they
  // are stored to LDS, so that the next stage's loads stay in flight during the MFMAs
  const int64_t ca = i0 + lc, cb = j0 + lc;
  auto ldpair = [&](const double* xr, int64_t c) -> d2 {
    if constexpr (VEC)
      return *(const d2*)(xr + (c < d ? c : 0));
    else
      return (d2){xr[c < d ? c : 0], xr[c + 1 < d ? c + 1 : 0]};
  };
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = k0 + lr + 8 * i;
      const double* xr = X + (r < r1 ? r : r0) * ldx;
      ra[i] = ldpair(xr, ca);
      rb[i] = ldpair(xr, cb);
    }
  };
  lsq_c_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (lsq_c_d4){0.0, 0.0, 0.0, 0.0};
  load(r0);
  for (int64_t k0 = r0; k0 < r1; k0 += GR_KS) {
    __syncthreads();  // the previous stage has been consumed
    // rows past r1 and columns past d as zero: multiplied by 0 (the loads read elements of X, which are
    // finite wherever the Gram is), so that no load is moved into a branch
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double rok = k0 + lr + 8 * i < r1 ? 1.0 : 0.0;
      As[lr + 8 * i][lc] = ra[i].x * (ca < d ? rok : 0.0);
      As[lr + 8 * i][lc + 1] = ra[i].y * (ca + 1 < d ? rok : 0.0);
      Bs[lr + 8 * i][lc] = rb[i].x * (cb < d ? rok : 0.0);
      Bs[lr + 8 * i][lc + 1] = rb[i].y * (cb + 1 < d ? rok : 0.0);
    }
    __syncthreads();
    load(k0 + GR_KS);  // past r1: never stored
    asm volatile("" ::: "memory");  // keeps the loads here, ahead of the MFMAs
#pragma unroll
    for (int kk = 0; kk < GR_KS; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kk + (lane >> 4)][32 * wi + 16 * a + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + (lane >> 4)][32 * wj + 16 * b + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma_d(av[a], bv[b], acc[a][b]);
    }
  }
  double* out = part + (int64_t)s * dp * dp;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + 32 * wi + 16 * a + (lane >> 4) + 4 * v;
        const int64_t j = j0 + 32 * wj + 16 * b + (lane & 15);
        out[i * dp + j] = acc[a][b][v];
      }
}

// G = sum_s part[s] on the upper tiles (fixed order), plus the identity on the padding and an optional
// shift on the diagonal.
__global__ void k_gram_reduce(const double* __restrict__ part, int S, int64_t d, int64_t dp,
                              const double* __restrict__ shift, double* __restrict__ G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= dp * dp) return;
  const int64_t i = idx / dp, j = idx % dp;
  if (i / CQ_T > j / CQ_T) return;  // lower tiles are never read
  double v = 0.0;
  for (int s = 0; s < S; ++s) v += part[(int64_t)s * dp * dp + idx];
  if (i == j) v = i < d ? v + (shift ? *shift : 0.0) : 1.0;
  G[idx] = v;
}

// G_ii += s for i < d.
__global__ void k_gram_add_shift(double* __restrict__ G, int64_t d, int64_t dp, const double* __restrict__ shift) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d) G[i * dp + i] += *shift;
}

// s = 11 (m d + d (d + 1)) u tr(G) with tr(G) = ||X||_F^2 (one workgroup).
__global__ __launch_bounds__(1024) void k_gram_shift(const double* __restrict__ G, int64_t m, int64_t d,
                                                     int64_t dp, double* __restrict__ shift) {
  __shared__ double sh[16];
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 1024) t += G[i * dp + i];
  t = grp_sum<64>(t);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += sh[w];
    *shift = 11.0 * ((double)m * (double)d + (double)d * (double)(d + 1)) * 1.1102230246251565e-16 * s;
  }
}

// --------------------------------------------------------------------------------------------------
// Blocked Cholesky G = R^T R (upper), 64-column blocks.
// --------------------------------------------------------------------------------------------------
// Diagonal block kb in one wavefront: lane j holds column j of the block in registers.  Step k takes
// the pivot from lane k, scales row k (element k of every lane), publishes it through LDS, and every
// lane subtracts r_ki r_kj from its elements i > k.  Entries below the diagonal (i > j in lane j) are
// updated too, without masks, and never read into a result: this keeps the step free of per-element
// selects, so the LDS reads of row k can all be in flight together.  Then R_kk and its inverse are
// written; the inverse overwrites the registers bottom-up (row i of X = R_kk^{-1} needs rows k > i of X
// and row i of R_kk, which stays in LDS).  A pivot that is not positive sets *flag and is replaced by 1
// so that the factorization completes.

// 1 / sqrt(p) for p > 0: the hardware estimate and two Newton steps y <- y + (y / 2)(1 - p y^2), each of
// which squares the relative error, to within about an ulp.
__device__ __forceinline__ double rsqrt_newton(double p) {
  double y = __builtin_amdgcn_rsq(p);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-p * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

__global__ __launch_bounds__(64) void k_chol_diag(const double* __restrict__ G, int64_t dp, int kb,
                                                  double* __restrict__ R, double* __restrict__ Dinv,
                                                  int* __restrict__ flag) {
  __shared__ double Rs[CQ_T][CQ_LP];
  const int j = threadIdx.x;
  const int64_t o = (int64_t)kb * CQ_T;
  double a[CQ_T];
#pragma unroll
  for (int i = 0; i < CQ_T; ++i) a[i] = i <= j ? G[(o + i) * dp + o + j] : 0.0;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < CQ_T; ++k) {
    const double piv = readlane_d(a[k], k);
    bad = bad || !(piv > 0.0);
    // r_kk = sqrt(piv) and its reciprocal from one refined reciprocal square root (no division on the
    // step's serial chain)
    const double inv = piv > 0.0 ? rsqrt_newton(piv) : 1.0;
    const double rkk = piv > 0.0 ? piv * inv : 1.0;
    a[k] = j == k ? rkk : a[k] * inv;
    Rs[k][j] = a[k];  // row k of R_kk in entries j >= k
    __syncthreads();
#pragma unroll
    for (int i = k + 1; i < CQ_T; ++i) a[i] = fma(-Rs[k][i], a[k], a[i]);
    __builtin_amdgcn_sched_barrier(0);  // one step at a time: hoisting later steps' reads only adds registers
  }
  if (j == 0 && bad) *flag = 1;
#pragma unroll
  for (int i = 0; i < CQ_T; ++i) R[(o + i) * dp + o + j] = i <= j ? a[i] : 0.0;
  // inverse, column j: X[i][j] = (delta_ij - sum_{k > i} R[i][k] X[k][j]) / R[i][i], i = 63 .. 0, with
  // X[k][j] = 0 for k > j
#pragma unroll
  for (int i = CQ_T - 1; i >= 0; --i) {
    double s = 0.0;
#pragma unroll
    for (int k = i + 1; k < CQ_T; ++k) s = fma(Rs[i][k], a[k], s);
    a[i] = i > j ? 0.0 : ((i == j ? 1.0 : -s) / Rs[i][i]);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = 0; i < CQ_T; ++i) Dinv[i * CQ_T + j] = a[i];
}

// Block row kb: R_kj = Dinv^T G_kj for column tiles right of the diagonal block.  One wavefront per
// 16 x 16 output block; grid covers 4 row blocks x the 16-column blocks right of the diagonal.
__global__ __launch_bounds__(256) void k_chol_row(const double* __restrict__ G, int64_t dp, int kb,
                                                  const double* __restrict__ Dinv, double* __restrict__ R) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)(kb + 1) * CQ_T;
  const int ncb = (int)((dp - c0) / 16);
  const int blk = blockIdx.x * 4 + wv;
  if (blk >= 4 * ncb) return;  // whole wavefronts
  const int ib = blk / ncb, jb = blk % ncb;
  const int64_t o = (int64_t)kb * CQ_T;
  const int li = lane & 15, lk = lane >> 4;
  lsq_c_d4 acc = {0.0, 0.0, 0.0, 0.0};
  // (Dinv^T)[i][k] = Dinv[k][i], nonzero for k <= i
  const int kend = 16 * (ib + 1);
  for (int k = 0; k < kend; k += 4) {
    const double a = Dinv[(k + lk) * CQ_T + 16 * ib + li];
    const double b = G[(o + k + lk) * dp + c0 + 16 * jb + li];
    acc = mfma_d(a, b, acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) R[(o + 16 * ib + lk + 4 * v) * dp + c0 + 16 * jb + li] = acc[v];
}

// Trailing update: G_ij -= R_ki^T R_kj (K = 64) on the upper 16 x 16 blocks right of and below block kb.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ G, int64_t dp, int kb,
                                                     const double* __restrict__ R) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)(kb + 1) * CQ_T;
  const int nb = (int)((dp - c0) / 16);
  int p = blockIdx.x * 4 + wv;
  if (p >= nb * (nb + 1) / 2) return;  // whole wavefronts
  int bi = 0;
  while (p >= nb - bi) {
    p -= nb - bi;
    ++bi;
  }
  const int bj = bi + p;
  const int64_t o = (int64_t)kb * CQ_T;
  const int li = lane & 15, lk = lane >> 4;
  lsq_c_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k = 0; k < CQ_T; k += 4) {
    const double a = R[(o + k + lk) * dp + c0 + 16 * bi + li];  // (R_k.)^T[i][k] = R[k][i]
    const double b = R[(o + k + lk) * dp + c0 + 16 * bj + li];
    acc = mfma_d(a, b, acc);
  }
  double* g = G + (c0 + 16 * bi) * dp + c0 + 16 * bj + li;
#pragma unroll
  for (int v = 0; v < 4; ++v) g[(int64_t)(lk + 4 * v) * dp] -= acc[v];
}

// --------------------------------------------------------------------------------------------------
// Q = X W with W upper triangular (dp x dp, identity on the padding): Q[r][j] = sum_{k <= j} X[r][k] W[k][j].
// Tile 64 rows x 64 columns per workgroup, four wavefronts of 32 x 32; stages of 32 values of k of X and W
// pass through LDS, the next stage's loads in flight during the MFMAs (as in the Gram kernel).  Column
// blocks are taken from the right (the most stages) first.  VEC: d and ldx even and X 16-byte aligned.
// --------------------------------------------------------------------------------------------------
template <bool VEC>
__global__ __launch_bounds__(256) void k_xw(const double* __restrict__ X, int64_t m, int64_t d, int64_t ldx,
                                            const double* __restrict__ W, int64_t dp, double* __restrict__ Q) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  __shared__ double Xs[CQ_T][GR_KS + 1];
  __shared__ double Ws[GR_KS][CQ_LP];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = wv >> 1, wj = wv & 1;
  const int64_t r0 = (int64_t)blockIdx.x * CQ_T, j0 = (int64_t)(gridDim.y - 1 - blockIdx.y) * CQ_T;
  // loaders: X row xr, columns xc .. xc + 7 of the stage; W row wr, columns wc .. wc + 7 of the tile
  const int xr = tid >> 2, xc = (tid & 3) * 8, wr = tid >> 3, wc = (tid & 7) * 8;
  const int64_t rx = r0 + xr;
  const double* xrow = X + (rx < m ? rx : m - 1) * ldx;  // rows past m are multiplied by 0 below
  const double xok = rx < m ? 1.0 : 0.0;
  d2 xv[4], wvv[4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t c = k0 + xc + 2 * e;
      if constexpr (VEC)
        xv[e] = *(const d2*)(xrow + (c < d ? c : 0));
      else
        xv[e] = (d2){xrow[c < d ? c : 0], xrow[c + 1 < d ? c + 1 : 0]};
    }
    const int64_t k = k0 + wr < dp ? k0 + wr : dp - 1;  // past the last stage: never stored
#pragma unroll
    for (int e = 0; e < 4; ++e) wvv[e] = *(const d2*)(W + k * dp + j0 + wc + 2 * e);
  };
  lsq_c_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (lsq_c_d4){0.0, 0.0, 0.0, 0.0};
  const int64_t kend = j0 + CQ_T;  // W[k][j] = 0 for k > j
  load(0);
  for (int64_t k0 = 0; k0 < kend; k0 += GR_KS) {
    __syncthreads();  // the previous stage has been consumed
    // columns past d and rows past m as zero (multiplied, so that no load is moved into a branch)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t c = k0 + xc + 2 * e;
      Xs[xr][xc + 2 * e] = xv[e].x * (c < d ? xok : 0.0);
      Xs[xr][xc + 2 * e + 1] = xv[e].y * (c + 1 < d ? xok : 0.0);
      Ws[wr][wc + 2 * e] = wvv[e].x;
      Ws[wr][wc + 2 * e + 1] = wvv[e].y;
    }
    __syncthreads();
    load(k0 + GR_KS);
    asm volatile("" ::: "memory");  // keeps the loads here, ahead of the MFMAs
#pragma unroll
    for (int kk = 0; kk < GR_KS; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Xs[32 * wi + 16 * a + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Ws[kk + (lane >> 4)][32 * wj + 16 * b + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma_d(av[a], bv[b], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + 32 * wi + 16 * a + (lane >> 4) + 4 * v;
        const int64_t j = j0 + 32 * wj + 16 * b + (lane & 15);
        if (r < m) Q[r * dp + j] = acc[a][b][v];
      }
}

static void launch_xw(hipStream_t st, dim3 grid, const double* X, int64_t m, int64_t d, int64_t ldx,
                      const double* W, int64_t dp, double* Q) {
  if (d % 2 == 0 && ldx % 2 == 0 && (uintptr_t)X % 16 == 0)
    hipLaunchKernelGGL(k_xw<true>, grid, dim3(256), 0, st, X, m, d, ldx, W, dp, Q);
  else
    hipLaunchKernelGGL(k_xw<false>, grid, dim3(256), 0, st, X, m, d, ldx, W, dp, Q);
}

// C = A B for upper triangular A, B (dp x dp): C[i][j] = sum_{i <= k <= j} A[i][k] B[k][j], upper 16 x 16
// blocks, one wavefront each; the strictly lower blocks of C are cleared.
__global__ __launch_bounds__(256) void k_trtr(const double* __restrict__ A, const double* __restrict__ B,
                                              int64_t dp, double* __restrict__ C) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nb = (int)(dp / 16);
  const int blk = blockIdx.x * 4 + wv;
  if (blk >= nb * nb) return;  // whole wavefronts
  const int bi = blk / nb, bj = blk % nb;
  const int li = lane & 15, lk = lane >> 4;
  double* c = C + (int64_t)(16 * bi) * dp + 16 * bj + li;
  if (bi > bj) {
#pragma unroll
    for (int v = 0; v < 4; ++v) c[(int64_t)(lk + 4 * v) * dp] = 0.0;
    return;
  }
  lsq_c_d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k = 16 * bi; k < 16 * (bj + 1); k += 4) {
    const double a = A[(int64_t)(16 * bi + li) * dp + k + lk];
    const double b = B[(int64_t)(k + lk) * dp + 16 * bj + li];
    acc = mfma_d(a, b, acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) c[(int64_t)(lk + 4 * v) * dp] = acc[v];
}

// R (d x d) from the padded factor; the lower triangle is zero.
__global__ void k_chol_extract(const double* __restrict__ Rp, int64_t dp, int64_t d, double* __restrict__ R) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int64_t i = idx / d, j = idx % d;
  R[idx] = j >= i ? Rp[i * dp + j] : 0.0;
}

// The spread max |R_jj| / min |R_jj| of the first factor: above lim, *flag = 1 (too inaccurate for two passes);
// else above lim2, *flag = 2 (the second pass is needed); else *flag stays 0.
__global__ __launch_bounds__(1024) void k_chol_diagratio(const double* __restrict__ Rp, int64_t dp, int64_t d,
                                                         double lim, double lim2, int* __restrict__ flag) {
  __shared__ double smx[16], smn[16];
  double mx = 0.0, mn = INFINITY;
  for (int64_t i = threadIdx.x; i < d; i += 1024) {
    const double v = fabs(Rp[i * dp + i]);
    mx = fmax(mx, v);
    mn = fmin(mn, v);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    mn = fmin(mn, __shfl_xor(mn, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    smx[threadIdx.x >> 6] = mx;
    smn[threadIdx.x >> 6] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < 16; ++w) {
      mx = fmax(mx, smx[w]);
      mn = fmin(mn, smn[w]);
    }
    if (!(mx <= lim * mn))
      *flag = 1;
    else if (!(mx <= lim2 * mn))
      *flag = 2;
  }
}

// --------------------------------------------------------------------------------------------------
// Host side.
// --------------------------------------------------------------------------------------------------
int64_t cholqr_padded(int64_t d) { return (d + CQ_T - 1) / CQ_T * CQ_T; }

int g_gram_wgs = 2048;

static int gram_splits(int64_t m, int64_t dp) {
  const int64_t tiles = (dp / CQ_T) * (dp / CQ_T + 1) / 2;
  // about g_gram_wgs (2048) workgroups: two rounds of four per compute unit (33 KB of LDS each), so that
  // the last round is nearly full
  int64_t s = (g_gram_wgs + tiles / 2) / tiles;
  const int64_t smax = (m + 255) / 256;  // at least 256 rows per split
  s = s > smax ? smax : s;
  return (int)(s < 1 ? 1 : (s > 32 ? 32 : s));
}

size_t cholqr_scratch_len(int64_t m, int64_t d) {
  const int64_t dp = cholqr_padded(d);
  // part (S dp^2), G, Ra, Rb, Rc, W (dp^2 each), Dinv (64^2), Q and Q2 (m dp each), shift
  return (size_t)gram_splits(m, dp) * dp * dp + 5 * (size_t)dp * dp + CQ_T * CQ_T + 2 * (size_t)m * dp + 8;
}

static void gram(hipStream_t st, const double* X, int64_t m, int64_t d, int64_t ldx, int64_t dp, double* part,
                 const double* shift, double* G) {
  const int S = gram_splits(m, dp);
  const int64_t nt = dp / CQ_T;
  const dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)S);
  if (d % 2 == 0 && ldx % 2 == 0 && (uintptr_t)X % 16 == 0)
    hipLaunchKernelGGL(k_gram_part<true>, grid, dim3(256), 0, st, X, m, d, ldx, dp, part);
  else
    hipLaunchKernelGGL(k_gram_part<false>, grid, dim3(256), 0, st, X, m, d, ldx, dp, part);
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((dp * dp + 255) / 256)), dim3(256), 0, st, part, S, d, dp, shift,
                     G);
}

static void cholesky(hipStream_t st, double* G, int64_t dp, double* R, double* Dinv, int* flag) {
  hipMemsetAsync(R, 0, (size_t)dp * dp * sizeof(double), st);
  const int nkb = (int)(dp / CQ_T);
  for (int kb = 0; kb < nkb; ++kb) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(64), 0, st, G, dp, kb, R, Dinv, flag);
    const int64_t rest = dp - (int64_t)(kb + 1) * CQ_T;
    if (rest <= 0) break;
    const int64_t ncb = rest / 16;
    hipLaunchKernelGGL(k_chol_row, dim3((unsigned)((4 * ncb + 3) / 4)), dim3(256), 0, st, G, dp, kb, Dinv, R);
    const int64_t nup = ncb * (ncb + 1) / 2;
    hipLaunchKernelGGL(k_chol_update, dim3((unsigned)((nup + 3) / 4)), dim3(256), 0, st, G, dp, kb, R);
  }
}

// One CholeskyQR pass on X (m x d used columns, leading dimension ldx): Rout = chol(X^T X [+ shift I])
// padded to dp with the identity.
static void cq_pass(hipStream_t st, const double* X, int64_t m, int64_t d, int64_t ldx, int64_t dp, double* part,
                    double* G, const double* shift, double* Rout, double* Dinv, int* flag) {
  gram(st, X, m, d, ldx, dp, part, shift, G);
  cholesky(st, G, dp, Rout, Dinv, flag);
}

int cholqr_factor(hipStream_t st, const double* SA, int64_t m, int64_t d, int64_t lds, double* scratch,
                  double* R, int* flags, int* hflags, double* trinv_scratch, int passes) {
  const int64_t dp = cholqr_padded(d);
  const int S = gram_splits(m, dp);
  double* part = scratch;
  double* G = part + (size_t)S * dp * dp;
  double* Ra = G + dp * dp;
  double* Rb = Ra + dp * dp;
  double* Rc = Rb + dp * dp;
  double* Wt = Rc + dp * dp;
  double* Dinv = Wt + dp * dp;
  double* Q = Dinv + CQ_T * CQ_T;
  double* Q2 = Q + (size_t)m * dp;
  double* shift = Q2 + (size_t)m * dp;
  const dim3 gx((unsigned)((m + CQ_T - 1) / CQ_T), (unsigned)(dp / CQ_T));
  // pass 1, then a check that it is usable for two passes, and whether it is accurate enough alone
  hipMemsetAsync(flags, 0, 2 * sizeof(int), st);
  cq_pass(st, SA, m, d, lds, dp, part, G, nullptr, Ra, Dinv, flags);
  hipLaunchKernelGGL(k_chol_diagratio, dim3(1), dim3(1024), 0, st, Ra, dp, d, 1e7, CHOLQR_ONE_PASS_SPREAD,
                     flags + 1);
  hipMemcpyAsync(hflags, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  if (hflags[0] || hflags[1] == 1) return 1;  // caller chooses the robust path
  if (passes == 1 || (passes == 0 && hflags[1] == 0)) {
    // R = chol(X^T X), the Cholesky factor of H_S itself.  Its error (about u kappa^2 relative, against
    // u kappa after the second pass) only perturbs the preconditioned operator R^{-T} A^T A R^{-1} by a
    // factor 1 + O(u kappa^2): invisible in the PCG iteration count while the spread is small.
    hipLaunchKernelGGL(k_chol_extract, dim3((unsigned)((d * d + 255) / 256)), dim3(256), 0, st, Ra, dp, d, R);
    return 0;
  }
  // Q1 = X R1^{-1}; pass 2 on Q1; R = R2 R1
  tri_inverse_padded(st, Ra, dp, Wt, trinv_scratch);
  launch_xw(st, gx, SA, m, d, lds, Wt, dp, Q);
  cq_pass(st, Q, m, d, dp, dp, part, G, nullptr, Rb, Dinv, flags);
  hipLaunchKernelGGL(k_trtr, dim3((unsigned)((dp / 16) * (dp / 16) / 4 + 1)), dim3(256), 0, st, Rb, Ra, dp, Rc);
  hipLaunchKernelGGL(k_chol_extract, dim3((unsigned)((d * d + 255) / 256)), dim3(256), 0, st, Rc, dp, d, R);
  return 0;
}

// ---- Haar embedding ------------------------------------------------------------------------------
// G (dp x dp) = scale Z on the leading md x md block (Z row-major, ld md), the identity on the padding.
__global__ __launch_bounds__(256) void k_pad_spd(const double* __restrict__ Z, int64_t md, int64_t dp, double scale,
                                                 double* __restrict__ G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= dp * dp) return;
  const int64_t i = idx / dp, j = idx % dp;
  G[idx] = (i < md && j < md) ? scale * Z[i * md + j] : (i == j ? 1.0 : 0.0);
}

size_t spd_inverse_scratch_len(int64_t md) {
  const int64_t dp = cholqr_padded(md);
  return 2 * (size_t)dp * dp + CQ_T * CQ_T;
}

void spd_chol_inverse(hipStream_t st, const double* Z, int64_t md, double scale, double* scratch, double* W,
                      int* flag, double* trinv_scratch) {
  const int64_t dp = cholqr_padded(md);
  double* G = scratch;
  double* R = G + dp * dp;
  double* Dinv = R + dp * dp;
  hipLaunchKernelGGL(k_pad_spd, dim3((unsigned)((dp * dp + 255) / 256)), dim3(256), 0, st, Z, md, dp, scale, G);
  cholesky(st, G, dp, R, Dinv, flag);
  tri_inverse_padded(st, R, dp, W, trinv_scratch);
}

// SA[i][c] = scale sum_{k <= i} W[k][i] Y[k][c]  (SA = scale W^T Y, W upper triangular, ld ldw).  One thread
// per output; a wavefront shares i, so W is read as a broadcast and Y row by row.
__global__ __launch_bounds__(256) void k_haar_apply(const double* __restrict__ W, int64_t ldw,
                                                    const double* __restrict__ Y, int64_t m, int64_t d,
                                                    double scale, double* __restrict__ SA, int64_t ldsa) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * d) return;
  const int64_t i = idx / d, c = idx % d;
  double s0 = 0.0, s1 = 0.0;
  int64_t k = 0;
  for (; k + 1 <= i; k += 2) {
    s0 = fma(W[k * ldw + i], Y[k * d + c], s0);
    s1 = fma(W[(k + 1) * ldw + i], Y[(k + 1) * d + c], s1);
  }
  if (k <= i) s0 = fma(W[k * ldw + i], Y[k * d + c], s0);
  SA[i * ldsa + c] = scale * (s0 + s1);
}

void haar_apply(hipStream_t st, const double* W, int64_t ldw, const double* Y, int64_t m, int64_t d, double scale,
                double* SA, int64_t ldsa) {
  hipLaunchKernelGGL(k_haar_apply, dim3((unsigned)((m * d + 255) / 256)), dim3(256), 0, st, W, ldw, Y, m, d, scale,
                     SA, ldsa);
}

int cholqr3_shifted(hipStream_t st, const double* SA, int64_t m, int64_t d, int64_t lds, double* scratch,
                    double* R, int* flags, double* trinv_scratch) {
  const int64_t dp = cholqr_padded(d);
  const int S = gram_splits(m, dp);
  double* part = scratch;
  double* G = part + (size_t)S * dp * dp;
  double* Ra = G + dp * dp;
  double* Rb = Ra + dp * dp;
  double* Rc = Rb + dp * dp;
  double* Wt = Rc + dp * dp;
  double* Dinv = Wt + dp * dp;
  double* Q = Dinv + CQ_T * CQ_T;
  double* Q2 = Q + (size_t)m * dp;
  double* shift = Q2 + (size_t)m * dp;
  const dim3 gx((unsigned)((m + CQ_T - 1) / CQ_T), (unsigned)(dp / CQ_T));
  const unsigned gt = (unsigned)((dp / 16) * (dp / 16) / 4 + 1);
  hipMemsetAsync(flags, 0, sizeof(int), st);
  // shift from ||X||_F^2 = tr(X^T X), then R1 = chol(X^T X + s I)
  gram(st, SA, m, d, lds, dp, part, nullptr, G);
  hipLaunchKernelGGL(k_gram_shift, dim3(1), dim3(1024), 0, st, G, m, d, dp, shift);
  hipLaunchKernelGGL(k_gram_add_shift, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, G, d, dp, shift);
  cholesky(st, G, dp, Ra, Dinv, flags);
  // Q1 = X R1^{-1}, R2 = chol(Q1^T Q1), R21 = R2 R1
  tri_inverse_padded(st, Ra, dp, Wt, trinv_scratch);
  launch_xw(st, gx, SA, m, d, lds, Wt, dp, Q);
  cq_pass(st, Q, m, d, dp, dp, part, G, nullptr, Rb, Dinv, flags);
  hipLaunchKernelGGL(k_trtr, dim3(gt), dim3(256), 0, st, Rb, Ra, dp, Rc);
  // Q2 = Q1 R2^{-1}, R3 = chol(Q2^T Q2), R = R3 R21
  tri_inverse_padded(st, Rb, dp, Wt, trinv_scratch);
  launch_xw(st, gx, Q, m, d, dp, Wt, dp, Q2);
  cq_pass(st, Q2, m, d, dp, dp, part, G, nullptr, Ra, Dinv, flags);
  hipLaunchKernelGGL(k_trtr, dim3(gt), dim3(256), 0, st, Ra, Rc, dp, Rb);
  hipLaunchKernelGGL(k_chol_extract, dim3((unsigned)((d * d + 255) / 256)), dim3(256), 0, st, Rb, dp, d, R);
  return 0;
}

}  // namespace lsq
