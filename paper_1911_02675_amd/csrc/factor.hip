// Factor step of the preconditioner (Section 1.2): H_S = (S A)^T (S A) = R^T R with R from a
// Householder QR of S A (m x d, m >= d), sign-normalised so that diag(R) > 0, and W = R^{-1}.
//
// Blocked Householder with panels of BW columns, one launch per panel.  Every workgroup (512
// threads) redundantly factors the m x BW panel in registers, builds the compact-WY
// factor T (Q_panel = I - V T V^T), and applies Q_panel^T to its own share of the trailing columns.
// No grid-wide synchronisation is needed inside a launch; the panel is re-read from L2/MALL by each
// workgroup instead.  Column-major scratch X keeps every column contiguous.
#include <algorithm>

#include "internal.h"

namespace lsq {

constexpr int QR_NT = 512;

__global__ void k_to_colmajor(const double* __restrict__ SA, int64_t m, int64_t d, int64_t lds,
                              double* __restrict__ X) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    tile[k][tx] = (r < m && c < d) ? SA[r * lds + c] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (r < m && c < d) X[c * m + r] = tile[tx][k];
  }
}

template <int RPT, int BW, int CB>
__global__ __launch_bounds__(QR_NT) void k_qr_panel(double* __restrict__ X, int64_t m, int64_t d,
                                                    int64_t k0, double* __restrict__ Rraw) {
  __shared__ double red[(QR_NT / 64) * (BW * CB > BW ? BW * CB : BW) + 64];
  __shared__ double Ts[BW][BW];
  const int tid = threadIdx.x;
  const int bw = (int)min((int64_t)BW, d - k0);
  double P[RPT][BW];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int64_t r = tid + (int64_t)QR_NT * i;
#pragma unroll
    for (int j = 0; j < BW; ++j) P[i][j] = (j < bw && r >= k0 && r < m) ? X[(k0 + j) * m + r] : 0.0;
  }
  // Ts (compact WY factor, Q_panel = I - V T V^T) is built column by column by thread 0 from the
  // Gram entries v_a^T v_j, which ride along in the same reduction as the update dot products.
  if (tid < BW * BW) Ts[tid / BW][tid % BW] = 0.0;
#pragma unroll
  for (int j = 0; j < BW; ++j) {
    if (j >= bw) continue;
    const int64_t diag = k0 + j;
    double s2[2] = {0.0, 0.0};
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t r = tid + (int64_t)QR_NT * i;
      if (r > diag) s2[0] += P[i][j] * P[i][j];
      if (r == diag) s2[1] = P[i][j];
    }
    block_sum<QR_NT, 2>(s2, red);
    const double sigma = s2[0], x0 = s2[1];
    const double nrm = sqrt(x0 * x0 + sigma);
    const double alpha = nrm == 0.0 ? 0.0 : (x0 >= 0.0 ? -nrm : nrm);
    const double v0 = x0 - alpha;
    const double vtv = sigma + v0 * v0;
    const double tau = vtv > 0.0 ? 2.0 / vtv : 0.0;
    // rows above the diagonal hold final R entries of this panel column
    if (blockIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int64_t r = tid + (int64_t)QR_NT * i;
        if (r >= k0 && r < diag) Rraw[r * d + diag] = P[i][j];
      }
      if (tid == 0) Rraw[diag * d + diag] = alpha;
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int64_t r = tid + (int64_t)QR_NT * i;
      if (r < diag) P[i][j] = 0.0;
      else if (r == diag) P[i][j] = v0;
    }
    // w[jj] = v_j^T (column jj) for jj > j (update), = v_jj^T v_j for jj < j (Gram column of T)
    double w[BW];
#pragma unroll
    for (int jj = 0; jj < BW; ++jj) {
      w[jj] = 0.0;
      if (jj != j) {
#pragma unroll
        for (int i = 0; i < RPT; ++i) w[jj] += P[i][j] * P[i][jj];
      }
    }
    block_sum<QR_NT, BW>(w, red);
    if (tid == 0) {
      // T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j);  T[j, j] = tau_j
      for (int a = 0; a < j; ++a) {
        double acc = 0.0;
        for (int b = a; b < j; ++b) acc += Ts[a][b] * w[b];
        Ts[a][j] = -tau * acc;
      }
      Ts[j][j] = tau;
    }
#pragma unroll
    for (int jj = 0; jj < BW; ++jj) {
      if (jj > j) {
        const double f = tau * w[jj];
#pragma unroll
        for (int i = 0; i < RPT; ++i) P[i][jj] -= f * P[i][j];
      }
    }
  }
  __syncthreads();
  // trailing columns of this workgroup
  const int64_t t0 = k0 + bw;
  const int64_t ntrail = d - t0;
  if (ntrail <= 0) return;
  const int64_t per = (ntrail + gridDim.x - 1) / gridDim.x;
  const int64_t cb = t0 + per * blockIdx.x, ce = min(d, cb + per);
  for (int64_t c = cb; c < ce; c += CB) {
    double x[RPT][CB];
#pragma unroll
    for (int q = 0; q < CB; ++q)
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int64_t r = tid + (int64_t)QR_NT * i;
        x[i][q] = (c + q < ce && r >= k0 && r < m) ? X[(c + q) * m + r] : 0.0;
      }
    double z[BW * CB];
#pragma unroll
    for (int a = 0; a < BW; ++a)
#pragma unroll
      for (int q = 0; q < CB; ++q) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) s += P[i][a] * x[i][q];
        z[a * CB + q] = s;
      }
    block_sum<QR_NT, BW * CB>(z, red);
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      double y[BW];
#pragma unroll
      for (int a = 0; a < BW; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b <= a; ++b) s += Ts[b][a] * z[b * CB + q];
        y[a] = s;
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < BW; ++a) s += P[i][a] * y[a];
        x[i][q] -= s;
      }
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      if (c + q >= ce) break;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int64_t r = tid + (int64_t)QR_NT * i;
        if (r >= k0 && r < m) {
          X[(c + q) * m + r] = x[i][q];
          if (r < t0) Rraw[r * d + (c + q)] = x[i][q];
        }
      }
    }
  }
}

// R = diag(sign(Rraw_kk)) Rraw, lower triangle zeroed; rank check on the diagonal.
__global__ void k_qr_finish(const double* __restrict__ Rraw, int64_t d, double* __restrict__ R,
                            int* __restrict__ status) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= d * d) return;
  const int64_t k = idx / d, c = idx % d;
  const double dk = Rraw[k * d + k];
  R[idx] = c < k ? 0.0 : (dk < 0.0 ? -Rraw[idx] : Rraw[idx]);
  if (c == k && !(fabs(dk) > 0.0)) atomicOr(status, 1);
}

// Relative pivot check: |R_kk| <= 8 d eps max_j |R_jj| means S A is numerically rank deficient.
__global__ __launch_bounds__(1024) void k_qr_rankcheck(const double* __restrict__ R, int64_t d,
                                                       int* __restrict__ status) {
  __shared__ double red[17 + 64];  // k_qr_rankcheck runs with 1024 threads
  double mx[1] = {0.0};
  for (int64_t k = threadIdx.x; k < d; k += 1024) mx[0] = fmax(mx[0], fabs(R[k * d + k]));
  // max-reduction via a sum of per-wave maxima is not valid; do a max butterfly explicitly
  for (int off = 32; off >= 1; off >>= 1) mx[0] = fmax(mx[0], __shfl_xor(mx[0], off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx[0];
  __syncthreads();
  double gmx = 0.0;
  for (int w = 0; w < 16; ++w) gmx = fmax(gmx, red[w]);
  const double thr = 8.0 * (double)d * 2.220446049250313e-16 * gmx;
  for (int64_t k = threadIdx.x; k < d; k += 1024)
    if (!(fabs(R[k * d + k]) > thr)) atomicOr(status, 1);
}

void householder_qr(hipStream_t st, const double* SA, int64_t m, int64_t d, int64_t lds, double* X,
                    double* R, int* status) {
  double* Rraw = X + m * d;  // caller provides m*d + d*d doubles of scratch
  hipLaunchKernelGGL(k_to_colmajor, dim3((unsigned)((m + 31) / 32), (unsigned)((d + 31) / 32)),
                     dim3(256), 0, st, SA, m, d, lds, X);
#define LSQ_QR(RPT, BW, CB)                                                                        \
  for (int64_t k0 = 0; k0 < d; k0 += BW) {                                                         \
    const int64_t ntrail = d - k0 - min((int64_t)BW, d - k0);                                      \
    int64_t g = (ntrail + CB - 1) / CB;                                                            \
    g = g < 1 ? 1 : (g > 256 ? 256 : g);                                                           \
    hipLaunchKernelGGL((k_qr_panel<RPT, BW, CB>), dim3((unsigned)g), dim3(QR_NT), 0, st, X, m, d, k0, \
                       Rraw);                                                                      \
  }
  if (m <= 512) {
    LSQ_QR(1, 8, 4)
  } else if (m <= 1024) {
    LSQ_QR(2, 8, 4)
  } else if (m <= 2048) {
    LSQ_QR(4, 8, 2)
  } else if (m <= 4096) {
    LSQ_QR(8, 8, 1)
  } else {
    LSQ_QR(16, 4, 1)
  }
#undef LSQ_QR
  hipLaunchKernelGGL(k_qr_finish, dim3((unsigned)((d * d + 255) / 256)), dim3(256), 0, st, Rraw, d, R,
                     status);
  hipLaunchKernelGGL(k_qr_rankcheck, dim3(1), dim3(1024), 0, st, R, d, status);
}

// --------------------------------------------------------------------------------------------------
// W = R^{-1} by recursive doubling of inverted diagonal blocks (the blocked form of triangular
// inversion).  R is padded to dp = 16 2^L >= d with the identity on the padding; the 16 x 16 diagonal
// blocks are inverted by substitution; then level by level two neighbouring inverted blocks of size
// h become one of size 2 h through W12 = -W11 (R12 W22), two FP64 matrix-core products per level that
// skip the zero triangles of W11 and W22.  One wavefront computes one 16 x 16 output block, reading
// its operands from L2.
// --------------------------------------------------------------------------------------------------
typedef double lsq_f_d4 __attribute__((ext_vector_type(4)));

static int64_t trinv_padded(int64_t d) {
  int64_t dp = 16;
  while (dp < d) dp *= 2;
  return dp;
}

size_t trinv_scratch_len(int64_t d) {
  const int64_t dp = trinv_padded(d);
  return (size_t)3 * dp * dp;
}

__global__ void k_trinv_pad(const double* __restrict__ R, int64_t d, int64_t dp, double* __restrict__ Rp,
                            double* __restrict__ Wp) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= dp * dp) return;
  const int64_t i = idx / dp, j = idx % dp;
  Rp[idx] = (i < d && j < d) ? R[i * d + j] : (i == j ? 1.0 : 0.0);
  Wp[idx] = 0.0;
}

// One wavefront per 16 x 16 diagonal block; lane j < 16 solves R_bb w = e_j bottom-up.
__global__ __launch_bounds__(64) void k_trinv_diag(const double* __restrict__ Rp, int64_t dp,
                                                   double* __restrict__ Wp) {
  __shared__ double Rb[16][17];
  const int64_t b0 = (int64_t)blockIdx.x * 16;
  for (int e = threadIdx.x; e < 256; e += 64) Rb[e / 16][e % 16] = Rp[(b0 + e / 16) * dp + b0 + e % 16];
  __syncthreads();
  const int j = threadIdx.x;
  if (j >= 16) return;
  double w[16];
#pragma unroll
  for (int i = 15; i >= 0; --i) {
    double s = 0.0;
#pragma unroll
    for (int k = i + 1; k < 16; ++k) s = fma(Rb[i][k], w[k], s);
    w[i] = i > j ? 0.0 : (i == j ? 1.0 / Rb[i][i] : -s / Rb[i][i]);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) Wp[(b0 + i) * dp + b0 + j] = w[i];
}

// Level with block size h: pair p joins the blocks at rows r1 = 2 p h and c2 = r1 + h.
// phase 0: T = R12 W22 -> Tp[r1.., c2..] (W22 upper: k <= j);  phase 1: W12 = -W11 T -> Wp[r1.., c2..]
// (W11 upper: k >= i).  Grid (ceil((h/16)^2 / 4), pairs), 4 wavefronts per workgroup.
__global__ __launch_bounds__(256) void k_trinv_level(const double* __restrict__ Rp, double* __restrict__ Wp,
                                                     double* __restrict__ Tp, int64_t dp, int h, int phase) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nb = h / 16;
  const int blk = blockIdx.x * 4 + wv;
  if (blk >= nb * nb) return;  // whole wavefronts
  const int bi = blk / nb, bj = blk % nb;
  const int64_t r1 = 2 * (int64_t)blockIdx.y * h, c2 = r1 + h;
  const int li = lane & 15, lk = lane >> 4;
  lsq_f_d4 acc = {0.0, 0.0, 0.0, 0.0};
  const double *A, *B;
  int k0, k1;
  if (phase == 0) {
    A = Rp + (r1 + 16 * bi + li) * dp + c2;  // R12 row, columns c2 + k
    B = Wp + c2 * dp + c2 + 16 * bj + li;    // W22 rows c2 + k, one column
    k0 = 0;
    k1 = 16 * (bj + 1);
  } else {
    A = Wp + (r1 + 16 * bi + li) * dp + r1;  // W11 row, columns r1 + k
    B = Tp + r1 * dp + c2 + 16 * bj + li;    // T rows r1 + k, one column
    k0 = 16 * bi;
    k1 = h;
  }
  for (int k = k0; k < k1; k += 16) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = A[k + 4 * u + lk];
      b[u] = B[(int64_t)(k + 4 * u + lk) * dp];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  }
  double* out = (phase == 0 ? Tp : Wp) + (r1 + 16 * bi) * dp + c2 + 16 * bj + li;
  const double sg = phase == 0 ? 1.0 : -1.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) out[(int64_t)(lk + 4 * v) * dp] = sg * acc[v];
}

// W and W^T (d x d) from the padded inverse, through a 32 x 32 LDS tile.
__global__ __launch_bounds__(256) void k_trinv_out(const double* __restrict__ Wp, int64_t dp, int64_t d,
                                                   double* __restrict__ W, double* __restrict__ WT) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k, c = c0 + tx;
    const double v = (r < d && c < d) ? Wp[r * dp + c] : 0.0;
    tile[k][tx] = v;
    if (r < d && c < d) W[r * d + c] = v;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t c = c0 + k, r = r0 + tx;
    if (r < d && c < d) WT[c * d + r] = tile[tx][k];
  }
}

__global__ void k_trinv_copy(const double* __restrict__ Wp, int64_t dq, int64_t dp, double* __restrict__ W) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= dp * dp) return;
  W[idx] = Wp[(idx / dp) * dq + idx % dp];
}

static void trinv_levels(hipStream_t st, double* Rp, double* Wp, double* Tp, int64_t dp) {
  hipLaunchKernelGGL(k_trinv_diag, dim3((unsigned)(dp / 16)), dim3(64), 0, st, Rp, dp, Wp);
  for (int64_t h = 16; h < dp; h *= 2) {
    const int64_t nb = h / 16;
    dim3 g((unsigned)((nb * nb + 3) / 4), (unsigned)(dp / (2 * h)));
    hipLaunchKernelGGL(k_trinv_level, g, dim3(256), 0, st, Rp, Wp, Tp, dp, (int)h, 0);
    hipLaunchKernelGGL(k_trinv_level, g, dim3(256), 0, st, Rp, Wp, Tp, dp, (int)h, 1);
  }
}

void tri_inverse_padded(hipStream_t st, const double* R, int64_t n, double* W, double* scratch) {
  const int64_t dq = trinv_padded(n);
  double* Rp = scratch;
  double* Wp = Rp + dq * dq;
  double* Tp = Wp + dq * dq;
  hipLaunchKernelGGL(k_trinv_pad, dim3((unsigned)((dq * dq + 255) / 256)), dim3(256), 0, st, R, n, dq, Rp, Wp);
  trinv_levels(st, Rp, Wp, Tp, dq);
  hipLaunchKernelGGL(k_trinv_copy, dim3((unsigned)((n * n + 255) / 256)), dim3(256), 0, st, Wp, dq, n, W);
}

// flag = 1 when some entry of X (m x d, row stride ld) is NaN or infinite.  Every writer stores the same
// value, so the unordered stores need no atomics.
__global__ __launch_bounds__(256) void k_nonfinite_scan(const double* __restrict__ X, int64_t m, int64_t d,
                                                        int64_t ld, int* __restrict__ flag) {
  bool bad = false;
  const int64_t total = m * d, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride)
    bad |= !isfinite(X[(i / d) * ld + i % d]);
  if (__ballot(bad) != 0ull && (threadIdx.x & 63) == 0) *flag = 1;
}

void nonfinite_scan(hipStream_t st, const double* X, int64_t m, int64_t d, int64_t ld, int* flag) {
  const int64_t blocks = std::min<int64_t>((m * d + 255) / 256, 2048);
  hipLaunchKernelGGL(k_nonfinite_scan, dim3((unsigned)blocks), dim3(256), 0, st, X, m, d, ld, flag);
}

// out[0] = max_i |R_ii| / min_i |R_ii| of the d x d row-major R (one workgroup).  A lower estimate of
// kappa(R) = kappa(S A): for a geometric spectrum and random right singular vectors it runs about 20-30
// times below it.
__global__ __launch_bounds__(1024) void k_diag_spread(const double* __restrict__ R, int64_t d, double* __restrict__ out) {
  __shared__ double smx[16], smn[16];
  double mx = 0.0, mn = INFINITY;
  for (int64_t i = threadIdx.x; i < d; i += 1024) {
    const double a = fabs(R[i * d + i]);
    mx = fmax(mx, a);
    mn = fmin(mn, a);
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
    for (int w = 1; w < 16; ++w) {
      mx = fmax(mx, smx[w]);
      mn = fmin(mn, smn[w]);
    }
    out[0] = mn > 0.0 ? mx / mn : INFINITY;
  }
}

void diag_spread(hipStream_t st, const double* R, int64_t d, double* out) {
  hipLaunchKernelGGL(k_diag_spread, dim3(1), dim3(1024), 0, st, R, d, out);
}

void qr_rank_check(hipStream_t st, const double* R, int64_t d, int* status) {
  hipLaunchKernelGGL(k_qr_rankcheck, dim3(1), dim3(1024), 0, st, R, d, status);
}

void tri_inverse(hipStream_t st, const double* R, int64_t d, double* W, double* WT, double* scratch) {
  const int64_t dp = trinv_padded(d);
  double* Rp = scratch;
  double* Wp = Rp + dp * dp;
  double* Tp = Wp + dp * dp;
  hipLaunchKernelGGL(k_trinv_pad, dim3((unsigned)((dp * dp + 255) / 256)), dim3(256), 0, st, R, d, dp, Rp, Wp);
  trinv_levels(st, Rp, Wp, Tp, dp);
  dim3 go((unsigned)((d + 31) / 32), (unsigned)((d + 31) / 32));
  hipLaunchKernelGGL(k_trinv_out, go, dim3(256), 0, st, Wp, dp, d, W, WT);
}

}  // namespace lsq
