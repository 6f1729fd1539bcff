// Gaussian sketch S A with S_ij = g(i, j) / sqrt(m), g standard normal from the counter-based
// specification (Section 2: i.i.d. N(0, 1/m) entries).  S is never stored: every workgroup generates
// its block of S in LDS from Philox words and multiplies it with a tile of A.  The reduction over the
// long dimension n is split across workgroups (partials), then summed in a fixed order.
#include "internal.h"

namespace lsq {

constexpr int GT_M = 64, GT_D = 64, GT_K = 32;

template <typename TA>
__global__ __launch_bounds__(256) void k_gauss_tile(uint64_t seed, uint64_t t, const TA* __restrict__ A,
                                                    int64_t n, int64_t d, int64_t lda, int64_t m,
                                                    int64_t kchunk, double* __restrict__ part) {
  __shared__ double Gs[GT_M][GT_K + 1];
  __shared__ double As[GT_K][GT_D + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * GT_M, c0 = (int64_t)blockIdx.y * GT_D;
  const int64_t k0 = (int64_t)blockIdx.z * kchunk, k1 = min(n, k0 + kchunk);
  double acc[4][4] = {};
  for (int64_t kb = k0; kb < k1; kb += GT_K) {
    __syncthreads();
    {
      // 64 rows x 32 columns of S: one Philox block (8 normals) per thread
      const int gi = tid >> 2, gq = (tid & 3) * 8;
      const int64_t i = i0 + gi, jb = kb + gq;
      const u64x4 w = philox4x64_10((uint64_t)(jb >> 3), TAG_GAUSS, t, (uint64_t)i, seed, 0);
      const uint64_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t j = jb + q;
        Gs[gi][gq + q] = (i < m && j < k1) ? (double)box_muller_f32(ws[q >> 1], q & 1) : 0.0;
      }
    }
    for (int idx = tid; idx < GT_K * GT_D; idx += 256) {
      const int kk = idx / GT_D, cc = idx % GT_D;
      const int64_t j = kb + kk, col = c0 + cc;
      As[kk][cc] = (j < k1 && col < d) ? (double)A[j * lda + col] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < GT_K; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = Gs[ty * 4 + u][kk];
        b[u] = As[kk][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
  }
  double* out = part + (int64_t)blockIdx.z * m * d;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + ty * 4 + u, col = c0 + tx * 4 + v;
      if (i < m && col < d) out[i * d + col] = acc[u][v];
    }
}

__global__ void k_gauss_reduce(const double* __restrict__ part, int64_t nks, int64_t m, int64_t d,
                               double scale, double* __restrict__ SA, int64_t ldsa) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * d) return;
  double s = 0.0;
  for (int64_t k = 0; k < nks; ++k) s += part[k * m * d + idx];
  const int64_t i = idx / d, c = idx % d;
  SA[i * ldsa + c] = s * scale;
}

// --------------------------------------------------------------------------------------------------
// Matrix-core version (v_mfma_f64_16x16x4f64).  Workgroup: 8 wavefronts, 128 rows of S A (16 per
// wavefront) x 256 columns (16 blocks of 16), over a range of rows of A split across workgroups.
// Per step of 8 rows of A: the 8 x 256 tile of A is staged in LDS (shared by all wavefronts) and
// each lane (row i = l % 16 of its wavefront, k offset kk = l / 16) evaluates one Philox block
// (8 consecutive entries of row i of S) and keeps the two entries it feeds to the matrix cores,
// j0 + kk and j0 + kk + 4.  Operand layouts: A operand lane l = S[l % 16][kk], B operand lane l =
// A[kk][l % 16]; result lane l, register v = (row l / 16 + 4 v, column l % 16).
// --------------------------------------------------------------------------------------------------
typedef double g_d4 __attribute__((ext_vector_type(4)));
constexpr int GM_WAVES = 8, GM_ROWS = GM_WAVES * 16, GM_BLK = 16, GM_COLS = GM_BLK * 16, GM_K = 8;
constexpr int GM_LDS_STRIDE = GM_COLS + 16;  // 272 doubles: the 4 k-rows of one read hit different banks

template <typename TA>
__global__ __launch_bounds__(GM_WAVES * 64) void k_gauss_mfma(uint64_t seed, uint64_t t,
                                                             const TA* __restrict__ A, int64_t n,
                                                             int64_t d, int64_t lda, int64_t m,
                                                             int64_t kchunk, double* __restrict__ part) {
  __shared__ double As[2][GM_K * GM_LDS_STRIDE];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int il = lane & 15, kk = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * GM_ROWS;
  const int64_t c0 = (int64_t)blockIdx.y * GM_COLS;
  const int64_t k0 = (int64_t)blockIdx.z * kchunk, k1 = min(n, k0 + kchunk);
  const int64_t irow = i0 + wv * 16 + il;       // row of S this lane generates
  const bool iok = irow < m;
  g_d4 acc[GM_BLK];
#pragma unroll
  for (int b = 0; b < GM_BLK; ++b) acc[b] = (g_d4){0.0, 0.0, 0.0, 0.0};
  // tile loader: thread -> (row tid / 64, 4 consecutive columns)
  const int lr = tid >> 6, lc = (tid & 63) * 4;
  auto load_tile = [&](int64_t kb, double (&v)[4]) {
    const int64_t row = kb + lr;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t col = c0 + lc + u;
      v[u] = (row < k1 && col < d) ? (double)A[row * lda + col] : 0.0;
    }
  };
  double nv[4];
  if (k0 < k1) load_tile(k0, nv);
  int buf = 0;
  for (int64_t kb = k0; kb < k1; kb += GM_K) {
#pragma unroll
    for (int u = 0; u < 4; ++u) As[buf][lr * GM_LDS_STRIDE + lc + u] = nv[u];
    __syncthreads();
    if (kb + GM_K < k1) load_tile(kb + GM_K, nv);  // next tile in flight during this step
    // the two entries of row irow of S used by this lane in this step
    double g0 = 0.0, g1 = 0.0;
    if (iok) {
      const u64x4 w = philox4x64_10((uint64_t)(kb >> 3), TAG_GAUSS, t, (uint64_t)irow, seed, 0);
      const uint64_t w0 = (kk >> 1) == 0 ? w.x : w.y;          // word of entry kk
      const uint64_t w1 = (kk >> 1) == 0 ? w.z : w.w;          // word of entry kk + 4
      const double sc = 1.0;
      g0 = (kb + kk < k1) ? sc * (double)box_muller_f32(w0, kk & 1) : 0.0;
      g1 = (kb + kk + 4 < k1) ? sc * (double)box_muller_f32(w1, kk & 1) : 0.0;
    }
    const double* T0 = &As[buf][kk * GM_LDS_STRIDE];
    const double* T1 = &As[buf][(kk + 4) * GM_LDS_STRIDE];
#pragma unroll
    for (int b = 0; b < GM_BLK; ++b) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(g0, T0[b * 16 + il], acc[b], 0, 0, 0);
#pragma unroll
    for (int b = 0; b < GM_BLK; ++b) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(g1, T1[b * 16 + il], acc[b], 0, 0, 0);
    buf ^= 1;
  }
  double* out = part + (int64_t)blockIdx.z * m * d;
#pragma unroll
  for (int b = 0; b < GM_BLK; ++b) {
    const int64_t col = c0 + b * 16 + il;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + wv * 16 + kk + 4 * v;
      if (i < m && col < d) out[i * d + col] = acc[b][v];
    }
  }
}

static int64_t gauss_nks(int64_t m, int64_t d, int64_t n) {
  const int64_t tiles = ((m + GM_ROWS - 1) / GM_ROWS) * ((d + GM_COLS - 1) / GM_COLS);
  int64_t nks = (1024 + tiles - 1) / tiles;
  const int64_t maxks = (n + 255) / 256;
  if (nks > maxks) nks = maxks;
  if (nks > 512) nks = 512;
  return nks < 1 ? 1 : nks;
}

size_t gauss_partial_bytes(int64_t m, int64_t d, int64_t n, int bf16) {
  (void)bf16;
  return (size_t)gauss_nks(m, d, n) * m * d * sizeof(double);
}

void gauss_apply(hipStream_t st, uint64_t seed, uint64_t t, const void* A, int a_f32, int64_t n,
                 int64_t d, int64_t lda, int64_t m, int bf16, double* partials, double* SA,
                 int64_t ldsa) {
  (void)bf16;
  const int64_t nks = gauss_nks(m, d, n);
  int64_t kchunk = (n + nks - 1) / nks;
  kchunk = (kchunk + GM_K - 1) / GM_K * GM_K;  // multiple of 8: Philox blocks never straddle chunks
  dim3 g((unsigned)((m + GM_ROWS - 1) / GM_ROWS), (unsigned)((d + GM_COLS - 1) / GM_COLS), (unsigned)nks);
  if (a_f32)
    hipLaunchKernelGGL(k_gauss_mfma<float>, g, dim3(GM_WAVES * 64), 0, st, seed, t, (const float*)A, n, d,
                       lda, m, kchunk, partials);
  else
    hipLaunchKernelGGL(k_gauss_mfma<double>, g, dim3(GM_WAVES * 64), 0, st, seed, t, (const double*)A, n,
                       d, lda, m, kchunk, partials);
  hipLaunchKernelGGL(k_gauss_reduce, dim3((unsigned)((m * d + 255) / 256)), dim3(256), 0, st, partials,
                     nks, m, d, 1.0 / sqrt((double)m), SA, ldsa);
}

}  // namespace lsq
