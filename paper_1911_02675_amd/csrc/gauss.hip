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

// --------------------------------------------------------------------------------------------------
// Precision form on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16).  S is rounded to BF16 (round
// to nearest even from the single-precision Box-Muller value; still a Gaussian-like embedding) and A
// is split into three BF16 terms A = A1 + A2 + A3 (A1 = bf16(a), A2 = bf16(a - A1),
// A3 = bf16(a - A1 - A2); relative error below 2^-26 after the FP32 rounding of a), so each product
// S A_k is exact in FP32 and S A is summed from the three.  FP32 accumulation chains are limited to
// GB_FOLD * 32 rows of A and then added into FP64 registers, so the accumulation error does not grow
// with n.  Workgroup: 8 wavefronts, 128 rows of S A (16 per wavefront) x 256 columns (16 tiles),
// per step 32 rows of A: the three BF16 planes of the 32 x 256 A tile are staged in LDS, column-major
// with 8 consecutive k per 16-byte lane read.  Operand layouts: A operand lane l = S[l % 16][8 (l / 16)
// + i] (exactly the 8 entries of one Philox block), B operand lane l = A_k[8 (l / 16) + i][l % 16],
// result lane l register v = (row 4 (l / 16) + v, column l % 16).
// --------------------------------------------------------------------------------------------------
typedef __bf16 g_bf8 __attribute__((ext_vector_type(8)));

// The pair of normals of one 64-bit word (cos branch, sin branch; same u1, u2 as box_muller_f32)
// from the hardware transcendentals: v_log_f32 (log2), v_sqrt_f32, and v_cos_f32 / v_sin_f32, which
// take the angle in revolutions, i.e. exactly 2 pi u2.  A few ulp of single precision, far below
// the BF16 rounding that follows.
__device__ __forceinline__ void box_muller_pair_hw(uint64_t w, float& c, float& s) {
  const uint32_t a = (uint32_t)w, b = (uint32_t)(w >> 32);
  const float u1 = ((float)a + 1.0f) * 2.3283064365386963e-10f;  // (0, 1]
  const float u2 = (float)b * 2.3283064365386963e-10f;            // [0, 1)
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));  // -2 ln 2
  c = r * __builtin_amdgcn_cosf(u2);
  s = r * __builtin_amdgcn_sinf(u2);
}
typedef float g_f4 __attribute__((ext_vector_type(4)));
constexpr int GB_WAVES = 8, GB_ROWS = GB_WAVES * 16, GB_TILES = 16, GB_COLS = GB_TILES * 16, GB_K = 32;
constexpr int GB_FOLD = 8;      // K-steps (of 32 rows) per FP32 accumulation chain
static_assert(GB_ROWS == GM_ROWS && GB_COLS == GM_COLS, "both Gaussian kernels share the split-K plan");
constexpr int GB_CSTRIDE = 40;  // BF16 entries per column in an LDS plane (32 k + 8 padding)

template <typename TA, bool V4>
__global__ __launch_bounds__(GB_WAVES * 64) void k_gauss_bf16(uint64_t seed, uint64_t t,
                                                             const TA* __restrict__ A, int64_t n,
                                                             int64_t d, int64_t lda, int64_t m,
                                                             int64_t kchunk, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) __bf16 Bs[3][GB_COLS * GB_CSTRIDE];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * GB_ROWS;
  const int64_t c0 = (int64_t)blockIdx.y * GB_COLS;
  const int64_t k0 = (int64_t)blockIdx.z * kchunk, k1 = min(n, k0 + kchunk);
  const int64_t irow = i0 + wv * 16 + li;  // row of S whose entries this lane generates
  const bool iok = irow < m;
  g_f4 acc[GB_TILES];
  double acc64[GB_TILES][4];
#pragma unroll
  for (int b = 0; b < GB_TILES; ++b) {
    acc[b] = (g_f4){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int v = 0; v < 4; ++v) acc64[b][v] = 0.0;
  }
  // tile loader: 4 consecutive columns, rows {2 rp, 2 rp + 1, 2 rp + 16, 2 rp + 17}; the next tile
  // is loaded into registers while the current one is multiplied
  const int c4 = tid & 63, rp = tid >> 6;
  const int64_t colb = c0 + 4 * c4;
  float v[4][4];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = kb + 2 * rp + (q & 1) + 16 * (q >> 1);
      if (V4) {
        // 16-byte rows (lda % 4 == 0, d % 4 == 0, A aligned): one vector load or none
        const bool ok = row < k1 && colb < d;
        const float4 f = ok ? *(const float4*)((const float*)A + row * lda + colb) : make_float4(0.f, 0.f, 0.f, 0.f);
        v[q][0] = f.x;
        v[q][1] = f.y;
        v[q][2] = f.z;
        v[q][3] = f.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t col = colb + u;
          v[q][u] = (row < k1 && col < d) ? (float)A[row * lda + col] : 0.0f;
        }
      }
    }
  };
  if (k0 < k1) load(k0);
  int step = 0;
  for (int64_t kb = k0; kb < k1; kb += GB_K) {
    // the 8 entries S[irow][kb + 8 lg + q], q = 0..7: one Philox block (independent of the tile)
    g_bf8 ga;
    {
      const u64x4 w = philox4x64_10((uint64_t)((kb + 8 * lg) >> 3), TAG_GAUSS, t, (uint64_t)irow, seed, 0);
      const uint64_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float c, sn;
        box_muller_pair_hw(ws[q], c, sn);
        ga[2 * q] = (__bf16)(iok ? c : 0.0f);
        ga[2 * q + 1] = (__bf16)(iok ? sn : 0.0f);
      }
    }
    __syncthreads();  // the previous step's operands have been read
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int col = 4 * c4 + u;
#pragma unroll
      for (int pr = 0; pr < 2; ++pr) {
        const float a0 = v[2 * pr][u], a1 = v[2 * pr + 1][u];
        const __bf16 h0 = (__bf16)a0, h1 = (__bf16)a1;
        const float r0 = a0 - (float)h0, r1 = a1 - (float)h1;
        const __bf16 g0 = (__bf16)r0, g1 = (__bf16)r1;
        const float s0 = r0 - (float)g0, s1 = r1 - (float)g1;
        const __bf16 e0 = (__bf16)s0, e1 = (__bf16)s1;
        const int k = 2 * rp + 16 * pr;  // even: the pair (k, k + 1) is one 32-bit LDS word
        uint32_t* base = (uint32_t*)&Bs[0][col * GB_CSTRIDE + k];
        base[0] = (uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16);
        base[GB_COLS * GB_CSTRIDE / 2] =
            (uint32_t)__builtin_bit_cast(uint16_t, g0) | ((uint32_t)__builtin_bit_cast(uint16_t, g1) << 16);
        base[GB_COLS * GB_CSTRIDE] =
            (uint32_t)__builtin_bit_cast(uint16_t, e0) | ((uint32_t)__builtin_bit_cast(uint16_t, e1) << 16);
      }
    }
    __syncthreads();
    if (kb + GB_K < k1) load(kb + GB_K);
#pragma unroll
    for (int b = 0; b < GB_TILES; ++b) {
      const int col = b * 16 + li;
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const g_bf8 bv = *(const g_bf8*)&Bs[p][col * GB_CSTRIDE + 8 * lg];
        acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ga, bv, acc[b], 0, 0, 0);
      }
    }
    if (++step == GB_FOLD) {
      step = 0;
#pragma unroll
      for (int b = 0; b < GB_TILES; ++b) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc64[b][q] += (double)acc[b][q];
        acc[b] = (g_f4){0.0f, 0.0f, 0.0f, 0.0f};
      }
    }
  }
  double* out = part + (int64_t)blockIdx.z * m * d;
#pragma unroll
  for (int b = 0; b < GB_TILES; ++b) {
    const int64_t col = c0 + b * 16 + li;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = i0 + wv * 16 + 4 * lg + q;
      if (i < m && col < d) out[i * d + col] = acc64[b][q] + (double)acc[b][q];
    }
  }
}

static int64_t gauss_nks(int64_t m, int64_t d, int64_t n) {
  // GM_ROWS x GM_COLS and GB_ROWS x GB_COLS tiles are the same size
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
  const int64_t nks = gauss_nks(m, d, n);
  int64_t kchunk = (n + nks - 1) / nks;
  dim3 g((unsigned)((m + GM_ROWS - 1) / GM_ROWS), (unsigned)((d + GM_COLS - 1) / GM_COLS), (unsigned)nks);
  if (bf16) {
    kchunk = (kchunk + GB_K - 1) / GB_K * GB_K;  // whole steps of 32 rows per chunk
    const bool v4 = a_f32 && ((uintptr_t)A % 16 == 0) && lda % 4 == 0 && d % 4 == 0;
    if (v4)
      hipLaunchKernelGGL((k_gauss_bf16<float, true>), g, dim3(GB_WAVES * 64), 0, st, seed, t, (const float*)A,
                         n, d, lda, m, kchunk, partials);
    else if (a_f32)
      hipLaunchKernelGGL((k_gauss_bf16<float, false>), g, dim3(GB_WAVES * 64), 0, st, seed, t,
                         (const float*)A, n, d, lda, m, kchunk, partials);
    else
      hipLaunchKernelGGL((k_gauss_bf16<double, false>), g, dim3(GB_WAVES * 64), 0, st, seed, t,
                         (const double*)A, n, d, lda, m, kchunk, partials);
    hipLaunchKernelGGL(k_gauss_reduce, dim3((unsigned)((m * d + 255) / 256)), dim3(256), 0, st, partials,
                       nks, m, d, 1.0 / sqrt((double)m), SA, ldsa);
    return;
  }
  kchunk = (kchunk + GM_K - 1) / GM_K * GM_K;  // multiple of 8: Philox blocks never straddle chunks
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
