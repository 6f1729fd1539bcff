// Gaussian sketch S A with S_ij = g(i, j) / sqrt(m), g standard normal from the counter-based
// specification (Section 2: i.i.d. N(0, 1/m) entries).  S is never stored: every workgroup generates
// its block of S in registers from Philox words and multiplies it with a tile of A on the matrix cores.
// The reduction over the long dimension n is split across workgroups (partials), then summed in a fixed
// order.
#include "internal.h"

namespace lsq {

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
// FP64 form on the matrix cores (v_mfma_f64_16x16x4f64).  Workgroup: 8 wavefronts, 128 rows of S A (16
// per wavefront) x 256 columns (16 blocks of 16), over a range of rows of A split across workgroups.
// Per step of 32 rows of A (columns kb .. kb + 31 of S): the 32 x 256 tile of A is staged in LDS (double
// buffered; whole FP64 tiles are loaded straight into the other buffer while this step computes, other
// tiles through registers after this step's MFMAs have issued) and shared by all wavefronts.  Lane l (row il = l % 16
// of its wavefront's S rows, group h = l / 16) evaluates the one Philox block of columns kb + 8 h .. + 7 of
// row il and its four Box-Muller pairs (FP64): e[p] = S[il][kb + 8 h + p].  Two 4 x 4 transposes across
// the four 16-lane rows of the wavefront (two rounds of row swaps each), of e[0..3] and of e[4..7], leave
// in lane (il, kk) the A operands of the eight substeps: S[il][kb + 8 q + kk] (substep 2 q) and
// S[il][kb + 8 q + 4 + kk] (substep 2 q + 1).  B operand lane l = A[kb + 4 s + l / 16][l % 16]; result
// lane l, register v = (row l / 16 + 4 v, column l % 16).  The next step's normals are formed while this
// step's MFMAs issue.
// --------------------------------------------------------------------------------------------------
typedef double g_d4 __attribute__((ext_vector_type(4)));
constexpr int GM_WAVES = 8, GM_ROWS = GM_WAVES * 16, GM_BLK = 16, GM_COLS = GM_BLK * 16, GM_K = 32;
constexpr int GM_LDS_STRIDE = GM_COLS + 16;  // 272 doubles: the 4 k-rows of one read fall in different banks
constexpr int GM_LROWS = GM_K / GM_WAVES;  // rows of the tile per loading thread (4)

// Exchange of one double between the 16-lane rows of a wavefront: rows (0, 1) and (2, 3) swap
// (x's odd rows with y's even rows) for XOR = 1; the wave halves swap (x's upper half with y's lower
// half) for XOR = 2.
template <int XOR>
__device__ __forceinline__ void row_swap(double& x, double& y) {
  const uint32_t xl = (uint32_t)__double2loint(x), xh = (uint32_t)__double2hiint(x);
  const uint32_t yl = (uint32_t)__double2loint(y), yh = (uint32_t)__double2hiint(y);
  if constexpr (XOR == 1) {
    const auto l = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    x = __hiloint2double((int)h[0], (int)l[0]);
    y = __hiloint2double((int)h[1], (int)l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
    x = __hiloint2double((int)h[0], (int)l[0]);
    y = __hiloint2double((int)h[1], (int)l[1]);
  }
}

// 4 x 4 transpose over (16-lane row h, element j) of e[0..3]: afterwards e[j] holds row j's former e[h].
// Swaps the low bits of row and element, then the high bits.  All 64 lanes must be active.
__device__ __forceinline__ void rows_transpose4(double& e0, double& e1, double& e2, double& e3) {
  row_swap<1>(e0, e1);
  row_swap<1>(e2, e3);
  row_swap<2>(e0, e2);
  row_swap<2>(e1, e3);
}

// The eight A operands of one step for lane (il, kk): g[s] = S[il][kb + 4 s + kk], s < 8 (see above).
// Every lane evaluates its block (rows past m take zeros afterwards), so the code has no branches and
// can be interleaved with the matrix-core instructions.
__device__ __forceinline__ void gauss_step_operands(uint64_t seed, uint64_t t, int64_t irow, bool iok, int64_t kb,
                                                    int h, double (&g)[8]) {
  double e[8];
  const u64x4 w = philox4x64_10((uint64_t)((kb >> 3) + h), TAG_GAUSS, t, (uint64_t)irow, seed, 0);
  box_muller_pair_f64(w.x, e[0], e[1]);
  box_muller_pair_f64(w.y, e[2], e[3]);
  box_muller_pair_f64(w.z, e[4], e[5]);
  box_muller_pair_f64(w.w, e[6], e[7]);
#pragma unroll
  for (int p = 0; p < 8; ++p) e[p] = iok ? e[p] : 0.0;
  rows_transpose4(e[0], e[1], e[2], e[3]);  // e[q] = S[il][kb + 8 q + kk]
  rows_transpose4(e[4], e[5], e[6], e[7]);  // e[4 + q] = S[il][kb + 8 q + 4 + kk]
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    g[2 * q] = e[q];
    g[2 * q + 1] = e[4 + q];
  }
}

// 16 bytes per lane from global memory straight into LDS: lane l's bytes land at dst + 16 l (dst must be
// the same for the whole wavefront).
__device__ __forceinline__ void lds_load16(const void* src, double* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// Rows kb + lr + 8 q (q < 4), columns c0 + lc .. + 3 of A into v, zero outside rows [k0, k1) and columns
// [0, d).  VEC: 16-byte rows (A aligned, lda and d multiples of 4 elements; FP64 also 2): vector loads.
// Out-of-range entries read a clamped in-range address and are replaced by zero, so there are no
// branches.  Ordinary (cached) loads: the tile is read again by the workgroups of the other rows of S.
template <typename TA, bool VEC>
__device__ __forceinline__ void gm_load_tile(const TA* __restrict__ A, int64_t kb, int64_t k0, int64_t k1, int64_t c0,
                                             int64_t d, int64_t lda, int lr, int lc, double (&v)[GM_LROWS][4]) {
  const int64_t col = c0 + lc;
#pragma unroll
  for (int q = 0; q < GM_LROWS; ++q) {
    const int64_t row = kb + lr + 8 * q;
    const bool rok = row < k1;
    const TA* base = A + (rok ? row : k0) * lda;
    if constexpr (VEC) {
      const bool ok = rok && col < d;
      const TA* pv = base + (col < d ? col : 0);
      if constexpr (sizeof(TA) == 4) {
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 x = *(const f4*)pv;
#pragma unroll
        for (int u = 0; u < 4; ++u) v[q][u] = ok ? (double)x[u] : 0.0;
      } else {
        typedef double d2 __attribute__((ext_vector_type(2)));
        const d2 x0 = *(const d2*)pv, x1 = *(const d2*)(pv + 2);
        v[q][0] = ok ? x0[0] : 0.0;
        v[q][1] = ok ? x0[1] : 0.0;
        v[q][2] = ok ? x1[0] : 0.0;
        v[q][3] = ok ? x1[1] : 0.0;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t cu = col + u;
        const bool ok = rok && cu < d;
        v[q][u] = ok ? (double)base[cu < d ? cu : d - 1] : 0.0;
      }
    }
  }
}

template <typename TA, bool VEC>
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
  const int64_t irow = i0 + wv * 16 + il;  // row of S whose entries this lane generates
  const bool iok = irow < m;
  g_d4 acc[GM_BLK];
#pragma unroll
  for (int b = 0; b < GM_BLK; ++b) acc[b] = (g_d4){0.0, 0.0, 0.0, 0.0};
  // tile loader: thread -> rows tid / 64 + 8 q (q < 4), 4 consecutive columns (64 x 4 = 256)
  const int lr = tid >> 6, lc = (tid & 63) * 4;
  auto store_tile = [&](int buf, const double (&v)[GM_LROWS][4]) {
#pragma unroll
    for (int q = 0; q < GM_LROWS; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) As[buf][(lr + 8 * q) * GM_LDS_STRIDE + lc + u] = v[q][u];
  };
  // FP64 rows of 16 bytes and a column block inside [0, d): whole tiles go from global memory straight
  // into LDS (global_load_lds, 16 bytes per lane: one instruction fills half a tile row; wavefront w fills
  // rows w, w + 8, w + 16, w + 24), issued at the start of the step before it so that the loads fly
  // under the MFMAs and occupy no registers
  const bool direct_cols = sizeof(TA) == 8 && VEC && c0 + GM_COLS <= d;
  auto direct_tile = [&](int buf, int64_t kb) {
#pragma unroll
    for (int q = 0; q < GM_LROWS; ++q) {
      const int r = wv + 8 * q;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh)
        lds_load16(A + (kb + r) * lda + c0 + 128 * hh + 2 * lane, &As[buf][r * GM_LDS_STRIDE + 128 * hh]);
    }
  };
  if (k0 < k1) {
    {
      double nv[GM_LROWS][4];
      gm_load_tile<TA, VEC>(A, k0, k0, k1, c0, d, lda, lr, lc, nv);
      store_tile(0, nv);
    }
    double g[8];
    gauss_step_operands(seed, t, irow, iok, k0, kk, g);
    __syncthreads();
    int buf = 0;
    for (int64_t kb = k0; kb < k1; kb += GM_K) {
      const bool more = kb + GM_K < k1;
      const bool direct = direct_cols && kb + 2 * GM_K <= k1;  // the next tile is whole (uniform)
      if (direct) direct_tile(buf ^ 1, kb + GM_K);
      // the next step's operands (past the range at the last step: computed and dropped), interleaved
      // with this step's MFMAs: per MFMA about five VALU instructions of the normals, and the LDS
      // reads of the B operands ahead of their MFMAs
      double gn[8];
      gauss_step_operands(seed, t, irow, iok, kb + GM_K, kk, gn);
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const double* T = &As[buf][(4 * s + kk) * GM_LDS_STRIDE + il];
#pragma unroll
        for (int b = 0; b < GM_BLK; ++b) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[s], T[b * 16], acc[b], 0, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < 8 * GM_BLK; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // one LDS read
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);  // five VALU
      }
#pragma unroll
      for (int s = 0; s < 8; ++s) g[s] = gn[s];
      if (direct) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's LDS loads have landed
      } else if (more) {
        // the next tile into the other buffer (its last readers passed the previous barrier); the other
        // wavefront of the SIMD keeps the matrix core busy while these loads are in flight
        double nv[GM_LROWS][4];
        gm_load_tile<TA, VEC>(A, kb + GM_K, k0, k1, c0, d, lda, lr, lc, nv);
        store_tile(buf ^ 1, nv);
      }
      __syncthreads();
      buf ^= 1;
    }
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

int g_gauss_wgs = 1024;

static int64_t gauss_nks(int64_t m, int64_t d, int64_t n) {
  // GM_ROWS x GM_COLS and GB_ROWS x GB_COLS tiles are the same size; about g_gauss_wgs workgroups in all
  const int64_t tiles = ((m + GM_ROWS - 1) / GM_ROWS) * ((d + GM_COLS - 1) / GM_COLS);
  int64_t nks = (g_gauss_wgs + tiles - 1) / tiles;
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
  kchunk = (kchunk + GM_K - 1) / GM_K * GM_K;  // multiple of 32: whole steps, Philox blocks never straddle chunks
  const bool v16 = ((uintptr_t)A % 16 == 0) && lda % 4 == 0 && d % 4 == 0;
#define LSQ_GM(TA, V)                                                                                       \
  hipLaunchKernelGGL((k_gauss_mfma<TA, V>), g, dim3(GM_WAVES * 64), 0, st, seed, t, (const TA*)A, n, d, lda, m, \
                     kchunk, partials)
  if (a_f32) {
    if (v16) LSQ_GM(float, true);
    else LSQ_GM(float, false);
  } else {
    if (v16) LSQ_GM(double, true);
    else LSQ_GM(double, false);
  }
#undef LSQ_GM
  hipLaunchKernelGGL(k_gauss_reduce, dim3((unsigned)((m * d + 255) / 256)), dim3(256), 0, st, partials,
                     nks, m, d, 1.0 / sqrt((double)m), SA, ldsa);
}

}  // namespace lsq
