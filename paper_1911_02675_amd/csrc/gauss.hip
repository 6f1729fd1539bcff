// Gaussian sketch S A with S_ij = g(i, j) / sqrt(m), g standard normal from the counter-based
// specification (Section 2: i.i.d. N(0, 1/m) entries).  S is never stored: every workgroup generates
// its block of S in registers from Philox words and multiplies it with a tile of A on the matrix cores.
// The reduction over the long dimension n is split across workgroups (partials), then summed in a fixed
// order.  The BF16 precision form at d >= 384 first writes the three BF16 terms of a chunk of rows of A
// in the matrix cores' fragment order (k_gauss_split3), then multiplies them (k_gauss_bf16_planes).
#include <type_traits>

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

// --------------------------------------------------------------------------------------------------
// Precision form for wide A (d >= g_gauss_planes_min_d).  The three BF16 terms of A are formed once per
// chunk of rows by k_gauss_split3 and stored in the order the matrix cores read them: unit (k-block kb
// of 32 rows, column group g of 512 columns, term p) is 32 KB, 32 column tiles of 1 KB, lane l of tile
// ct holding rows 8 (l / 16) .. + 7 of column 512 g + 16 ct + l % 16 (zero past the chunk and past d).
// The product kernel moves whole units into LDS with global-to-LDS loads (no registers, no VALU), and
// every normal meets 512 columns (three MFMAs per 16 of them), twice the reach of k_gauss_bf16: the
// Philox and Box-Muller work per MFMA halves and the split leaves the product loop altogether.
// Workgroup: 8 wavefronts (two per SIMD), 64 rows of S A x 512 columns; wavefront w keeps the 4 x 4
// tiles of columns 64 w .. 64 w + 63 (row tile r, column tile c: acc[r][c]).  The four fragments of S
// a step needs are evaluated by four wavefronts, one Philox block per lane: wavefront w (row tile w % 4)
// forms the fragments of the steps of parity w / 4, during the step two before, and passes them on
// through LDS; on each SIMD one wavefront forms normals while both issue MFMAs.  A ring of 4 units in
// LDS keeps three in flight.  FP32 chains of GP_FOLD steps are added into FP32 sums, and those into the
// FP64 partial in global memory every GP_FLUSH steps and at the end.
// --------------------------------------------------------------------------------------------------
constexpr int GP_WAVES = 8, GP_MT = 64, GP_NT = 512, GP_WCT = 4, GP_UNIT = 32768, GP_RING = 4;
constexpr int GP_DMA = GP_UNIT / (GP_WAVES * 64 * 16);  // 16-byte global-to-LDS loads per thread per unit
constexpr int GP_FOLD = 8, GP_FLUSH = 64;
static_assert(GP_WAVES * GP_WCT * 16 == GP_NT && GP_NT * 32 * 2 == GP_UNIT && GP_DMA >= 1, "unit shape");
static_assert(GP_FLUSH % GP_FOLD == 0, "flushes at fold boundaries");

// One workgroup per (k-block, column group): wavefront w forms column tiles w + 4 j (j < 8), lane l
// its fragment of 8 rows; the three terms a = A1 + A2 + A3 as in k_gauss_bf16 (rounded to FP32 first).
template <typename TA>
__global__ __launch_bounds__(256) void k_gauss_split3(const TA* __restrict__ A, int64_t lda, int64_t d,
                                                      int64_t r0, int64_t r1, int ng, char* __restrict__ planes) {
  const int64_t kb = blockIdx.x / ng;
  const int g = (int)(blockIdx.x - kb * ng);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t rb = r0 + kb * 32 + 8 * (lane >> 4);
  char* ub = planes + (kb * ng + g) * 3 * (int64_t)GP_UNIT + lane * 16;
#pragma unroll 2
  for (int j = 0; j < GP_NT / 16 / 4; ++j) {
    const int ct = w + 4 * j;
    const int64_t col = (int64_t)g * GP_NT + ct * 16 + (lane & 15);
    g_bf8 h, gg, e;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t row = rb + i;
      const float a = (row < r1 && col < d) ? (float)A[row * lda + col] : 0.0f;
      const __bf16 h0 = (__bf16)a;
      const float r = a - (float)h0;
      const __bf16 g0 = (__bf16)r;
      const float q = r - (float)g0;
      h[i] = h0;
      gg[i] = g0;
      e[i] = (__bf16)q;
    }
    *(g_bf8*)(ub + ct * 1024) = h;
    *(g_bf8*)(ub + GP_UNIT + ct * 1024) = gg;
    *(g_bf8*)(ub + 2 * GP_UNIT + ct * 1024) = e;
  }
}

// Eight normals S[irow][8 blk + i] rounded to BF16 (zeros for rows past m) from a finished Philox block.
__device__ __forceinline__ g_bf8 gp_normals(const PhiloxState& P, bool iok) {
  const uint64_t ws[4] = {P.c0, P.c1, P.c2, P.c3};
  g_bf8 o;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float c, sn;
    box_muller_pair_hw(ws[q], c, sn);
    o[2 * q] = (__bf16)(iok ? c : 0.0f);
    o[2 * q + 1] = (__bf16)(iok ? sn : 0.0f);
  }
  return o;
}

__global__ __launch_bounds__(GP_WAVES * 64, 1) void k_gauss_bf16_planes(
    uint64_t seed, uint64_t t, const char* __restrict__ planes, int64_t r0, int64_t nkb, int ng, int64_t kbps,
    int rtiles, int64_t m, int64_t d, int fresh_in, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) char Ring[GP_RING * GP_UNIT];
  __shared__ __attribute__((aligned(16))) g_bf8 Nrm[2][4][64];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // XCD-aware order: consecutive workgroups are dispatched to different XCDs, so the logical index
  // L = (b mod 8) (G / 8) + b / 8 puts the row tiles of one (column group, k-split) on one XCD, where they
  // read the same units from that XCD's L2
  const int G = gridDim.x, b = blockIdx.x;
  const int L = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int rt = L % rtiles, rest = L / rtiles, g = rest % ng, ksi = rest / ng;
  const int64_t kb0 = (int64_t)ksi * kbps, kb1 = min(nkb, kb0 + kbps);
  const int ns = kb1 > kb0 ? (int)(kb1 - kb0) : 0;
  const int nu = 3 * ns;
  const int lg = lane >> 4;
  const int myrt = wv & 3, par = wv >> 2;  // the row tile and the step parity whose normals this wavefront forms
  const int64_t irow = (int64_t)rt * GP_MT + myrt * 16 + (lane & 15);
  const bool iok = irow < m;
  const char* gsrc = planes + ((kb0 * ng + g) * 3) * (int64_t)GP_UNIT + (wv * 1024 + lane * 16);
  const int64_t ustride = (int64_t)ng * 3 * GP_UNIT;  // bytes from one step's units to the next step's

  // unit j (step j / 3, term j % 3) into ring slot j % 4, one 16-byte load per lane per piece q < GP_DMA;
  // past the last unit the last one is loaded again into a slot nobody reads, so every unit section
  // waits for the same count of loads
  auto unit_src = [&](int j) {
    const int jj = j < nu ? j : nu - 1;
    const int s = jj / 3, p = jj - 3 * s;
    return gsrc + s * ustride + p * (int64_t)GP_UNIT;
  };
  auto issue_piece = [&](const char* src, int j, int q) {
    char* dst = Ring + (j % GP_RING) * GP_UNIT + wv * 1024;
    __builtin_amdgcn_global_load_lds(src + q * GP_WAVES * 1024,
                                     (__attribute__((address_space(3))) void*)(dst + q * GP_WAVES * 1024), 16, 0, 0);
  };
  auto issue = [&](int j) {
    const char* src = unit_src(j);
#pragma unroll
    for (int q = 0; q < GP_DMA; ++q) issue_piece(src, j, q);
  };
  auto philox_at = [&](int s) {
    return PhiloxState{(uint64_t)((r0 >> 3) + (kb0 + s) * 4 + lg), TAG_GAUSS, t, (uint64_t)irow, seed, 0};
  };

  g_f4 acc[4][GP_WCT], hi[4][GP_WCT];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < GP_WCT; ++c) {
      acc[r][c] = (g_f4){0.0f, 0.0f, 0.0f, 0.0f};
      hi[r][c] = (g_f4){0.0f, 0.0f, 0.0f, 0.0f};
    }
  bool fresh = fresh_in != 0;
  // element offsets inside this k-split's partial (m d < 2^28 on this path: 32-bit byte offsets)
  char* pbase = (char*)(part + (int64_t)ksi * m * d);
  const int64_t row0 = (int64_t)rt * GP_MT + 4 * lg, col0 = (int64_t)g * GP_NT + wv * (GP_WCT * 16) + (lane & 15);
  const uint32_t o0 = (uint32_t)(row0 * d + col0);
  const int64_t rlim = m - row0, clim = d - col0;  // rows r 16 + v < rlim, columns c 16 < clim
  // The sums into the FP64 partial: the first store of a launch sequence, then atomic adds without
  // return (no registers held, no wait).  Each address has one writer (this lane), whose adds are applied
  // in program order, so the partial is the same at every run.
  auto flush = [&]() {
    const bool st = fresh;
    // the addresses are formed here, not hoisted out of the step loop (they would hold 64+ registers)
    uint32_t ob = o0;
    asm volatile("" : "+v"(ob));
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = r * 16 + v;
        if (rr < rlim) {
          const uint32_t orow = ob + (uint32_t)(rr * d);
#pragma unroll
          for (int c = 0; c < GP_WCT; ++c)
            if (c * 16 < clim) {
              double* q = (double*)(pbase + (orow + (uint32_t)(c * 16)) * 8u);
              if (st) *q = (double)hi[r][c][v];
              else __hip_atomic_fetch_add(q, (double)hi[r][c][v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
      }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < GP_WCT; ++c) hi[r][c] = (g_f4){0.0f, 0.0f, 0.0f, 0.0f};
    fresh = false;
    vm_wait<0>();  // the stores and adds have left: unit loads are counted from zero again
  };

  if (ns > 0) {
    issue(0);
    issue(1);
    issue(2);
    {
      PhiloxState P = philox_at(par);
      P.rounds<0, 10>();
      Nrm[par][myrt][lane] = gp_normals(P, iok);
    }
    g_bf8 af[4];
    // one unit of step s: wait for it, pass the barrier, start the unit three ahead, 16 MFMAs; GEN: the
    // Philox rounds [R0, R1) of this wavefront's next block ride along
    auto unit = [&](int s, auto pc, auto gen, PhiloxState& P) {
      constexpr int p = decltype(pc)::value;
      constexpr bool GEN = decltype(gen)::value;
      const int j = 3 * s + p;
      vm_wait<2 * GP_DMA>();
      lds_barrier();  // unit j has landed for every wavefront; unit j - 1's slot is no longer read
      const char* nsrc = unit_src(j + 3);
      if constexpr (p == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) af[r] = Nrm[s & 1][r][lane];
      }
      g_bf8 bv[GP_WCT];
      {
        static_assert(GP_WCT == 4, "one four-read statement per unit");
        const uint32_t U = (uint32_t)(uintptr_t)(Ring + (j % GP_RING) * GP_UNIT + wv * GP_WCT * 1024 + lane * 16);
        int4 x0, x1, x2, x3;
        lds_read4_b128<1024>(U, x0, x1, x2, x3);
        bv[0] = __builtin_bit_cast(g_bf8, x0);
        bv[1] = __builtin_bit_cast(g_bf8, x1);
        bv[2] = __builtin_bit_cast(g_bf8, x2);
        bv[3] = __builtin_bit_cast(g_bf8, x3);
      }
      // the loads of unit j + 3 go out one piece per column tile, between the MFMAs: the CU's address
      // unit takes about 20 cycles per 1 KB piece, and a wavefront whose load waits for it issues nothing
      // after it, so eight wavefronts issuing all their pieces at once would stall their MFMAs
      static_assert(GP_DMA == GP_WCT, "one piece per column tile");
#pragma unroll
      for (int c = 0; c < GP_WCT; ++c) {
        issue_piece(nsrc, j + 3, c);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[r], bv[c], acc[r][c], 0, 0, 0);
      }
      if constexpr (GEN) {
        if constexpr (p == 0) P.rounds<0, 4>();
        else if constexpr (p == 1) P.rounds<4, 8>();
        else P.rounds<8, 10>();
      }
      // the order the scheduler keeps: one load piece, four MFMAs (and a share of the Philox rounds)
#pragma unroll
      for (int c = 0; c < GP_WCT; ++c) {
        __builtin_amdgcn_sched_group_barrier(0x010, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);

      }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using T = std::true_type;
    using F = std::false_type;
    for (int s = 0; s < ns; ++s) {
      if ((s & 1) == par) {
        // this wavefront's fragment of step s is consumed now: form the one of step s + 2
        PhiloxState P = philox_at(s + 2);
        unit(s, I0{}, T{}, P);
        unit(s, I1{}, T{}, P);
        unit(s, I2{}, T{}, P);
        Nrm[s & 1][myrt][lane] = gp_normals(P, iok);  // every wavefront read slot s & 1 before this step's
                                                      // second barrier
      } else {
        PhiloxState P{};
        unit(s, I0{}, F{}, P);
        unit(s, I1{}, F{}, P);
        unit(s, I2{}, F{}, P);
      }
      if ((s + 1) % GP_FOLD == 0 || s == ns - 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int c = 0; c < GP_WCT; ++c) {
            hi[r][c] += acc[r][c];
            acc[r][c] = (g_f4){0.0f, 0.0f, 0.0f, 0.0f};
          }
        if ((s + 1) % GP_FLUSH == 0 || s == ns - 1) flush();
      }
    }
  } else if (fresh) {
    flush();  // an empty k-split still initialises its partial
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

int g_gauss_planes_min_d = 384;
int g_gauss_planes_wgs = 512;
int g_gauss_chunk_rows = 0;

// The plan of the planes form: column groups, row tiles, k-splits per launch (about g_gauss_planes_wgs
// workgroups, one per compute unit) and rows per chunk (planes of about 1 GiB unless set).
struct GpPlan {
  int ng, rtiles, ks;
  int64_t rc;
};
// (m d below 2^28: the product kernel addresses its partial with 32-bit byte offsets)
static bool gauss_planes(int64_t m, int64_t d, int bf16) {
  return bf16 && d >= g_gauss_planes_min_d && m * d < ((int64_t)1 << 28);
}
static GpPlan gp_plan(int64_t m, int64_t d, int64_t n) {
  GpPlan p;
  p.ng = (int)((d + GP_NT - 1) / GP_NT);
  p.rtiles = (int)((m + GP_MT - 1) / GP_MT);
  const int64_t tiles = (int64_t)p.ng * p.rtiles;
  int64_t ks = (g_gauss_planes_wgs + tiles - 1) / tiles;
  const int64_t nkb = (n + 31) / 32;
  if (ks > nkb) ks = nkb;
  if (ks > 512) ks = 512;
  p.ks = ks < 1 ? 1 : (int)ks;
  int64_t rc = g_gauss_chunk_rows > 0 ? g_gauss_chunk_rows : ((int64_t)1 << 30) / (6 * (int64_t)GP_NT * p.ng);
  rc = rc / 32 * 32;
  if (rc < 32) rc = 32;
  const int64_t n32 = nkb * 32;
  p.rc = rc < n32 ? rc : n32;
  return p;
}
static size_t gp_part_bytes(int64_t m, int64_t d, const GpPlan& p) {
  return ((size_t)p.ks * m * d * sizeof(double) + 255) / 256 * 256;
}

size_t gauss_partial_bytes(int64_t m, int64_t d, int64_t n, int bf16) {
  if (gauss_planes(m, d, bf16)) {
    const GpPlan p = gp_plan(m, d, n);
    return gp_part_bytes(m, d, p) + (size_t)(p.rc / 32) * p.ng * 3 * GP_UNIT;
  }
  return (size_t)gauss_nks(m, d, n) * m * d * sizeof(double);
}

void gauss_apply(hipStream_t st, uint64_t seed, uint64_t t, const void* A, int a_f32, int64_t n,
                 int64_t d, int64_t lda, int64_t m, int bf16, double* partials, double* SA,
                 int64_t ldsa) {
  const int64_t nks = gauss_nks(m, d, n);
  int64_t kchunk = (n + nks - 1) / nks;
  dim3 g((unsigned)((m + GM_ROWS - 1) / GM_ROWS), (unsigned)((d + GM_COLS - 1) / GM_COLS), (unsigned)nks);
  if (gauss_planes(m, d, bf16)) {
    const GpPlan p = gp_plan(m, d, n);
    char* planes = (char*)partials + gp_part_bytes(m, d, p);
    const int grid = p.rtiles * p.ng * p.ks;
    for (int64_t r0 = 0; r0 < n; r0 += p.rc) {
      const int64_t r1 = min(n, r0 + p.rc), nkb = (r1 - r0 + 31) / 32;
      const dim3 gs((unsigned)(nkb * p.ng));
      if (a_f32)
        hipLaunchKernelGGL(k_gauss_split3<float>, gs, dim3(256), 0, st, (const float*)A, lda, d, r0, r1, p.ng, planes);
      else
        hipLaunchKernelGGL(k_gauss_split3<double>, gs, dim3(256), 0, st, (const double*)A, lda, d, r0, r1, p.ng,
                           planes);
      const int64_t kbps = (nkb + p.ks - 1) / p.ks;
      hipLaunchKernelGGL(k_gauss_bf16_planes, dim3((unsigned)grid), dim3(GP_WAVES * 64), 0, st, seed, t,
                         (const char*)planes, r0, nkb, p.ng, kbps, p.rtiles, m, d, r0 == 0 ? 1 : 0, partials);
    }
    hipLaunchKernelGGL(k_gauss_reduce, dim3((unsigned)((m * d + 255) / 256)), dim3(256), 0, st, partials,
                       (int64_t)p.ks, m, d, 1.0 / sqrt((double)m), SA, ldsa);
    return;
  }
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
