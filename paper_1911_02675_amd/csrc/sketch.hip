// SRHT and SJLT sketches S A (Section 2).
//
// SRHT, S = m^{-1/2} R H_N E with the +-1 Sylvester Hadamard H_N[k, j] = (-1)^popcount(k & j) and A
// zero-padded to N rows.  Writing j = j_hi N1 + j_lo and k = k_hi N1 + k_lo gives
// H_N = H_{N2} (x) H_{N1}, so
//     (H E A)[k] = sum_{j_hi} (-1)^popcount(k_hi & j_hi) T[j_hi, k_lo],
//     T[j_hi, k_lo] = sum_{j_lo} H_{N1}[k_lo, j_lo] e_j A[j].
// Pass A computes T block by block (a column slice of N1 = 256 consecutive rows, or N rows when
// N < 256), keeping only the k_lo that some selected row needs.  T is stored k_lo-major: row-major,
// T[(slot(k_lo) N2 + j_hi) dT + col] with dT = d rounded up to 16 bytes, or, for the LDS-staged pass B,
// in stripes of 64 columns, T[((slot(k_lo) ncbs + col / 64) N2 + j_hi) 64 + col mod 64], so that each
// pass B workgroup streams its bucket's N2 x 64 stripe contiguously while it evaluates the high-bit sum
// for the bucket's selected rows on the matrix cores.  HBM traffic is about |A| + 2 f |T| with f the
// fraction of k_lo values used; pass B does m N2 d / F multiply-adds after an F-point fold.
//
// SJLT: the hashed scatter is done as a stable counting sort of the (target, row) pairs followed by
// a segmented reduction per target row, in increasing row order: no atomics touch S A, and the
// result is bitwise reproducible.
#include "internal.h"

#include <type_traits>

namespace lsq {

constexpr int SRHT_N1_MAX = 512;
int g_srht_fold8_rows_f32 = 64;
int g_srht_fold8_rows_f64 = 128;
int g_srht_stream_rows_f32 = 192;
int g_srht_stream_rows_f64 = 192;
int g_srht_passa_wgs = 0;
int g_srht_passb_wgs = 8192;

// --------------------------------------------------------------------------------------------------
// Grouping of the selected rows by k_lo (single workgroup): bucket counts, their scan, a scatter.
// --------------------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_srht_groups(const int64_t* __restrict__ rows, int64_t m,
                                                      int N1, int* __restrict__ slot,
                                                      int* __restrict__ order,
                                                      int* __restrict__ bstart,
                                                      int* __restrict__ nneeded) {
  __shared__ int cnt[SRHT_N1_MAX];
  __shared__ int cur[SRHT_N1_MAX];
  __shared__ int sh[17];
  const int tid = threadIdx.x;
  if (tid < N1) cnt[tid] = 0;
  __syncthreads();
  for (int64_t q = tid; q < m; q += 1024) atomicAdd(&cnt[rows[q] & (N1 - 1)], 1);
  __syncthreads();
  // exclusive scans of cnt and of (cnt > 0): one entry per thread (N1 <= 512 < 1024)
  const int c = tid < N1 ? cnt[tid] : 0;
  const int lane = tid & 63, wv = tid >> 6;
  int inc = c, incu = c > 0 ? 1 : 0;
  const int used = incu;
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(inc, off, 64), ou = __shfl_up(incu, off, 64);
    if (lane >= off) {
      inc += o;
      incu += ou;
    }
  }
  __shared__ int wsum[16], wsumu[16];
  if (lane == 63) {
    wsum[wv] = inc;
    wsumu[wv] = incu;
  }
  __syncthreads();
  int pre = 0, preu = 0;
  for (int w = 0; w < wv; ++w) {
    pre += wsum[w];
    preu += wsumu[w];
  }
  const int ex = pre + inc - c, exu = preu + incu - used;
  if (tid < N1) {
    bstart[tid] = ex;
    slot[tid] = used ? exu : -1;
    cur[tid] = ex;
  }
  if (tid == N1 - 1) {
    bstart[N1] = ex + c;
    *nneeded = exu + used;
  }
  __syncthreads();
  for (int64_t q = tid; q < m; q += 1024) {
    const int pos = atomicAdd(&cur[rows[q] & (N1 - 1)], 1);
    order[pos] = (int)q;
  }
  // The order inside a bucket is left as the atomics made it: every selected row's value is a sum over
  // j_hi computed by itself (the rows sharing a tile only share the loads of T), so no output bit depends
  // on it.
  (void)sh;
}

void srht_plan_groups(hipStream_t st, const int64_t* rows, int64_t m, int64_t N1, int* slot,
                      int* order, int* bstart, int* nneeded_dev) {
  hipLaunchKernelGGL(k_srht_groups, dim3(1), dim3(1024), 0, st, rows, m, (int)N1, slot, order, bstart,
                     nneeded_dev);
}

// Row stride of T in elements: d rounded up to a 16-byte multiple of the compute type.
static int64_t srht_dT(int64_t d, int compute_f32) {
  const int64_t v = compute_f32 ? 4 : 2;
  return (d + v - 1) / v * v;
}

// T is sized for either layout: row-major rows of dT, or 64-column stripes (dT rounded up to 64).
size_t srht_tbuf_bytes(int64_t N2, int64_t nneeded, int64_t d, int compute_f32) {
  const int64_t w = (srht_dT(d, compute_f32) + 63) / 64 * 64;
  return (size_t)N2 * (size_t)nneeded * (size_t)w * (compute_f32 ? 4 : 8);
}

// Element (slot sl, j_hi, column col) of T.  ncbs = 0: row-major, rows of dT; otherwise each slot's
// block is ncbs stripes of 64 columns, each stripe N2 rows of 64 contiguous elements, so that a
// workgroup of the LDS-staged pass B streams its stripe as one contiguous range.
__device__ __forceinline__ int64_t srht_tpos(int64_t sl, int64_t jh, int64_t col, int64_t N2, int64_t dT,
                                             int64_t ncbs) {
  return ncbs ? ((sl * ncbs + (col >> 6)) * N2 + jh) * 64 + (col & 63) : (sl * N2 + jh) * dT + col;
}

template <typename T, int W>
struct SVec;
template <>
struct SVec<float, 4> {
  typedef float __attribute__((ext_vector_type(4))) t;
};
template <>
struct SVec<float, 2> {
  typedef float __attribute__((ext_vector_type(2))) t;
};
template <>
struct SVec<double, 2> {
  typedef double __attribute__((ext_vector_type(2))) t;
};
template <>
struct SVec<double, 4> {
  typedef double __attribute__((ext_vector_type(4))) t;
};

// --------------------------------------------------------------------------------------------------
// Pass A (N >= 256): blocks of SRHT_N1 = 256 rows.  Layout 1: thread (c, g) holds rows g + G i;
// butterflies over i transform the high row bits in registers.  One LDS transpose to layout 2:
// thread (c, h) holds the G consecutive rows of each of its row groups; butterflies over the low
// bits.  LDS traffic is one write and one read of the tile.
// --------------------------------------------------------------------------------------------------
constexpr int SRHT_N1 = 256;

template <int V, typename T>
__device__ __forceinline__ void fwht_regs(T (&x)[V]) {
#pragma unroll
  for (int h = 1; h < V; h <<= 1)
#pragma unroll
    for (int i = 0; i < V; ++i)
      if ((i & h) == 0) {
        const T u = x[i], v = x[i + h];
        x[i] = u + v;
        x[i + h] = u - v;
      }
}

// Vector form: 16 lanes per row, each holding VW = 16 / sizeof(TC) consecutive columns (256-byte row
// segments of T), G = 16 row groups of 16 rows per thread.  Needs lda and d multiples of VW and A
// aligned to VW elements.  Loads are never masked: lanes past the last column read a clamped column
// (columns do not mix in the transform, and those lanes store nothing), and rows past n read row
// n - 1 and are multiplied by a zero sign.  Grid (N2, slice groups): a workgroup walks the column
// slices blockIdx.y, blockIdx.y + gridDim.y, ... of its block, loading the next slice while
// transforming the current one.
//   GRAD: the workgroup also forms its block's share of A^T y (the first gradient of the least-squares
// solve from x = 0, taken here while the rows are in registers instead of in a separate pass over A):
// row jhi of gpart (width d + 1) gets sum_r y_r A[r][col] over the block's 256 rows for every column of
// its slices, and the slice group 0 workgroup adds sum_r y_r^2 in column d, in the layout of the fused
// pass's partials.  FP64 products and sums: per thread over its 16 rows, then across the 4 row groups of
// a wavefront, then across the 4 wavefronts, in that order.
template <typename TA, typename TC, bool GRAD>
__global__ __launch_bounds__(256) void k_srht_passA_vec(const TA* __restrict__ A, int64_t n, int64_t d,
                                                            int64_t lda, const int8_t* __restrict__ signs,
                                                            const int* __restrict__ slot, int64_t N2,
                                                            int64_t dT, int64_t ncbs, TC* __restrict__ T,
                                                            const double* __restrict__ y,
                                                            double* __restrict__ gpart) {
  constexpr int VW = 16 / sizeof(TC);
  typedef typename SVec<TA, VW>::t va;
  typedef typename SVec<TC, VW>::t vc;
  constexpr int LR = 16;          // lanes per row segment
  constexpr int DC = LR * VW;     // columns per slice
  constexpr int G = 256 / LR;     // row groups
  constexpr int V = SRHT_N1 / G;  // rows per thread
  constexpr int RS = LR + 1;      // padded LDS row stride (vectors)
  static_assert(V == G, "layout 2 assumes one row group per thread");
  __shared__ vc tile[SRHT_N1 * RS];
  __shared__ int slot_s[SRHT_N1];
  __shared__ int8_t sg_s[SRHT_N1];
  __shared__ double ys[GRAD ? SRHT_N1 : 1];        // y of the block's rows (0 past n)
  __shared__ double gred[GRAD ? 4 * LR * VW : 1];  // per-wavefront column partials of A^T y
  __shared__ double yred[GRAD ? 4 : 1];
  const int64_t jhi = blockIdx.x;
  const int tid = threadIdx.x;
  const int c = tid % LR, g = tid / LR, h = g;
  const int64_t rbase = jhi * SRHT_N1;
  const int nslices = (int)((d + DC - 1) / DC);
  const bool full = rbase + SRHT_N1 <= n;
  slot_s[tid] = slot[tid];
  sg_s[tid] = rbase + tid < n ? signs[rbase + tid] : (int8_t)0;
  if constexpr (GRAD) {
    const double yv = rbase + tid < n ? y[rbase + tid] : 0.0;
    ys[tid] = yv;
    const double yy = wave_sum(yv * yv);
    if ((tid & 63) == 0) yred[tid >> 6] = yy;
  }
  __syncthreads();
  if constexpr (GRAD) {
    if (blockIdx.y == 0 && tid == 0) gpart[jhi * (d + 1) + d] = ((yred[0] + yred[1]) + yred[2]) + yred[3];
  }
  int sidx = blockIdx.y;
  if (sidx >= nslices) return;
  const int64_t step = (int64_t)G * lda / VW;
  auto load = [&](int s, vc(&x)[V]) {
    int64_t col = (int64_t)s * DC + (int64_t)c * VW;
    col = col < d ? col : d - VW;  // d is a multiple of VW
    if (full) {
      const va* p = (const va*)(A + (rbase + g) * lda + col);
#pragma unroll
      for (int i = 0; i < V; ++i) x[i] = __builtin_convertvector(__builtin_nontemporal_load(p + i * step), vc);
    } else {
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const int64_t r = min(rbase + g + G * i, n - 1);
        x[i] = __builtin_convertvector(__builtin_nontemporal_load((const va*)(A + r * lda + col)), vc);
      }
    }
  };
  vc x[V];
  load(sidx, x);
  for (; sidx < nslices; sidx += gridDim.y) {
    const int64_t col = (int64_t)sidx * DC + (int64_t)c * VW;
    const int nxt = sidx + gridDim.y;
    vc xn[V];
    if (nxt < nslices) load(nxt, xn);
    if constexpr (GRAD) {
      // rows g + 16 i of the block, columns col .. col + VW - 1, before the sign flips
      double sg[VW];
#pragma unroll
      for (int u = 0; u < VW; ++u) sg[u] = 0.0;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        const double yv = ys[g + G * i];
#pragma unroll
        for (int u = 0; u < VW; ++u) sg[u] = fma(yv, (double)x[i][u], sg[u]);
      }
#pragma unroll
      for (int u = 0; u < VW; ++u) {
        sg[u] += __shfl_xor(sg[u], 16, 64);
        sg[u] += __shfl_xor(sg[u], 32, 64);
      }
      if ((tid & 63) < LR)
#pragma unroll
        for (int u = 0; u < VW; ++u) gred[((tid >> 6) * LR + c) * VW + u] = sg[u];
    }
#pragma unroll
    for (int i = 0; i < V; ++i) x[i] *= (TC)sg_s[g + G * i];
    fwht_regs<V>(x);
#pragma unroll
    for (int i = 0; i < V; ++i) tile[(g + G * i) * RS + c] = x[i];
    __syncthreads();
    if constexpr (GRAD) {
      if (tid < LR && col < d)
#pragma unroll
        for (int u = 0; u < VW; ++u)
          gpart[jhi * (d + 1) + col + u] = ((gred[c * VW + u] + gred[(LR + c) * VW + u]) +
                                            gred[(2 * LR + c) * VW + u]) + gred[(3 * LR + c) * VW + u];
    }
    vc z[G];
#pragma unroll
    for (int j = 0; j < G; ++j) z[j] = tile[(G * h + j) * RS + c];
    fwht_regs<G>(z);
    if (col < d) {
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const int sl = slot_s[G * h + j];
        if (sl >= 0) __builtin_nontemporal_store(z[j], (vc*)(T + srht_tpos(sl, jhi, col, N2, dT, ncbs)));
      }
    }
    __syncthreads();
    if (nxt < nslices) {
#pragma unroll
      for (int i = 0; i < V; ++i) x[i] = xn[i];
    }
  }
}

// Scalar form for any lda, d and alignment: 128-byte column slices, one column per lane.
template <typename TA, typename TC, int V, int G>
__device__ __forceinline__ void srht_load_slice(const TA* __restrict__ A, int64_t n, int64_t d,
                                                int64_t lda, const int8_t* __restrict__ sg_s,
                                                int64_t rbase, int g, int64_t col, TC (&x)[V]) {
  // row rbase + g + G i: one base pointer and a uniform stride G * lda
  const TA* p = A + (rbase + g) * lda + col;
  const int64_t step = (int64_t)G * lda;
  if (rbase + SRHT_N1 <= n && col < d) {
#pragma unroll
    for (int i = 0; i < V; ++i) x[i] = (TC)__builtin_nontemporal_load(p + i * step);
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i)
      x[i] = (rbase + g + G * i < n && col < d) ? (TC)__builtin_nontemporal_load(p + i * step) : (TC)0;
  }
#pragma unroll
  for (int i = 0; i < V; ++i)
    if (sg_s[g + G * i] < 0) x[i] = -x[i];
}

template <typename TA, typename TC>
__global__ __launch_bounds__(256) void k_srht_passA2(const TA* __restrict__ A, int64_t n, int64_t d,
                                                     int64_t lda, const int8_t* __restrict__ signs,
                                                     const int* __restrict__ slot, int64_t N2,
                                                     int64_t dT, int64_t ncbs, TC* __restrict__ T) {
  constexpr int DC = 128 / sizeof(TC);   // columns per slice
  constexpr int G = 256 / DC;            // row groups (low row bits)
  constexpr int V = SRHT_N1 / G;         // rows per thread
  constexpr int K = V / G;               // row groups per thread in layout 2
  __shared__ TC tile[SRHT_N1 * DC];
  __shared__ int slot_s[SRHT_N1];
  __shared__ int8_t sg_s[SRHT_N1];
  const int64_t jhi = blockIdx.x;
  const int tid = threadIdx.x;
  const int c = tid % DC, g = tid / DC, h = g;
  const int64_t rbase = jhi * SRHT_N1;
  const int nslices = (int)((d + DC - 1) / DC);
  slot_s[tid] = slot[tid];
  sg_s[tid] = rbase + tid < n ? signs[rbase + tid] : (int8_t)1;
  __syncthreads();
  int sidx = blockIdx.y;
  if (sidx >= nslices) return;
  TC x[V];
  srht_load_slice<TA, TC, V, G>(A, n, d, lda, sg_s, rbase, g, (int64_t)sidx * DC + c, x);
  for (; sidx < nslices; sidx += gridDim.y) {
    const int64_t col = (int64_t)sidx * DC + c;
    const int nxt = sidx + gridDim.y;
    TC xn[V];
    if (nxt < nslices) srht_load_slice<TA, TC, V, G>(A, n, d, lda, sg_s, rbase, g, (int64_t)nxt * DC + c, xn);
    fwht_regs<V>(x);
#pragma unroll
    for (int i = 0; i < V; ++i) tile[(g + G * i) * DC + c] = x[i];
    __syncthreads();
    // layout 2: thread (c, h) holds rows G (h + G k) + j, j < G, k < K
#pragma unroll
    for (int k = 0; k < K; ++k) {
      TC z[G];
#pragma unroll
      for (int j = 0; j < G; ++j) z[j] = tile[(G * (h + G * k) + j) * DC + c];
      fwht_regs<G>(z);
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const int r = G * (h + G * k) + j;
        const int sl = slot_s[r];
        if (sl >= 0 && col < d) __builtin_nontemporal_store(z[j], T + srht_tpos(sl, jhi, col, N2, dT, ncbs));
      }
    }
    __syncthreads();
    if (nxt < nslices) {
#pragma unroll
      for (int i = 0; i < V; ++i) x[i] = xn[i];
    }
  }
}

// --------------------------------------------------------------------------------------------------
// Pass A for N < 256 (one block of N1 = N rows): sign flip, zero padding and the transform in LDS.
// --------------------------------------------------------------------------------------------------
template <typename TA, typename TC>
__global__ __launch_bounds__(256) void k_srht_passA(const TA* __restrict__ A, int64_t n, int64_t d,
                                                    int64_t lda, int N1, const int8_t* __restrict__ signs,
                                                    const int* __restrict__ slot, int64_t N2, int64_t dT,
                                                    TC* __restrict__ T) {
  constexpr int DC = 128 / sizeof(TC);
  __shared__ TC tile[SRHT_N1_MAX * DC];
  const int64_t jhi = blockIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * DC;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < N1 * DC; idx += 256) {
    const int r = idx / DC, c = idx % DC;
    const int64_t row = jhi * N1 + r, col = c0 + c;
    TC v = 0;
    if (row < n && col < d) {
      v = (TC)A[row * lda + col];
      if (signs[row] < 0) v = -v;
    }
    tile[idx] = v;
  }
  for (int h = 1; h < N1; h <<= 1) {
    __syncthreads();
    for (int pidx = tid; pidx < (N1 / 2) * DC; pidx += 256) {
      const int c = pidx % DC, pr = pidx / DC;
      const int i0 = ((pr / h) * 2 * h) + (pr % h), i1 = i0 + h;
      const TC u = tile[i0 * DC + c], v = tile[i1 * DC + c];
      tile[i0 * DC + c] = u + v;
      tile[i1 * DC + c] = u - v;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < N1 * DC; idx += 256) {
    const int r = idx / DC, c = idx % DC;
    const int sl = slot[r];
    const int64_t col = c0 + c;
    if (sl >= 0 && col < d) T[((int64_t)sl * N2 + jhi) * dT + col] = tile[idx];
  }
}

// --------------------------------------------------------------------------------------------------
// Pass B on FP64 matrix cores.  Workgroup (bucket k_lo, j_hi range, 512-column group); each wavefront
// owns NL * 16 * VW columns.  Per step of 4 consecutive j_hi: the +-1 signs form the 16 x 4 A operand
// of v_mfma_f64_16x16x4 (lane l: selected row l % 16 of the tile, j_hi offset l / 16), and 16-byte
// loads of the bucket's T rows (lane l: T row offset l / 16, VW columns) supply VW B operands each
// (block (il, e) takes element e of load il: columns c0 + 16 VW il + VW (l % 16) + e).  Up to QT = 2
// tiles of 16 selected rows share every load, so a bucket's T block is read once when it has at most
// 32 selected rows.  The 16 x 16 result blocks (lane l, register v: tile row l / 16 + 4 v, column
// l % 16 of the block) accumulate over the workgroup's j_hi range.
// --------------------------------------------------------------------------------------------------
typedef double lsq_d4 __attribute__((ext_vector_type(4)));
constexpr int SRHT_WGC = 512;  // columns per workgroup

template <typename TC, int NL, int QT>
__device__ __forceinline__ void srht_passB_tiles(const TC* __restrict__ base, int64_t dT, int64_t jh0,
                                                 int64_t jh1, int64_t c0, int64_t d,
                                                 const uint64_t (&khi)[QT], const bool (&qok)[QT],
                                                 int kk, int qi, double* __restrict__ out,
                                                 const int* __restrict__ ord, int nq) {
  constexpr int VW = 16 / sizeof(TC);
  constexpr int SRHT_PF = sizeof(TC) == 4 ? 4 : 3;  // steps of 4 rows in flight per wavefront
  typedef typename SVec<TC, VW>::t vc;
  lsq_d4 acc[QT][NL * VW];
#pragma unroll
  for (int t = 0; t < QT; ++t)
#pragma unroll
    for (int b = 0; b < NL * VW; ++b) acc[t][b] = (lsq_d4){0.0, 0.0, 0.0, 0.0};
  const vc* p = (const vc*)(base + c0) + qi;
  bool colok[NL];
#pragma unroll
  for (int il = 0; il < NL; ++il) colok[il] = c0 + (int64_t)(il * 16 + qi) * VW < dT;
  const int64_t rstep = dT / VW;
  vc raw[SRHT_PF][NL];
#pragma unroll
  for (int f = 0; f < SRHT_PF; ++f) {
    const int64_t j = jh0 + 4 * f + kk;
#pragma unroll
    for (int il = 0; il < NL; ++il)
      raw[f][il] = (j < jh1 && colok[il]) ? __builtin_nontemporal_load(p + j * rstep + il * 16) : (vc)(TC)0;
  }
  for (int64_t jh = jh0; jh < jh1; jh += 4 * SRHT_PF) {
#pragma unroll
    for (int f = 0; f < SRHT_PF; ++f) {
      const int64_t j = jh + 4 * f + kk;
      double a[QT];
#pragma unroll
      for (int t = 0; t < QT; ++t)
        a[t] = (qok[t] && j < jh1) ? ((__popcll(khi[t] & (uint64_t)j) & 1) ? -1.0 : 1.0) : 0.0;
      vc cur[NL];
#pragma unroll
      for (int il = 0; il < NL; ++il) cur[il] = raw[f][il];
      const int64_t jn = j + 4 * SRHT_PF;
#pragma unroll
      for (int il = 0; il < NL; ++il)
        raw[f][il] = (jn < jh1 && colok[il]) ? __builtin_nontemporal_load(p + jn * rstep + il * 16) : (vc)(TC)0;
#pragma unroll
      for (int il = 0; il < NL; ++il)
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const double bv = (double)cur[il][e];
#pragma unroll
          for (int t = 0; t < QT; ++t)
            acc[t][il * VW + e] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], bv, acc[t][il * VW + e], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int t = 0; t < QT; ++t)
#pragma unroll
    for (int il = 0; il < NL; ++il)
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int64_t col = c0 + (int64_t)(il * 16 + qi) * VW + e;
        if (col >= d) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int q = 16 * t + kk + 4 * v;
          if (q < nq) out[(int64_t)ord[q] * d + col] = acc[t][il * VW + e][v];
        }
      }
}

// Rows of one bucket are taken QMAX tiles (16 QMAX rows) at a time, each chunk in one sweep of the
// bucket's T block; QMAX = 4 halves the columns per wavefront to keep the accumulators in registers.
template <typename TC, int NL, int QT>
__device__ __forceinline__ void srht_passB_chunk(const TC* __restrict__ base, int64_t dT, int64_t jh0, int64_t jh1,
                                                 int64_t c0, int64_t d, const int64_t* __restrict__ rows,
                                                 const int* __restrict__ ord, int nq, int L1, int kk, int qi,
                                                 double* __restrict__ out) {
  bool qok[QT];
  uint64_t khi[QT];
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    qok[t] = 16 * t + qi < nq;
    khi[t] = qok[t] ? ((uint64_t)rows[ord[16 * t + qi]] >> L1) : 0ull;
  }
  srht_passB_tiles<TC, NL, QT>(base, dT, jh0, jh1, c0, d, khi, qok, kk, qi, out, ord, nq);
}

template <typename TC, int WGC, int QMAX>
__global__ __launch_bounds__(256, 2) void k_srht_passB(const TC* __restrict__ T, int64_t N2, int64_t d,
                                                       int64_t dT, int L1, const int64_t* __restrict__ rows,
                                                       const int* __restrict__ slot,
                                                       const int* __restrict__ order,
                                                       const int* __restrict__ bstart, int64_t m,
                                                       double* __restrict__ partial) {
  constexpr int VW = 16 / sizeof(TC);
  constexpr int NL = WGC / (4 * 16 * VW);
  const int klo = blockIdx.x;
  const int sl = slot[klo];
  if (sl < 0) return;
  const int js = blockIdx.y, JS = gridDim.y;
  const int64_t jh0 = N2 * js / JS, jh1 = N2 * (js + 1) / JS;
  const int b0 = bstart[klo], b1 = bstart[klo + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int qi = lane & 15, kk = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.z * WGC + (int64_t)wv * (NL * 16 * VW);
  const TC* base = T + (int64_t)sl * N2 * dT;
  double* out = partial + (int64_t)js * m * d;
  for (int cb = b0; cb < b1; cb += 16 * QMAX) {
    const int nq = min(16 * QMAX, b1 - cb);
    const int* ord = order + cb;
    if (nq <= 16) {
      srht_passB_chunk<TC, NL, 1>(base, dT, jh0, jh1, c0, d, rows, ord, nq, L1, kk, qi, out);
    } else if (QMAX == 2 || nq <= 32) {
      srht_passB_chunk<TC, NL, 2>(base, dT, jh0, jh1, c0, d, rows, ord, nq, L1, kk, qi, out);
    } else if (nq <= 48) {
      srht_passB_chunk<TC, NL, (QMAX > 2 ? 3 : 2)>(base, dT, jh0, jh1, c0, d, rows, ord, nq, L1, kk, qi, out);
    } else {
      srht_passB_chunk<TC, NL, QMAX>(base, dT, jh0, jh1, c0, d, rows, ord, nq, L1, kk, qi, out);
    }
  }
}

// FP32 T on the FP32 matrix cores (v_mfma_f32_16x16x4, twice the FP64 rate): chains of 4 steps (16
// terms) accumulate in FP32 and are then added into FP64 accumulators, so the summation error stays
// within 16 u of the sum of |T| terms on top of the 8 u of the transform (u = 2^-24), below the
// (log2 N + 2) 2u bound of an FP32 SRHT.  One load of VW floats per lane feeds VW blocks of 16
// columns (16 VW columns per wavefront).  Output layout of the FP32 16 x 16 result: lane l, register v
// holds row 4 (l / 16) + v, column l % 16.
typedef float lsq_f4v __attribute__((ext_vector_type(4)));

template <int QT, int VW>
__device__ __forceinline__ void srht_passB_tiles_f32(const float* __restrict__ base, int64_t dT, int64_t jh0,
                                                     int64_t jh1, int64_t c0, int64_t d,
                                                     const uint64_t (&khi)[QT], const bool (&qok)[QT], int kk,
                                                     int qi, double* __restrict__ out,
                                                     const int* __restrict__ ord, int nq) {
  constexpr int PF = 4;
  typedef typename SVec<float, VW>::t vc;
  lsq_f4v acc32[QT][VW];
  lsq_d4 acc64[QT][VW];
#pragma unroll
  for (int t = 0; t < QT; ++t)
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      acc32[t][e] = (lsq_f4v){0.f, 0.f, 0.f, 0.f};
      acc64[t][e] = (lsq_d4){0.0, 0.0, 0.0, 0.0};
    }
  const bool colok = c0 + (int64_t)qi * VW < dT;
  const vc* p = (const vc*)(base + c0) + qi;
  const int64_t rstep = dT / VW;
  vc raw[PF];
#pragma unroll
  for (int f = 0; f < PF; ++f) {
    const int64_t j = jh0 + 4 * f + kk;
    raw[f] = (j < jh1 && colok) ? __builtin_nontemporal_load(p + j * rstep) : (vc)0.f;
  }
  for (int64_t jh = jh0; jh < jh1; jh += 4 * PF) {
#pragma unroll
    for (int f = 0; f < PF; ++f) {
      const int64_t j = jh + 4 * f + kk;
      float a[QT];
#pragma unroll
      for (int t = 0; t < QT; ++t)
        a[t] = (qok[t] && j < jh1) ? ((__popcll(khi[t] & (uint64_t)j) & 1) ? -1.f : 1.f) : 0.f;
      const vc cur = raw[f];
      const int64_t jn = j + 4 * PF;
      raw[f] = (jn < jh1 && colok) ? __builtin_nontemporal_load(p + jn * rstep) : (vc)0.f;
#pragma unroll
      for (int e = 0; e < VW; ++e)
#pragma unroll
        for (int t = 0; t < QT; ++t)
          acc32[t][e] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], cur[e], acc32[t][e], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < QT; ++t)
#pragma unroll
      for (int e = 0; e < VW; ++e) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc64[t][e][v] += (double)acc32[t][e][v];
        acc32[t][e] = (lsq_f4v){0.f, 0.f, 0.f, 0.f};
      }
  }
#pragma unroll
  for (int t = 0; t < QT; ++t)
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const int64_t col = c0 + (int64_t)qi * VW + e;
      if (col >= d) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q = 16 * t + 4 * kk + v;
        if (q < nq) out[(int64_t)ord[q] * d + col] = acc64[t][e][v];
      }
    }
}

template <int QT, int VW>
__device__ __forceinline__ void srht_passB_chunk_f32(const float* __restrict__ base, int64_t dT, int64_t jh0,
                                                     int64_t jh1, int64_t c0, int64_t d,
                                                     const int64_t* __restrict__ rows, const int* __restrict__ ord,
                                                     int nq, int L1, int kk, int qi, double* __restrict__ out) {
  bool qok[QT];
  uint64_t khi[QT];
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    qok[t] = 16 * t + qi < nq;
    khi[t] = qok[t] ? ((uint64_t)rows[ord[16 * t + qi]] >> L1) : 0ull;
  }
  srht_passB_tiles_f32<QT, VW>(base, dT, jh0, jh1, c0, d, khi, qok, kk, qi, out, ord, nq);
}

template <int QMAX>
__global__ __launch_bounds__(256, 2) void k_srht_passB_f32(const float* __restrict__ T, int64_t N2, int64_t d,
                                                           int64_t dT, int L1, const int64_t* __restrict__ rows,
                                                           const int* __restrict__ slot,
                                                           const int* __restrict__ order,
                                                           const int* __restrict__ bstart, int64_t m,
                                                           double* __restrict__ partial) {
  const int klo = blockIdx.x;
  const int sl = slot[klo];
  if (sl < 0) return;
  const int js = blockIdx.y, JS = gridDim.y;
  const int64_t jh0 = N2 * js / JS, jh1 = N2 * (js + 1) / JS;
  const int b0 = bstart[klo], b1 = bstart[klo + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int qi = lane & 15, kk = lane >> 4;
  constexpr int VW = QMAX > 2 ? 2 : 4;  // four row tiles: 32 columns per wavefront keep the sums in registers
  const int64_t c0 = (int64_t)blockIdx.z * (64 * VW) + (int64_t)wv * (16 * VW);
  const float* base = T + (int64_t)sl * N2 * dT;
  double* out = partial + (int64_t)js * m * d;
  for (int cb = b0; cb < b1; cb += 16 * QMAX) {
    const int nq = min(16 * QMAX, b1 - cb);
    const int* ord = order + cb;
    if (nq <= 16) {
      srht_passB_chunk_f32<1, VW>(base, dT, jh0, jh1, c0, d, rows, ord, nq, L1, kk, qi, out);
    } else if (QMAX == 2 || nq <= 32) {
      srht_passB_chunk_f32<2, VW>(base, dT, jh0, jh1, c0, d, rows, ord, nq, L1, kk, qi, out);
    } else if (nq <= 48) {
      srht_passB_chunk_f32<(QMAX > 2 ? 3 : 2), VW>(base, dT, jh0, jh1, c0, d, rows, ord, nq, L1, kk, qi, out);
    } else {
      srht_passB_chunk_f32<QMAX, VW>(base, dT, jh0, jh1, c0, d, rows, ord, nq, L1, kk, qi, out);
    }
  }
}

// Large buckets (FP32 T): the two low bits e of k_hi are folded into a 4-point Walsh-Hadamard transform
// of each 4 consecutive T rows.  With j_hi = 4 j_a + j_b and k_hi = 4 k_a + e,
//     sum_{j_hi} (-1)^{k_hi . j_hi} T[j_hi] = sum_{j_a} (-1)^{k_a . j_a} U_e[j_a],
//     U_e[j_a] = sum_{j_b < 4} (-1)^{e . j_b} T[4 j_a + j_b],
// so the bucket's rows are grouped by e into tiles of 16, and each FP32 matrix-core step (K = 4 values
// of j_a) consumes 16 rows of T instead of 4.  The tile list (row, k_a, e) is built in LDS once per
// workgroup; at most SRHT_WT tiles are carried per sweep of the bucket's T block.  Each lane loads the
// 4 rows of its j_a (two columns each, 32 columns per wavefront) and forms U_0..U_3 with 8 adds.
// The tile list is built in parallel: one thread per row of the bucket.
// Summation: the 4-point transform adds 2 roundings (2 u) per term to the chains of 4 steps (16 terms)
// that are folded into FP64, so the bound stays below the (log2 N + 2) 2u of an FP32 SRHT.
constexpr int SRHT_WT = 6;        // tiles per sweep
constexpr int SRHT_WROWS = 192;   // rows of a bucket per tile build (larger buckets loop)
constexpr int SRHT_WMAXT = SRHT_WROWS / 16 + 4;  // at most this many tiles per build

__global__ __launch_bounds__(256, 2) void k_srht_passB_f32w(const float* __restrict__ T, int64_t N2, int64_t d,
                                                            int64_t dT, int L1, const int64_t* __restrict__ rows,
                                                            const int* __restrict__ slot,
                                                            const int* __restrict__ order,
                                                            const int* __restrict__ bstart, int64_t m,
                                                            double* __restrict__ partial) {
  typedef typename SVec<float, 2>::t vc;
  __shared__ int tq[SRHT_WMAXT][16];        // order[] positions of the tile's rows (-1: empty)
  __shared__ unsigned long long tka[SRHT_WMAXT][16];
  __shared__ int te[SRHT_WMAXT];
  __shared__ int ntiles;
  const int klo = blockIdx.x;
  const int sl = slot[klo];
  if (sl < 0) return;
  const int js = blockIdx.y, JS = gridDim.y;
  const int64_t jh0 = N2 * js / JS, jh1 = N2 * (js + 1) / JS;  // multiples of 4 (N2 / JS >= 512)
  const int b0 = bstart[klo], b1 = bstart[klo + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int qi = lane & 15, kk = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.z * 128 + (int64_t)wv * 32;
  const float* base = T + (int64_t)sl * N2 * dT;
  double* out = partial + (int64_t)js * m * d;
  const bool colok = c0 + (int64_t)qi * 2 < dT;
  const vc* p = (const vc*)(base + c0) + qi;
  const int64_t rstep = dT / 2;
  __shared__ int cnt[4], tbase[4];
  for (int cb = b0; cb < b1; cb += SRHT_WROWS) {
    const int ce = min(b1, cb + SRHT_WROWS);
    // tiles of rows grouped by e: count the groups, place each row (the order of rows inside a tile
    // does not change any output row), empty slots stay -1
    __syncthreads();
    for (int i = tid; i < SRHT_WMAXT * 16; i += 256) tq[i / 16][i % 16] = -1;
    if (tid < 4) cnt[tid] = 0;
    __syncthreads();
    int e_me = 0, slot_me = 0;
    uint64_t khi_me = 0;
    if (tid < ce - cb) {
      khi_me = (uint64_t)rows[order[cb + tid]] >> L1;
      e_me = (int)(khi_me & 3);
      slot_me = atomicAdd(&cnt[e_me], 1);
    }
    __syncthreads();
    if (tid == 0) {
      int nt = 0;
      for (int e = 0; e < 4; ++e) {
        tbase[e] = nt;
        const int k = (cnt[e] + 15) / 16;
        for (int t = 0; t < k; ++t) te[nt + t] = e;
        nt += k;
      }
      ntiles = nt;
    }
    __syncthreads();
    if (tid < ce - cb) {
      const int t = tbase[e_me] + slot_me / 16;
      tq[t][slot_me % 16] = cb + tid;
      tka[t][slot_me % 16] = khi_me >> 2;
    }
    __syncthreads();
    const int nt = ntiles;
    for (int t0 = 0; t0 < nt; t0 += SRHT_WT) {
      lsq_f4v acc32[SRHT_WT][2];
      lsq_d4 acc64[SRHT_WT][2];
      bool qok[SRHT_WT];
      uint64_t ka[SRHT_WT];
      int et[SRHT_WT];
#pragma unroll
      for (int t = 0; t < SRHT_WT; ++t) {
        const bool tv = t0 + t < nt;
        const int q = tv ? tq[t0 + t][qi] : -1;
        qok[t] = q >= 0;
        ka[t] = qok[t] ? tka[t0 + t][qi] : 0ull;
        et[t] = tv ? te[t0 + t] : 0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          acc32[t][e] = (lsq_f4v){0.f, 0.f, 0.f, 0.f};
          acc64[t][e] = (lsq_d4){0.0, 0.0, 0.0, 0.0};
        }
      }
      // j_a runs over [jh0/4, jh1/4); a step covers 4 consecutive j_a (lane group kk takes one)
      const int64_t ja0 = jh0 >> 2, ja1 = jh1 >> 2;
      for (int64_t jb = ja0; jb < ja1; jb += 16) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const int64_t ja = jb + 4 * f + kk;
          vc r[4];
#pragma unroll
          for (int b = 0; b < 4; ++b)
            r[b] = (ja < ja1 && colok) ? __builtin_nontemporal_load(p + (4 * ja + b) * rstep) : (vc)0.f;
          vc u[4];
          const vc s01 = r[0] + r[1], d01 = r[0] - r[1], s23 = r[2] + r[3], d23 = r[2] - r[3];
          u[0] = s01 + s23;
          u[1] = d01 + d23;
          u[2] = s01 - s23;
          u[3] = d01 - d23;
#pragma unroll
          for (int t = 0; t < SRHT_WT; ++t) {
            if (t0 + t >= nt) break;  // uniform
            const float a = (qok[t] && ja < ja1) ? ((__popcll(ka[t] & (uint64_t)ja) & 1) ? -1.f : 1.f) : 0.f;
            const int e = et[t];
            const vc ue = e == 0 ? u[0] : (e == 1 ? u[1] : (e == 2 ? u[2] : u[3]));
#pragma unroll
            for (int c = 0; c < 2; ++c)
              acc32[t][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, ue[c], acc32[t][c], 0, 0, 0);
          }
        }
#pragma unroll
        for (int t = 0; t < SRHT_WT; ++t)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[t][c][v] += (double)acc32[t][c][v];
            acc32[t][c] = (lsq_f4v){0.f, 0.f, 0.f, 0.f};
          }
      }
#pragma unroll
      for (int t = 0; t < SRHT_WT; ++t) {
        if (t0 + t >= nt) break;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const int64_t col = c0 + (int64_t)qi * 2 + c;
          if (col >= d) continue;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int q = tq[t0 + t][4 * kk + v];
            if (q >= 0) out[(int64_t)order[q] * d + col] = acc64[t][c][v];
          }
        }
      }
    }
  }
}

// j_hi ranges of pass B: enough workgroups to fill the chip at large N2, one range for small N2.
static int srht_js(int64_t N2) {
  const int64_t js = N2 / 512;
  return (int)(js < 1 ? 1 : (js > 8 ? 8 : js));
}
static int srht_js_cap(int64_t N2) { return srht_js(N2); }

constexpr int SRHT_LROWS = 256;                 // rows of a bucket per tile build
constexpr int SRHT_LMAXT = SRHT_LROWS / 16 + 8; // tiles per build at most (up to 8 fold groups)

// Row tiles of one chunk [cb, ce) of a bucket's selected rows (ce - cb <= SRHT_LROWS), grouped by
// e = k_hi mod F (F = 2^FB, the width of the fold) in tiles of 16 (the order of rows inside a tile does not
// change any output row; empty slots stay -1): one thread per row places itself with an LDS counter per
// group.  All threads of the workgroup call it; returns the tile count.
template <int MAXT>
struct SrhtTilesT {
  static constexpr int LMAXT = MAXT;
  int tq[MAXT][16];        // order[] positions of the tile's rows (-1: empty)
  uint32_t tka[MAXT][16];  // k_a = k_hi >> FB of each row
  int te[MAXT];            // e of the tile
  int cnt[16], tbase[16], nt;
};
typedef SrhtTilesT<SRHT_LMAXT> SrhtTiles;

template <int FB, typename TS>
__device__ __forceinline__ int srht_tile_build(TS& S, int cb, int ce, const int64_t* __restrict__ rows,
                                               const int* __restrict__ order, int L1) {
  constexpr int F = 1 << FB;
  static_assert(F <= 16, "fold width");
  const int tid = threadIdx.x;
  __syncthreads();  // the previous chunk's tiles are no longer read
  for (int i = tid; i < TS::LMAXT * 16; i += blockDim.x) S.tq[i / 16][i % 16] = -1;
  if (tid < F) S.cnt[tid] = 0;
  __syncthreads();
  int e_me = 0, slot_me = 0;
  uint32_t khi_me = 0;
  if (tid < ce - cb) {
    khi_me = (uint32_t)((uint64_t)rows[order[cb + tid]] >> L1);
    e_me = (int)(khi_me & (F - 1));
    slot_me = atomicAdd(&S.cnt[e_me], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int nt = 0;
    for (int e = 0; e < F; ++e) {
      S.tbase[e] = nt;
      const int k = (S.cnt[e] + 15) / 16;
      for (int t = 0; t < k; ++t) S.te[nt + t] = e;
      nt += k;
    }
    S.nt = nt;
  }
  __syncthreads();
  if (tid < ce - cb) {
    const int t = S.tbase[e_me] + slot_me / 16;
    S.tq[t][slot_me % 16] = cb + tid;
    S.tka[t][slot_me % 16] = khi_me >> FB;
  }
  __syncthreads();
  return S.nt;
}

// Pass B over large buckets, staged through LDS with the fold by the F-point transform (F = 2^FB, 4 or
// 8) done once per staged element: the thread that loads rows F j_a + b (b < F) of a column forms
// U_e = sum_b (-1)^{popcount(e & b)} T[F j_a + b] for every e < F with one in-place butterfly and stores
// them.  A tile's rows share e = k_hi mod F, and (-1)^{k_hi . j_hi} = (-1)^{k_a . j_a} (-1)^{e . b} with
// k_hi = F k_a + e, j_hi = F j_a + b, so a row's value is sum_{j_a} (-1)^{k_a . j_a} U_e[j_a]: N2 / F MFMA
// terms instead of N2.  A wavefront reads its tile's U_e directly, one LDS read per MFMA step.  The
// wider fold takes fewer MFMA terms per row but splits a bucket into more, emptier tiles (F groups of
// tiles of 16); F = 8 pays once groups average about 10 rows or more.
//   Workgroup: bucket k_lo, a j_hi range, 64 columns, NW wavefronts; wavefront w owns tile w (then
// w + NW, ... in later sweeps when a chunk has more than NW tiles) over all 64 columns, as four
// 16-column MFMA blocks interleaved so that a lane's B operands are adjacent in LDS (FP32: block cb,
// lane column qi is column 4 qi + cb).  With NW = 16 one sweep carries every tile of a typical bucket, so
// the bucket's T block is read from HBM once.
//   Stages of JA values of j_a (F JA rows of T) x 64 columns are loaded two stages ahead into registers,
// written as U_e[j_a][column] to a double buffer in LDS, and consumed JA / 4 MFMA steps per stage.
// FP32 T: FP32 chains of 32 values of j_a (at most 31 + FB roundings per term) folded into FP64, within
// the (log2 N + 2) 2u of an FP32 SRHT since N >= 2^17 on this path.  FP64 T: FP64 MFMA, no fold.
template <typename TC, int FB>
struct SrhtU;
template <>
struct SrhtU<float, 2> {
  static constexpr int JA = 32;  // j_a per stage
  static constexpr int VU = 2;   // columns per staging unit (one 8-byte load per row)
  typedef float vu_t __attribute__((ext_vector_type(2)));
};
template <>
struct SrhtU<float, 3> {
  static constexpr int JA = 16;
  static constexpr int VU = 1;
  typedef float vu_t;
};
template <>
struct SrhtU<double, 2> {
  static constexpr int JA = 16;
  static constexpr int VU = 1;
  typedef double vu_t;
};
template <>
struct SrhtU<double, 3> {
  static constexpr int JA = 16;  // 64 KB per stage buffer: one workgroup per CU
  static constexpr int VU = 1;
  typedef double vu_t;
};
// column of MFMA block c at lane column qi.  FP32: a lane's four columns adjacent (one 16-byte LDS read);
// FP64: columns 2 qi, 2 qi + 1 (blocks 0, 1) and 32 + 2 qi, 33 + 2 qi (blocks 2, 3), two 16-byte LDS
// reads, each contiguous over the 16 lanes of a j_a.
template <typename TC>
__device__ __forceinline__ int srht_ucol(int qi, int c) {
  return sizeof(TC) == 4 ? 4 * qi + c : 32 * (c >> 1) + 2 * qi + (c & 1);
}

template <typename TC, int NW, int FB>
__global__ __launch_bounds__(64 * NW, 1) void k_srht_passB_u(const TC* __restrict__ T, int64_t N2, int64_t d,
                                                           int64_t dT, int L1, const int64_t* __restrict__ rows,
                                                           const int* __restrict__ slot,
                                                           const int* __restrict__ order,
                                                           const int* __restrict__ bstart, int64_t m,
                                                           double* __restrict__ partial) {
  constexpr int F = 1 << FB;
  constexpr int JA = SrhtU<TC, FB>::JA, VU = SrhtU<TC, FB>::VU;
  constexpr int STAGE = F * JA * 64;            // elements per LDS stage buffer: U_e[j_a][64 columns]
  constexpr int UNITS = JA * (64 / VU);         // staging units (j_a, column group) per stage
  constexpr bool PART = UNITS < 64 * NW;        // only threads tid < UNITS stage (whole wavefronts)
  constexpr int UPT = PART ? 1 : UNITS / (64 * NW);  // units per staging thread
  constexpr int NSTEP = JA / 4;                 // MFMA steps per stage
  constexpr int FOLD = 32 / JA;                 // stages per FP32 chain (32 values of j_a)
  static_assert(PART ? UNITS % 64 == 0 : UNITS % (64 * NW) == 0, "staging map");
  static_assert(sizeof(TC) == 8 || FOLD == 1 || FOLD == 2, "chain length");
  typedef typename SrhtU<TC, FB>::vu_t vu_t;
  __shared__ __attribute__((aligned(16))) TC L[2 * STAGE];
  __shared__ SrhtTiles S;
  // column block fastest in the grid: workgroups that run together read whole rows of T
  const int klo = blockIdx.z;
  const int sl = slot[klo];
  if (sl < 0) return;
  const int js = blockIdx.y, JS = gridDim.y;
  const int64_t jh0 = N2 * js / JS, jh1 = N2 * (js + 1) / JS;  // multiples of 2 F JA
  const uint32_t ja0 = (uint32_t)(jh0 >> FB);
  const int nst = (int)((jh1 - jh0) / (F * JA));                 // even
  const int b0 = bstart[klo], b1 = bstart[klo + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int qi = lane & 15, kk = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  double* out = partial + (int64_t)js * m * d;
  // staging map: unit tid + 64 NW i -> j_a group uq (rows F uq + b of the stage), columns uc .. uc + VU - 1
  // of the workgroup's 64-column stripe of T (columns past d hold no data and are never output)
  const bool stager = !PART || tid < UNITS;  // uniform per wavefront
  const TC* gsrc[UPT];
  int lofs[UPT];
#pragma unroll
  for (int i = 0; i < UPT; ++i) {
    const int u = stager ? tid + 64 * NW * i : 0;
    const int uq = u / (64 / VU), uc = (u % (64 / VU)) * VU;
    gsrc[i] = T + (((int64_t)sl * gridDim.x + blockIdx.x) * N2 + jh0 + F * uq) * 64 + uc;
    lofs[i] = uq * 64 + uc;
  }
  auto gload = [&](int st, vu_t(&v)[UPT][F]) {
    if (!stager) return;
#pragma unroll
    for (int i = 0; i < UPT; ++i)
#pragma unroll
      for (int b = 0; b < F; ++b)
        v[i][b] = __builtin_nontemporal_load((const vu_t*)(gsrc[i] + ((int64_t)(F * JA) * st + b) * 64));
  };
  auto lstore = [&](int buf, const vu_t(&v)[UPT][F]) {
    if (!stager) return;
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      vu_t x[F];
#pragma unroll
      for (int b = 0; b < F; ++b) x[b] = v[i][b];
      // in-place butterfly: afterwards x[e] = U_e (natural order)
#pragma unroll
      for (int h = 1; h < F; h <<= 1)
#pragma unroll
        for (int b = 0; b < F; ++b)
          if ((b & h) == 0) {
            const vu_t p = x[b], q = x[b + h];
            x[b] = p + q;
            x[b + h] = p - q;
          }
      TC* w = L + buf * STAGE + lofs[i];
#pragma unroll
      for (int e = 0; e < F; ++e) *(vu_t*)(w + e * JA * 64) = x[e];
    }
  };
  for (int cb = b0; cb < b1; cb += SRHT_LROWS) {
    const int nt =
        __builtin_amdgcn_readfirstlane(srht_tile_build<FB>(S, cb, min(b1, cb + SRHT_LROWS), rows, order, L1));
    for (int tg = 0; tg < nt; tg += NW) {
      const int t = tg + wv;
      const bool has = t < nt;  // uniform per wavefront
      const int q = has ? S.tq[t][qi] : -1;
      const TC pos = q >= 0 ? (TC)1 : (TC)0;
      const uint32_t ka = q >= 0 ? S.tka[t][qi] : 0u;
      const int e = has ? S.te[t] : 0;
      // (-1)^{k_a . j_a} with j_a = ja_stage + 4 s + kk, ja_stage a multiple of JA: the parity splits into
      // that of k_a & ja_stage (once per stage) and that of k_a & (4 s + kk) (bit s of lowpar)
      uint32_t lowpar = 0u;
#pragma unroll
      for (int s = 0; s < NSTEP; ++s) lowpar |= (uint32_t)(__popc(ka & (uint32_t)(4 * s + kk)) & 1) << s;
      constexpr uint32_t ALL = (1u << NSTEP) - 1u;
      const int rofs = (e * JA + kk) * 64 + srht_ucol<TC>(qi, 0);
      typedef float f4 __attribute__((ext_vector_type(4)));
      typedef double d2 __attribute__((ext_vector_type(2)));
      lsq_f4v acc[4];
      lsq_d4 acc64[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[c] = (lsq_f4v){0.f, 0.f, 0.f, 0.f};
        acc64[c] = (lsq_d4){0.0, 0.0, 0.0, 0.0};
      }
      // one stage from LDS buffer Lb; fold: the FP32 chains end here
      auto compute = [&](const TC* Lb, uint32_t ja_stage, bool fold) {
        if (!has) return;
        const uint32_t sb = lowpar ^ ((__popc(ka & ja_stage) & 1) ? ALL : 0u);
        const TC* r = Lb + rofs;
        if constexpr (sizeof(TC) == 4) {
          // each step's LDS read is issued before the previous step's MFMAs
          f4 un = *(const f4*)r;
#pragma unroll
          for (int s = 0; s < NSTEP; ++s) {
            const f4 u = un;
            if (s + 1 < NSTEP) un = *(const f4*)(r + 4 * (s + 1) * 64);
            const float a = ((sb >> s) & 1u) ? -pos : pos;
            acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u.x, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u.y, acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u.z, acc[2], 0, 0, 0);
            acc[3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u.w, acc[3], 0, 0, 0);
          }
          if (fold) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
#pragma unroll
              for (int v = 0; v < 4; ++v) acc64[c][v] += (double)acc[c][v];
              acc[c] = (lsq_f4v){0.f, 0.f, 0.f, 0.f};
            }
          }
        } else {
          d2 un0 = *(const d2*)r, un1 = *(const d2*)(r + 32);
#pragma unroll
          for (int s = 0; s < NSTEP; ++s) {
            const d2 u0 = un0, u1 = un1;
            if (s + 1 < NSTEP) {
              un0 = *(const d2*)(r + 4 * (s + 1) * 64);
              un1 = *(const d2*)(r + 4 * (s + 1) * 64 + 32);
            }
            const double a = ((sb >> s) & 1u) ? -pos : pos;
            acc64[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, u0.x, acc64[0], 0, 0, 0);
            acc64[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, u0.y, acc64[1], 0, 0, 0);
            acc64[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, u1.x, acc64[2], 0, 0, 0);
            acc64[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, u1.y, acc64[3], 0, 0, 0);
          }
        }
      };
      // two stages in flight in registers, one being consumed from LDS.  nst is even; loads are issued
      // without conditions (stages past the last reload the last one, never used) so that the compiler's
      // wait counts stay exact and two stages stay in flight.
      vu_t ra[UPT][F], rb[UPT][F];
      gload(0, ra);
      gload(1, rb);
      lds_barrier();  // the previous sweep's last stage has been consumed
      lstore(0, ra);
      lds_barrier();
      gload(min(2, nst - 1), ra);
      for (int st = 0; st < nst; st += 2) {
        compute(L, ja0 + JA * st, FOLD == 1);
        lstore(1, rb);
        lds_barrier();
        gload(min(st + 3, nst - 1), rb);
        compute(L + STAGE, ja0 + JA * (st + 1), true);
        lstore(0, ra);
        lds_barrier();
        gload(min(st + 4, nst - 1), ra);
      }
      if (has) {
        // result lane l, register v: tile row 4 (l / 16) + v (FP32 MFMA) or l / 16 + 4 v (FP64 MFMA)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int qq = S.tq[t][sizeof(TC) == 4 ? 4 * kk + v : kk + 4 * v];
          if (qq < 0) continue;
          double* o = out + (int64_t)order[qq] * d;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int64_t col = c0 + srht_ucol<TC>(qi, c);
            if (col < d) o[col] = acc64[c][v];
          }
        }
      }
    }
  }
}

// Pass B over large buckets with the intermediate streamed into LDS by the memory system itself
// (global_load_lds, 16 bytes per lane; no staging registers) and folded there in place.  A stage is
// SR = F JA consecutive rows j_hi of the bucket's 64-column stripe of T (16 KB, or 32 KB for the FP64
// 16-point fold; one contiguous range of the stripe layout), and NBUF = 128 KB / stage buffers rotate:
// while the matrix cores consume stage s, stage s + 1 is folded in place and stages s + 2 .. s + NBUF - 1
// are in flight (96 KB per CU with 16 KB stages, enough to cover the memory latency at this CU's share
// of the bandwidth), so each wave waits (vmcnt) only for its own loads of stage s + 1 before the one
// barrier per stage.  In place: the rows of stage buffer position (j_a, b) = row F j_a + b, column c,
// become U_e[j_a] at position (j_a, e), the thread of unit (j_a, c) reading its F values, transforming
// and writing them back.
//   Eight wavefronts (two per SIMD, up to 256 registers each) carry up to QT tiles of 16 rows each, so one
// sweep over the bucket's T block serves up to 8 QT tiles: with the 16-point fold, about 16 + (rows - 256)
// / 16 tiles once a bucket passes 256 selected rows, which keeps sketches of m up to about 2^17 at one
// read of T.  The tile of wavefront w, slot q is tile tg + w + 8 q of the chunk's list.  Signs, operand
// layouts, chain lengths and the FP64 folding of the FP32 chains are those of k_srht_passB_u.
constexpr int SRHT2_NW = 8;
constexpr int SRHT2_LDS = 131072;                       // bytes of stage buffers
constexpr int SRHT2_LROWS = 64 * SRHT2_NW;              // rows of a bucket per tile build (one thread each)
typedef SrhtTilesT<SRHT2_LROWS / 16 + 16> SrhtTiles2;   // up to 16 fold groups

template <typename TC, int FB>
struct Srht2Shape {
  static constexpr int STG = 32768;  // bytes per stage
  static constexpr int NBUF = SRHT2_LDS / STG;
};

__device__ __forceinline__ void srht_dma16(const void* src, void* lds) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

// vmcnt(k IPT) for a runtime k in [0, KMAX] (the waitcnt operand is an immediate)
template <int IPT, int KMAX>
__device__ __forceinline__ void srht_vm_wait_stages(int k) {
  if constexpr (KMAX <= 0) {
    vm_wait<0>();
  } else {
    if (k >= KMAX)
      vm_wait<KMAX * IPT>();
    else
      srht_vm_wait_stages<IPT, KMAX - 1>(k);
  }
}

// Per-wavefront state of up to QT row tiles (lane qi: row qi of each tile).
template <typename TC, int QT>
struct Srht2Tiles {
  TC pos[QT];
  uint32_t ka[QT], lowpar[QT];
  int rofs[QT];
  lsq_f4v acc[QT][4];
  lsq_d4 acc64[QT][4];
};

// One stage of the streamed pass B for a wavefront holding K tiles: the matrix-core sums of stage buffer
// Lc interleaved with the in-place fold of stage buffer Lf (when fold_next).  The fold's LDS reads,
// butterflies and writes are independent of the MFMAs, so the scheduler is asked to alternate them.
template <typename TC, int FB, int QT, int K, int JA, int UPT, int UNITS>
__device__ __forceinline__ void srht2_stage(Srht2Tiles<TC, QT>& W, const TC* Lc, TC* Lf, bool fold_next,
                                           uint32_t ja_stage, bool chain_end, int tid) {
  constexpr int F = 1 << FB;
  constexpr int NT = 64 * SRHT2_NW;
  constexpr int NSTEP = JA / 4;
  constexpr uint32_t ALL = (1u << NSTEP) - 1u;
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  // Every access to the stage buffers goes through the asm statements of internal.h: the buffers are
  // filled by global-to-LDS loads, and an ordinary LDS access would make the compiler wait for all of
  // them (the ones issued ahead for later stages included).  The caller's vm_wait and barrier order
  // these accesses after the loads they need.
  typedef typename std::conditional<sizeof(TC) == 4, lds_u2, lds_q2>::type V2;
  typedef typename std::conditional<sizeof(TC) == 4, uint32_t, uint64_t>::type UB;
  // fold operands first
  TC x[UPT][F];
  uint32_t pf[UPT];
  // (the last stage folds the buffer after it too: stale or unused data that nothing reads, so that the
  // fold needs no branch around it when every thread has a unit)
  const bool fa = UNITS >= NT || (fold_next && tid < UNITS);
#pragma unroll
  for (int i = 0; i < UPT; ++i) {
    const int u = tid + NT * i;
    pf[i] = (uint32_t)(uintptr_t)(Lf + (u >> 6) * F * 64 + (u & 63));
    if (fa) {
      V2 x2[F / 2];
      if constexpr (F == 16) lds_read16_st64<V2>(pf[i], x2);
      else lds_read8_st64<V2>(pf[i], x2);
#pragma unroll
      for (int b = 0; b < F / 2; ++b) {
        x[i][2 * b] = __builtin_bit_cast(TC, (UB)x2[b][0]);
        x[i][2 * b + 1] = __builtin_bit_cast(TC, (UB)x2[b][1]);
      }
    }
  }
  static_assert(F == 8 || F == 16, "fold widths of the streamed form");
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const uint32_t sb = W.lowpar[q] ^ ((__popc(W.ka[q] & ja_stage) & 1) ? ALL : 0u);
    const uint32_t r = (uint32_t)(uintptr_t)(Lc + W.rofs[q]);
    // the tile's operands of the stage: NSTEP 16-byte reads (FP32) or 2 NSTEP (FP64)
    int4 v[4];
    if constexpr (sizeof(TC) == 4) {
      if constexpr (NSTEP == 2) lds_read2_b128_at<0, 4 * F * 64 * 4>(r, v[0], v[1]);
      else lds_read4_b128_at<0, 4 * F * 64 * 4, 8 * F * 64 * 4, 12 * F * 64 * 4>(r, v[0], v[1], v[2], v[3]);
    } else {
      if constexpr (NSTEP == 1) lds_read2_b128_at<0, 256>(r, v[0], v[1]);
      else lds_read4_b128_at<0, 256, 4 * F * 64 * 8, 4 * F * 64 * 8 + 256>(r, v[0], v[1], v[2], v[3]);
    }
    static_assert(sizeof(TC) == 4 ? (NSTEP == 2 || NSTEP == 4) : (NSTEP == 1 || NSTEP == 2), "stage steps");
#pragma unroll
    for (int s2 = 0; s2 < NSTEP; ++s2) {
      const TC a = ((sb >> s2) & 1u) ? -W.pos[q] : W.pos[q];
      if constexpr (sizeof(TC) == 4) {
        const f4 u = __builtin_bit_cast(f4, v[s2]);
        W.acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u.x, W.acc[q][0], 0, 0, 0);
        W.acc[q][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u.y, W.acc[q][1], 0, 0, 0);
        W.acc[q][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u.z, W.acc[q][2], 0, 0, 0);
        W.acc[q][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, u.w, W.acc[q][3], 0, 0, 0);
      } else {
        const d2 u0 = __builtin_bit_cast(d2, v[2 * s2]), u1 = __builtin_bit_cast(d2, v[2 * s2 + 1]);
        W.acc64[q][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, u0.x, W.acc64[q][0], 0, 0, 0);
        W.acc64[q][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, u0.y, W.acc64[q][1], 0, 0, 0);
        W.acc64[q][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, u1.x, W.acc64[q][2], 0, 0, 0);
        W.acc64[q][3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, u1.y, W.acc64[q][3], 0, 0, 0);
      }
    }
  }
  if (fa) {
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
#pragma unroll
      for (int h = 1; h < F; h <<= 1)
#pragma unroll
        for (int b = 0; b < F; ++b)
          if ((b & h) == 0) {
            const TC a = x[i][b], c = x[i][b + h];
            x[i][b] = a + c;
            x[i][b + h] = a - c;
          }
      auto wr = [&](auto kc) {
        constexpr int k = decltype(kc)::value;
        lds_write2_st64<k>(pf[i], __builtin_bit_cast(UB, x[i][2 * k]), __builtin_bit_cast(UB, x[i][2 * k + 1]));
      };
      wr(std::integral_constant<int, 0>());
      wr(std::integral_constant<int, 1>());
      wr(std::integral_constant<int, 2>());
      wr(std::integral_constant<int, 3>());
      if constexpr (F == 16) {
        wr(std::integral_constant<int, 4>());
        wr(std::integral_constant<int, 5>());
        wr(std::integral_constant<int, 6>());
        wr(std::integral_constant<int, 7>());
      }
    }
  }
  if constexpr (sizeof(TC) == 4) {
    // the FP32 chains end every 32 values of j_a, and at the last stage
    if (chain_end) {
#pragma unroll
      for (int q = 0; q < K; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
          for (int v = 0; v < 4; ++v) W.acc64[q][c][v] += (double)W.acc[q][c][v];
          W.acc[q][c] = (lsq_f4v){0.f, 0.f, 0.f, 0.f};
        }
    }
  }
}

template <typename TC, int FB, int QT>
__global__ __launch_bounds__(64 * SRHT2_NW, 1) void k_srht_passB_v2(
    const TC* __restrict__ T, int64_t N2, int64_t d, int64_t dT, int L1, const int64_t* __restrict__ rows,
    const int* __restrict__ slot, const int* __restrict__ order, const int* __restrict__ bstart, int64_t m,
    double* __restrict__ partial) {
  constexpr int F = 1 << FB;
  constexpr int NT = 64 * SRHT2_NW;
  constexpr int STG = Srht2Shape<TC, FB>::STG, NBUF = Srht2Shape<TC, FB>::NBUF;
  constexpr int SR = STG / (64 * (int)sizeof(TC));         // rows of T per stage
  constexpr int JA = SR / F;                               // values of j_a per stage
  constexpr int NSTEP = JA / 4;                            // MFMA steps per stage
  constexpr int IPT = STG / (NT * 16);                     // 16-byte loads per thread per stage
  constexpr int STE = STG / (int)sizeof(TC);               // elements per stage
  constexpr int UNITS = JA * 64;                           // fold units (j_a, column) per stage
  constexpr int UPT = UNITS > NT ? UNITS / NT : 1;
  constexpr int CHAINS = sizeof(TC) == 4 ? 32 / JA : 1;    // stages per FP32 chain (32 values of j_a)
  static_assert(NSTEP >= 1 && JA % 4 == 0, "stage shape");
  static_assert(IPT >= 1 && IPT * NT * 16 == STG, "stage loads");
  static_assert(NBUF >= 4 && NBUF * STG == SRHT2_LDS, "stage buffers");
  static_assert(UNITS <= NT || UNITS % NT == 0, "fold map");
  static_assert(sizeof(TC) == 8 || (JA <= 32 && 32 % JA == 0), "chain length");
  __shared__ __attribute__((aligned(16))) TC L[NBUF * STE];
  __shared__ SrhtTiles2 S;
  const int klo = blockIdx.z;
  const int sl = slot[klo];
  if (sl < 0) return;
  const int js = blockIdx.y, JS = gridDim.y;
  const int64_t jh0 = N2 * js / JS, jh1 = N2 * (js + 1) / JS;  // multiples of SR
  const uint32_t ja0 = (uint32_t)(jh0 >> FB);
  const int nst = (int)((jh1 - jh0) / SR);
  const int b0 = bstart[klo], b1 = bstart[klo + 1];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int qi = lane & 15, kk = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  double* out = partial + (int64_t)js * m * d;
  // the workgroup's stages, one contiguous range each
  const TC* gbase = T + (((int64_t)sl * gridDim.x + blockIdx.x) * N2 + jh0) * 64;
  auto issue = [&](int st) {
    const char* g = (const char*)(gbase + (int64_t)st * STE);
    char* l = (char*)(L + (st % NBUF) * STE);
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const int c = k * SRHT2_NW + wv;  // 1 KB chunk of the stage
      srht_dma16(g + c * 1024 + lane * 16, l + c * 1024);
    }
  };
  for (int cb = b0; cb < b1; cb += SRHT2_LROWS) {
    const int nt = __builtin_amdgcn_readfirstlane(
        srht_tile_build<FB>(S, cb, min(b1, cb + SRHT2_LROWS), rows, order, L1));
    for (int tg = 0; tg < nt; tg += SRHT2_NW * QT) {
      // this wavefront's tiles: tg + wv + 8 q for q < nq
      const int nq = __builtin_amdgcn_readfirstlane(max(0, min(QT, (nt - tg - wv + SRHT2_NW - 1) / SRHT2_NW)));
      Srht2Tiles<TC, QT> W;
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        const int t = tg + wv + SRHT2_NW * q;
        const int qq = q < nq ? S.tq[t][qi] : -1;
        W.pos[q] = qq >= 0 ? (TC)1 : (TC)0;
        W.ka[q] = qq >= 0 ? S.tka[t][qi] : 0u;
        const int e = q < nq ? S.te[t] : 0;
        W.lowpar[q] = 0u;
#pragma unroll
        for (int st = 0; st < NSTEP; ++st)
          W.lowpar[q] |= (uint32_t)(__popc(W.ka[q] & (uint32_t)(4 * st + kk)) & 1) << st;
        W.rofs[q] = (kk * F + e) * 64 + srht_ucol<TC>(qi, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          W.acc[q][c] = (lsq_f4v){0.f, 0.f, 0.f, 0.f};
          W.acc64[q][c] = (lsq_d4){0.0, 0.0, 0.0, 0.0};
        }
      }
      // One sweep: stage st from buffer st % NBUF, interleaved with the fold of stage st + 1 (if any), for a
      // wavefront of KC tiles (a compile-time count, so that each count has its own straight-line body).
      auto sweep = [&](auto kc) {
        constexpr int KC = decltype(kc)::value;
        // Prologue: stages 0 .. NBUF - 2 in flight, stage 0 folded (a stage call with no tiles).  The counts
        // of the waits are of this wave's stage loads alone: the previous sweep's result stores are drained
        // first.
        vm_wait<0>();
        lds_barrier();  // the previous sweep no longer reads the buffers
        const int npro = min(nst, NBUF - 1);
        for (int st = 0; st < npro; ++st) issue(st);
        srht_vm_wait_stages<IPT, NBUF - 2>(npro - 1);  // stage 0 landed
        lds_barrier();
        srht2_stage<TC, FB, QT, 0, JA, UPT, UNITS>(W, L, L, true, 0u, false, tid);  // fold of stage 0
        for (int st = 0; st < nst; ++st) {
          // this wave's loads of stage st + 1 have landed; stages st + 2 .. min(nst, st + NBUF - 1) - 1 may
          // still be in flight
          srht_vm_wait_stages<IPT, NBUF - 3>(max(0, min(nst, st + NBUF - 1) - (st + 2)));
          lds_barrier();  // every wave's loads of st + 1, the fold of st, the compute of st - 1: done
          if (st + NBUF - 1 < nst) issue(st + NBUF - 1);  // into the buffer of stage st - 1
          const uint32_t ja_stage = ja0 + (uint32_t)(JA * st);
          const bool ce = (st + 1) % CHAINS == 0 || st + 1 == nst;
          srht2_stage<TC, FB, QT, KC, JA, UPT, UNITS>(W, L + (st % NBUF) * STE, L + ((st + 1) % NBUF) * STE,
                                                     st + 1 < nst, ja_stage, ce, tid);
        }
      };
      switch (nq) {
        case 0: sweep(std::integral_constant<int, 0>()); break;
        case 1: sweep(std::integral_constant<int, (1 < QT ? 1 : QT)>()); break;
        case 2: sweep(std::integral_constant<int, (2 < QT ? 2 : QT)>()); break;
        case 3: sweep(std::integral_constant<int, (3 < QT ? 3 : QT)>()); break;
        default: sweep(std::integral_constant<int, QT>()); break;
      }
#pragma unroll
      for (int q = 0; q < QT; ++q) {
        if (q >= nq) continue;
        const int t = tg + wv + SRHT2_NW * q;
        // result lane l, register v: tile row 4 (l / 16) + v (FP32 MFMA) or l / 16 + 4 v (FP64 MFMA)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int qq = S.tq[t][sizeof(TC) == 4 ? 4 * kk + v : kk + 4 * v];
          if (qq < 0) continue;
          double* o = out + (int64_t)order[qq] * d;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int64_t col = c0 + srht_ucol<TC>(qi, c);
            if (col < d) o[col] = W.acc64[q][c][v];
          }
        }
      }
    }
  }
}

// j_hi ranges of the LDS-staged pass B: about g_srht_passb_wgs (8192) workgroups in all, at most the
// partial buffer's ranges, at least two stages (256 rows of T for FP32, 128 for FP64) per range.
static int srht_js_lds(int64_t N1, int64_t N2, int64_t ncb) {
  int js = 1;
  while (js < 8 && N1 * ncb * js < g_srht_passb_wgs && N2 / (2 * js) >= 256 && 2 * js <= srht_js_cap(N2)) js *= 2;
  return js;
}

__global__ void k_srht_final(const double* __restrict__ partial, int JS, int64_t m, int64_t d,
                             double scale, double* __restrict__ SA, int64_t ldsa) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * d) return;
  double s = 0.0;
  for (int k = 0; k < JS; ++k) s += partial[(int64_t)k * m * d + idx];
  SA[(idx / d) * ldsa + idx % d] = s * scale;
}


size_t srht_partial_bytes(int64_t N2, int64_t m, int64_t d) {
  return (size_t)srht_js(N2) * (size_t)m * (size_t)d * sizeof(double);
}

template <typename TA, typename TC>
static void srht_apply_t(hipStream_t st, const TA* A, int64_t n, int64_t d, int64_t lda,
                         const SrhtPlan& p, const int8_t* signs, const int64_t* rows,
                         const int* slot, const int* order, const int* bstart, TC* T,
                         double* partial, double* SA, int64_t ldsa, const double* y, double* gpart,
                         bool* grad_done) {
  constexpr int VW = 16 / sizeof(TC);
  *grad_done = false;
  const int64_t dT = srht_dT(d, sizeof(TC) == 4);
  int L1 = 0;
  while ((1ll << L1) < p.N1) ++L1;
  // buckets of more than about 24 selected rows on average: 64-row chunks (one sweep of T per bucket)
  const bool big = p.m > 24 * p.N1;
  // the LDS-staged pass B reads T in 64-column stripes, written so by pass A
  const bool lds_b = p.N1 == SRHT_N1 && big && p.N2 >= 512 && p.passb != 1;
  const int64_t ncbs = lds_b ? (dT + 63) / 64 : 0;
  if (p.N1 == SRHT_N1) {
    const bool vec = d % VW == 0 && lda % VW == 0 && ((uintptr_t)A % (VW * sizeof(TA))) == 0;
    if (vec) {
      // slice groups: about 2^17 (FP32 T) or 2^15 (FP64 T) workgroups in all, measured best on gfx950
      constexpr int64_t DC = 16 * VW;
      const int64_t nslices = (d + DC - 1) / DC;
      const int64_t target = g_srht_passa_wgs > 0 ? g_srht_passa_wgs : (sizeof(TC) == 4 ? (1 << 17) : (1 << 15));
      int64_t sg = (target + p.N2 - 1) / p.N2;
      sg = sg > nslices ? nslices : (sg < 1 ? 1 : sg);
      // (the gradient needs A's values exactly: not with an FP32 transform of FP64 A)
      if (gpart && sizeof(TC) >= sizeof(TA)) {
        hipLaunchKernelGGL((k_srht_passA_vec<TA, TC, true>), dim3((unsigned)p.N2, (unsigned)sg), dim3(256), 0, st,
                           A, n, d, lda, signs, slot, p.N2, dT, ncbs, T, y, gpart);
        *grad_done = true;
      } else {
        hipLaunchKernelGGL((k_srht_passA_vec<TA, TC, false>), dim3((unsigned)p.N2, (unsigned)sg), dim3(256), 0, st,
                           A, n, d, lda, signs, slot, p.N2, dT, ncbs, T, nullptr, nullptr);
      }
    } else {
      constexpr int64_t DC = 128 / sizeof(TC);
      const int64_t nslices = (d + DC - 1) / DC;
      int64_t sg = (4096 + p.N2 - 1) / p.N2;
      sg = sg > nslices ? nslices : (sg < 1 ? 1 : sg);
      hipLaunchKernelGGL((k_srht_passA2<TA, TC>), dim3((unsigned)p.N2, (unsigned)sg), dim3(256), 0, st, A, n,
                         d, lda, signs, slot, p.N2, dT, ncbs, T);
    }
  } else {
    constexpr int64_t DC = 128 / sizeof(TC);
    const int64_t nslices = (d + DC - 1) / DC;
    hipLaunchKernelGGL((k_srht_passA<TA, TC>), dim3((unsigned)p.N2, (unsigned)nslices), dim3(256), 0, st, A,
                       n, d, lda, (int)p.N1, signs, slot, p.N2, dT, T);
  }
  int JS = srht_js(p.N2);
  if constexpr (sizeof(TC) == 4) {
    const int64_t wgc = big ? 128 : 256;  // 64 VW columns per workgroup
    dim3 gb((unsigned)p.N1, (unsigned)JS, (unsigned)((dT + wgc - 1) / wgc));
    if (lds_b) {
      const int64_t ncb = ncbs;
      JS = srht_js_lds(p.N1, p.N2, ncb);
      dim3 gl((unsigned)ncb, (unsigned)JS, (unsigned)p.N1);
      // Sixteen wavefronts of one tile each (register-staged), one sweep over T for up to 16 tiles, the
      // 8-point fold from 64 rows per bucket on average (measured at n = 2^22, d = 1024: sketches 3-8 %
      // faster from 64 to 256 rows, where its tiles take half the MFMA terms); from 192 rows (more than 16
      // tiles: a second sweep) the streamed form with up to 32 tiles per sweep and the 16-point fold
      // (12.2 against 15.4 ms at m = 65536).  Options: 2 eight wavefronts, 4-point; 3 sixteen, 4-point;
      // 4 sixteen, 8-point; 5 and 6 streamed, 8- and 16-point.
      const bool stream = p.passb >= 5 || (p.passb == 0 && p.m >= (int64_t)g_srht_stream_rows_f32 * p.N1);
      const bool f8 = p.passb == 4 || (p.passb == 0 && p.m >= (int64_t)g_srht_fold8_rows_f32 * p.N1);
      if (stream) {
        const bool f16 = p.passb != 5;
        if (f16)
          hipLaunchKernelGGL((k_srht_passB_v2<float, 4, 4>), gl, dim3(64 * SRHT2_NW), 0, st, (const float*)T, p.N2,
                             d, dT, L1, rows, slot, order, bstart, p.m, partial);
        else
          hipLaunchKernelGGL((k_srht_passB_v2<float, 3, 4>), gl, dim3(64 * SRHT2_NW), 0, st, (const float*)T, p.N2,
                             d, dT, L1, rows, slot, order, bstart, p.m, partial);
      } else if (p.passb == 2)
        hipLaunchKernelGGL((k_srht_passB_u<float, 8, 2>), gl, dim3(512), 0, st, (const float*)T, p.N2, d, dT, L1,
                           rows, slot, order, bstart, p.m, partial);
      else if (f8)
        hipLaunchKernelGGL((k_srht_passB_u<float, 16, 3>), gl, dim3(1024), 0, st, (const float*)T, p.N2, d, dT, L1,
                           rows, slot, order, bstart, p.m, partial);
      else
        hipLaunchKernelGGL((k_srht_passB_u<float, 16, 2>), gl, dim3(1024), 0, st, (const float*)T, p.N2, d, dT, L1,
                           rows, slot, order, bstart, p.m, partial);
    } else if (big && p.N2 >= 512)
      hipLaunchKernelGGL(k_srht_passB_f32w, gb, dim3(256), 0, st, (const float*)T, p.N2, d, dT, L1, rows, slot,
                         order, bstart, p.m, partial);
    else if (big)
      hipLaunchKernelGGL(k_srht_passB_f32<4>, gb, dim3(256), 0, st, (const float*)T, p.N2, d, dT, L1, rows, slot,
                         order, bstart, p.m, partial);
    else
      hipLaunchKernelGGL(k_srht_passB_f32<2>, gb, dim3(256), 0, st, (const float*)T, p.N2, d, dT, L1, rows, slot,
                         order, bstart, p.m, partial);
  } else if (lds_b) {
    const int64_t ncb = ncbs;
    JS = srht_js_lds(p.N1, p.N2, ncb);
    dim3 gl((unsigned)ncb, (unsigned)JS, (unsigned)p.N1);
    // as for FP32 T; the register-staged FP64 8-point form's 64 KB stages leave one workgroup per CU
    // (measured at n = 2^22, d = 1024: sketches 5-9 % faster from 128 to 256 rows per bucket, even at 96)
    const bool stream = p.passb >= 5 || (p.passb == 0 && p.m >= (int64_t)g_srht_stream_rows_f64 * p.N1);
    const bool f8 = p.passb == 4 || (p.passb == 0 && p.m >= (int64_t)g_srht_fold8_rows_f64 * p.N1);
    if (stream) {
      const bool f16 = p.passb != 5;
      if (f16)
        hipLaunchKernelGGL((k_srht_passB_v2<double, 4, 4>), gl, dim3(64 * SRHT2_NW), 0, st, (const double*)T, p.N2,
                           d, dT, L1, rows, slot, order, bstart, p.m, partial);
      else
        hipLaunchKernelGGL((k_srht_passB_v2<double, 3, 4>), gl, dim3(64 * SRHT2_NW), 0, st, (const double*)T, p.N2,
                           d, dT, L1, rows, slot, order, bstart, p.m, partial);
    } else if (p.passb == 2)
      hipLaunchKernelGGL((k_srht_passB_u<double, 8, 2>), gl, dim3(512), 0, st, (const double*)T, p.N2, d, dT, L1, rows,
                         slot, order, bstart, p.m, partial);
    else if (f8)
      hipLaunchKernelGGL((k_srht_passB_u<double, 16, 3>), gl, dim3(1024), 0, st, (const double*)T, p.N2, d, dT, L1,
                         rows, slot, order, bstart, p.m, partial);
    else
      hipLaunchKernelGGL((k_srht_passB_u<double, 16, 2>), gl, dim3(1024), 0, st, (const double*)T, p.N2, d, dT, L1,
                         rows, slot, order, bstart, p.m, partial);
  } else if (big) {
    constexpr int WGC = SRHT_WGC / 2;
    dim3 gb((unsigned)p.N1, (unsigned)JS, (unsigned)((dT + WGC - 1) / WGC));
    hipLaunchKernelGGL((k_srht_passB<TC, WGC, 4>), gb, dim3(256), 0, st, T, p.N2, d, dT, L1, rows, slot, order,
                       bstart, p.m, partial);
  } else {
    dim3 gb((unsigned)p.N1, (unsigned)JS, (unsigned)((dT + SRHT_WGC - 1) / SRHT_WGC));
    hipLaunchKernelGGL((k_srht_passB<TC, SRHT_WGC, 2>), gb, dim3(256), 0, st, T, p.N2, d, dT, L1, rows, slot, order,
                       bstart, p.m, partial);
  }
  hipLaunchKernelGGL(k_srht_final, dim3((unsigned)((p.m * d + 255) / 256)), dim3(256), 0, st, partial, JS,
                     p.m, d, 1.0 / sqrt((double)p.m), SA, ldsa);
}

bool srht_apply(hipStream_t st, const void* A, int a_f32, int64_t n, int64_t d, int64_t lda,
                int compute_f32, const SrhtPlan& plan, const int8_t* signs, const int64_t* rows,
                const int* slot, const int* order, const int* bstart, void* tbuf, double* partial,
                double* SA, int64_t ldsa, const double* y, double* gpart) {
  bool g = false;
  if (a_f32 && compute_f32)
    srht_apply_t<float, float>(st, (const float*)A, n, d, lda, plan, signs, rows, slot, order, bstart,
                               (float*)tbuf, partial, SA, ldsa, y, gpart, &g);
  else if (a_f32)
    srht_apply_t<float, double>(st, (const float*)A, n, d, lda, plan, signs, rows, slot, order,
                                bstart, (double*)tbuf, partial, SA, ldsa, y, gpart, &g);
  else if (compute_f32)
    srht_apply_t<double, float>(st, (const double*)A, n, d, lda, plan, signs, rows, slot, order,
                                bstart, (float*)tbuf, partial, SA, ldsa, y, gpart, &g);
  else
    srht_apply_t<double, double>(st, (const double*)A, n, d, lda, plan, signs, rows, slot, order,
                                 bstart, (double*)tbuf, partial, SA, ldsa, y, gpart, &g);
  return g;
}

// --------------------------------------------------------------------------------------------------
// SJLT: stable counting sort of (target, row, sign) by target, then per-target reduction.
// --------------------------------------------------------------------------------------------------
constexpr int SJLT_RB = 4096;  // rows of A per counting block
constexpr int SJLT_MMAX = 16384;

int64_t sjlt_nblk(int64_t n) { return (n + SJLT_RB - 1) / SJLT_RB; }

__global__ __launch_bounds__(256) void k_sjlt_count(const int32_t* __restrict__ targets, int64_t n,
                                                    int s, int m, int64_t nblk,
                                                    int* __restrict__ cnt) {
  __shared__ int hist[SJLT_MMAX];
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;
  for (int h = tid; h < m; h += 256) hist[h] = 0;
  __syncthreads();
  const int64_t q0 = b * SJLT_RB * s;
  const int64_t q1 = min(n * s, (b + 1) * SJLT_RB * (int64_t)s);
  for (int64_t q = q0 + tid; q < q1; q += 256) atomicAdd(&hist[targets[q]], 1);
  __syncthreads();
  for (int h = tid; h < m; h += 256) cnt[(int64_t)h * nblk + b] = hist[h];
}

// One wavefront per counting block: ranks equal targets in (row, k) order with ballots.
__global__ __launch_bounds__(64) void k_sjlt_scatter(const int32_t* __restrict__ targets,
                                                     const int8_t* __restrict__ signs, int64_t n,
                                                     int s, int m, int nbits, int64_t nblk,
                                                     const int* __restrict__ off,
                                                     uint32_t* __restrict__ sorted) {
  __shared__ int base[SJLT_MMAX];
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  for (int h = lane; h < m; h += 64) base[h] = off[(int64_t)h * nblk + b];
  __syncthreads();
  const int64_t q0 = b * SJLT_RB * s;
  const int64_t q1 = min(n * s, (b + 1) * SJLT_RB * (int64_t)s);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint64_t gt = (lane == 63) ? 0ull : (~0ull << (lane + 1));
  for (int64_t qb = q0; qb < q1; qb += 64) {
    const int64_t q = qb + lane;
    const bool act = q < q1;
    const int h = act ? targets[q] : 0;
    uint64_t same = __ballot(act);
    for (int bit = 0; bit < nbits; ++bit) {
      const bool on = (h >> bit) & 1;
      const uint64_t bal = __ballot(on);
      same &= on ? bal : ~bal;
    }
    int pos = 0;
    if (act) pos = base[h] + __popcll(same & lt);
    __syncthreads();
    if (act) {
      const int64_t row = q / s;
      sorted[pos] = ((uint32_t)row << 1) | (signs[q] < 0 ? 1u : 0u);
      if ((same & gt) == 0) base[h] = pos + 1;
    }
    __syncthreads();
  }
}

__global__ void k_sjlt_bstart(const int* __restrict__ off, int m, int64_t nblk, int64_t total,
                              int* __restrict__ bstart) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < m) bstart[h] = off[(int64_t)h * nblk];
  if (h == m) bstart[m] = (int)total;
}

template <typename TA, int NCOL>
__global__ __launch_bounds__(256) void k_sjlt_reduce(const TA* __restrict__ A, int64_t d,
                                                     int64_t lda, const uint32_t* __restrict__ sorted,
                                                     const int* __restrict__ bstart, double scale,
                                                     double* __restrict__ SA, int64_t ldsa) {
  const int h = blockIdx.x;
  const int tid = threadIdx.x;
  const int e0 = bstart[h], e1 = bstart[h + 1];
  double acc[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) acc[c] = 0.0;
  int e = e0;
  for (; e + 4 <= e1; e += 4) {
    uint32_t en[4];
    double v[4][NCOL];
#pragma unroll
    for (int u = 0; u < 4; ++u) en[u] = sorted[e + u];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const TA* row = A + (int64_t)(en[u] >> 1) * lda;
#pragma unroll
      for (int c = 0; c < NCOL; ++c) {
        const int64_t col = tid + 256 * c;
        v[u][c] = col < d ? (double)row[col] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < NCOL; ++c) acc[c] += (en[u] & 1u) ? -v[u][c] : v[u][c];
  }
  for (; e < e1; ++e) {
    const uint32_t en = sorted[e];
    const TA* row = A + (int64_t)(en >> 1) * lda;
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
      const int64_t col = tid + 256 * c;
      const double v = col < d ? (double)row[col] : 0.0;
      acc[c] += (en & 1u) ? -v : v;
    }
  }
#pragma unroll
  for (int c = 0; c < NCOL; ++c) {
    const int64_t col = tid + 256 * c;
    if (col < d) SA[(int64_t)h * ldsa + col] = acc[c] * scale;
  }
}

void sjlt_apply(hipStream_t st, uint64_t seed, uint64_t t, const void* A, int a_f32, int64_t n,
                int64_t d, int64_t lda, int64_t m, int s, SjltScratch sc, double* SA, int64_t ldsa) {
  const int64_t nblk = sjlt_nblk(n);
  launch_sjlt_draw(st, seed, t, n, m, s, sc.targets, sc.signs, sc.err);
  hipLaunchKernelGGL(k_sjlt_count, dim3((unsigned)nblk), dim3(256), 0, st, sc.targets, n, s, (int)m,
                     nblk, sc.cnt);
  exclusive_scan_i32(st, sc.cnt, sc.off, m * nblk, sc.scan_tmp);
  int nbits = 0;
  while ((1ll << nbits) < m) ++nbits;
  hipLaunchKernelGGL(k_sjlt_scatter, dim3((unsigned)nblk), dim3(64), 0, st, sc.targets, sc.signs, n,
                     s, (int)m, nbits, nblk, sc.off, sc.sorted);
  hipLaunchKernelGGL(k_sjlt_bstart, dim3((unsigned)((m + 256) / 256)), dim3(256), 0, st, sc.off,
                     (int)m, nblk, n * (int64_t)s, sc.bstart);
  const double scale = 1.0 / sqrt((double)s);
  const int ncol = (int)((d + 255) / 256);
#define LSQ_RED(TA, NC)                                                                           \
  hipLaunchKernelGGL((k_sjlt_reduce<TA, NC>), dim3((unsigned)m), dim3(256), 0, st, (const TA*)A, d, \
                     lda, sc.sorted, sc.bstart, scale, SA, ldsa)
  if (a_f32) {
    if (ncol <= 1) LSQ_RED(float, 1);
    else if (ncol <= 2) LSQ_RED(float, 2);
    else LSQ_RED(float, 4);
  } else {
    if (ncol <= 1) LSQ_RED(double, 1);
    else if (ncol <= 2) LSQ_RED(double, 2);
    else LSQ_RED(double, 4);
  }
#undef LSQ_RED
}

}  // namespace lsq
