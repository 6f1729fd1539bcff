// Extra-precise residual for iterative refinement: r = A^T (y - A x) with the dot products a_j . x,
// the differences y_j - a_j . x and the accumulation over rows carried in double-double arithmetic
// (pairs hi + lo with |lo| <= u |hi|), rounded to FP64 once at the end.  Near the solution r is a
// small difference of large terms; computed in plain FP64 its error (about u times the sum of
// |q_j a_j|, amplified by kappa^2 through H_S^{-1}) sets a floor under the refinement's stop estimate,
// which the double-double form lowers by about 1/u.  The products are error-free (a product of two
// doubles is exactly p + fma(a, b, -p)), sums use Knuth's TwoSum.
//
// The arithmetic is about 21 FP64 operations per element of A, so on this GPU the kernel is bound by
// the vector ALU rather than by HBM.  Each wavefront takes two rows at a time (64 lanes x 16 columns
// per lane cover d <= 1024), with the next pair's loads in flight while the current pair is computed.
// The two row dot products are reduced across the wavefront by a reduce-scatter: one permlane32 swap
// leaves row 0's partials in one half of the wavefront and row 1's in the other, then a permlane16
// swap and four DPP steps finish each half, so a row costs three double-double additions instead of
// six.  Every wavefront keeps its own (hi, lo) column sums and writes them as a partial; the partials
// are added in a fixed order by two small kernels.
#include "internal.h"

// The error-free transforms need every + and * rounded as written: no contraction of a product into a
// following add (the product errors are taken with explicit fma calls).
#pragma clang fp contract(off)

namespace lsq {

struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}

// (a.hi + a.lo) + (b.hi + b.lo), renormalised
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  const dd s = two_sum(a.hi, b.hi);
  const double lo = s.lo + (a.lo + b.lo);
  const double hi = s.hi + lo;
  return {hi, lo - (hi - s.hi)};
}

// Unnormalised accumulation of two partial pairs (hi carries the rounded sum, lo the exact rounding
// errors and the low parts).  Symmetric in its two operands bit for bit: TwoSum's error term is
// unique and the remaining additions commute, so the lanes of a reduction group end identical.
__device__ __forceinline__ void dd_acc(double& hi, double& lo, double hi2, double lo2) {
  const dd s = two_sum(hi, hi2);
  hi = s.hi;
  lo = s.lo + (lo + lo2);
}

struct dpair {
  double a, b;
};
// permlane16 / permlane32 swaps of a value with itself: every lane receives its own value and its
// partner's (xor 16, xor 32), in an order that depends on the lane.
__device__ __forceinline__ dpair swap16(double v) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  return {__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1])};
}
// One permlane32 swap of x (in vdst) with y (in vsrc): the two results of each lane are the same
// wavefront half-pair of one of the two inputs.
__device__ __forceinline__ dpair swap32(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
  return {__hiloint2double(hi[0], lo[0]), __hiloint2double(hi[1], lo[1])};
}

constexpr int RDD_NT = 256;
constexpr int RDD_NW = RDD_NT / 64;
constexpr int RDD_GRID = 512;  // 2048 wavefronts: two per SIMD at the kernel's register use
constexpr int RDD_SEG = 32;    // segments of the first reduction stage

template <typename TA, int VEC>
struct RddVec;
template <>
struct RddVec<float, 4> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct RddVec<double, 2> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct RddVec<float, 1> {
  typedef float type;
};
template <>
struct RddVec<double, 1> {
  typedef double type;
};

template <int VEC, typename V>
__device__ __forceinline__ double rdd_elem(const V& v, int u) {
  if constexpr (VEC == 1)
    return (double)v;
  else
    return (double)v[u];
}

// NC chunks of VEC elements per lane; element (chunk c, lane l, u) is column (64 c + l) VEC + u.
// Columns at or beyond d load column 0 of the row (valid memory) and meet x = 0, so they add nothing
// to the dot products; their column sums are never written.
// part: (gridDim.x * RDD_NW) rows of 2 d + 1 doubles: (hi, lo) per column, then sum q_j^2.
template <typename TA, int VEC, int NC, bool PF>
__global__ __launch_bounds__(RDD_NT) void k_resid_dd(const TA* __restrict__ A, int64_t n, int d, int64_t lda,
                                                     const double* __restrict__ x, const double* __restrict__ y,
                                                     double* __restrict__ part) {
  typedef typename RddVec<TA, VEC>::type V;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t gw = (int64_t)blockIdx.x * RDD_NW + wv, nw = (int64_t)gridDim.x * RDD_NW;
  const int64_t npair = (n + 1) / 2;
  double xv[NC][VEC];
  double whi[NC][VEC], wlo[NC][VEC];
  int off[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int e0 = (64 * c + lane) * VEC;
    const bool ok = e0 < d;  // d is a multiple of VEC
    off[c] = ok ? e0 : 0;
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      xv[c][u] = ok ? x[e0 + u] : 0.0;
      whi[c][u] = 0.0;
      wlo[c][u] = 0.0;
    }
  }
  // Row tag through the same half swap as the partials: after it, the lane holds row `mine` of the
  // pair (0 in one half of the wavefront, 1 in the other).
  const int mine = __builtin_amdgcn_permlane32_swap(0, 1, false, false)[0];
  double qq = 0.0;

  V nb[2][NC];
  auto load_pair = [&](int64_t g) {
    const int64_t r0 = 2 * g, r1 = (2 * g + 1 < n) ? 2 * g + 1 : n - 1;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      nb[0][c] = __builtin_nontemporal_load((const V*)(A + r0 * lda + off[c]));
      nb[1][c] = __builtin_nontemporal_load((const V*)(A + r1 * lda + off[c]));
    }
  };
  if constexpr (PF) {
    if (gw < npair) load_pair(gw);
  }
  for (int64_t g = gw; g < npair; g += nw) {
    if constexpr (!PF) load_pair(g);
    double a[2][NC][VEC];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int u = 0; u < VEC; ++u) a[r][c][u] = rdd_elem<VEC>(nb[r][c], u);
    if constexpr (PF) {
      if (g + nw < npair) load_pair(g + nw);
    }
    // s_r = a_r . x per lane: error-free products, TwoSum accumulation (two independent chains)
    double sh[2] = {0.0, 0.0}, sl[2] = {0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int u = 0; u < VEC; ++u)
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const double p = a[r][c][u] * xv[c][u];
          const double pe = fma(a[r][c][u], xv[c][u], -p);
          const dd t = two_sum(sh[r], p);
          sh[r] = t.hi;
          sl[r] = sl[r] + (t.lo + pe);
        }
    // reduce-scatter over the wavefront: half swap (one row per half), then xor 16, 1, 2 and the
    // 8- and 16-lane mirrors within each half
    double hi, lo;
    {
      const dpair h = swap32(sh[0], sh[1]);
      const dpair l = swap32(sl[0], sl[1]);
      hi = h.a;
      lo = l.a;
      dd_acc(hi, lo, h.b, l.b);
    }
    {
      const dpair h = swap16(hi);
      const dpair l = swap16(lo);
      hi = h.a;
      lo = l.a;
      dd_acc(hi, lo, h.b, l.b);
    }
    dd_acc(hi, lo, dpp_d<0xB1>(hi), dpp_d<0xB1>(lo));
    dd_acc(hi, lo, dpp_d<0x4E>(hi), dpp_d<0x4E>(lo));
    dd_acc(hi, lo, dpp_d<0x141>(hi), dpp_d<0x141>(lo));
    dd_acc(hi, lo, dpp_d<0x140>(hi), dpp_d<0x140>(lo));
    // q = y_r - s_r for this half's row, renormalised; zero for the padding row of an odd n
    const int64_t row = 2 * g + mine;
    dd q = two_sum(y[row < n ? row : n - 1], -hi);
    q.lo = q.lo - lo;
    q = two_sum(q.hi, q.lo);
    if (row >= n) q = {0.0, 0.0};
    qq = fma(q.hi, q.hi, qq);
    // both rows' q to every lane (lane 0 holds row `m0`, lane 32 the other)
    const int m0 = __builtin_amdgcn_readlane(mine, 0);
    const double qa_hi = readlane_d(q.hi, 0), qa_lo = readlane_d(q.lo, 0);
    const double qb_hi = readlane_d(q.hi, 32), qb_lo = readlane_d(q.lo, 32);
    const double q0h = m0 == 0 ? qa_hi : qb_hi, q0l = m0 == 0 ? qa_lo : qb_lo;
    const double q1h = m0 == 0 ? qb_hi : qa_hi, q1l = m0 == 0 ? qb_lo : qa_lo;
    // w += q_r a_r (a exact): q.hi a is p + pe exactly, q.lo a is below u of it
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        {
          const double p = q0h * a[0][c][u];
          const double pe = fma(q0h, a[0][c][u], -p);
          const dd t = two_sum(whi[c][u], p);
          whi[c][u] = t.hi;
          wlo[c][u] = wlo[c][u] + (t.lo + fma(q0l, a[0][c][u], pe));
        }
        {
          const double p = q1h * a[1][c][u];
          const double pe = fma(q1h, a[1][c][u], -p);
          const dd t = two_sum(whi[c][u], p);
          whi[c][u] = t.hi;
          wlo[c][u] = wlo[c][u] + (t.lo + fma(q1l, a[1][c][u], pe));
        }
      }
  }
  double* out = part + gw * (2 * (int64_t)d + 1);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int e0 = (64 * c + lane) * VEC;
    if (e0 < d) {
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        out[2 * (e0 + u)] = whi[c][u];
        out[2 * (e0 + u) + 1] = wlo[c][u];
      }
    }
  }
  // each half of the wavefront holds the same q^2 sum for its rows
  const double qq0 = readlane_d(qq, 0), qq1 = readlane_d(qq, 32);
  if (lane == 0) out[2 * d] = qq0 + qq1;
}

// First stage: partials [s np / SEG, (s+1) np / SEG) of column e (e < d: double-double pairs; e = d:
// the q^2 sums) into part2 row s.
__global__ __launch_bounds__(64) void k_resid_dd_seg(const double* __restrict__ part, int64_t np, int d,
                                                     double* __restrict__ part2) {
  const int e = blockIdx.x * 64 + threadIdx.x;
  if (e > d) return;
  const int s = blockIdx.y;
  const int64_t k0 = (int64_t)s * np / RDD_SEG, k1 = (int64_t)(s + 1) * np / RDD_SEG;
  const int64_t stride = 2 * (int64_t)d + 1;
  double* out = part2 + (int64_t)s * stride;
  if (e == d) {
    double acc = 0.0;
    for (int64_t k = k0; k < k1; ++k) acc += part[k * stride + 2 * d];
    out[2 * d] = acc;
    return;
  }
  dd acc = {0.0, 0.0};
  for (int64_t k = k0; k < k1; ++k) acc = dd_add(acc, {part[k * stride + 2 * e], part[k * stride + 2 * e + 1]});
  out[2 * e] = acc.hi;
  out[2 * e + 1] = acc.lo;
}

// Second stage: r[e] = round(sum of the SEG pairs); scal = sum of the q^2 segment sums.
__global__ __launch_bounds__(256) void k_resid_dd_final(const double* __restrict__ part2, int d,
                                                        double* __restrict__ r, double* __restrict__ scal) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > d) return;
  const int64_t stride = 2 * (int64_t)d + 1;
  if (e == d) {
    double s = 0.0;
    for (int k = 0; k < RDD_SEG; ++k) s += part2[k * stride + 2 * d];
    if (scal) *scal = s;
    return;
  }
  dd acc = {0.0, 0.0};
  for (int k = 0; k < RDD_SEG; ++k) acc = dd_add(acc, {part2[k * stride + 2 * e], part2[k * stride + 2 * e + 1]});
  r[e] = acc.hi + acc.lo;
}

size_t resid_dd_part_len(int64_t d) { return (size_t)(RDD_GRID * RDD_NW + RDD_SEG) * (2 * d + 1); }

template <typename TA, int VEC, bool PF>
static bool resid_dd_t(hipStream_t st, const TA* A, int64_t n, int64_t d, int64_t lda, const double* x,
                       const double* y, double* part) {
  const int64_t nc = (d + 64 * VEC - 1) / (64 * VEC);
#define LSQ_RDD(NC)                                                                                  \
  if constexpr (VEC * NC <= 16) {                                                                    \
    if (nc <= NC) {                                                                                  \
      hipLaunchKernelGGL((k_resid_dd<TA, VEC, NC, PF>), dim3(RDD_GRID), dim3(RDD_NT), 0, st, A, n, (int)d, \
                         lda, x, y, part);                                                           \
      return true;                                                                                   \
    }                                                                                                \
  }
  LSQ_RDD(1)
  LSQ_RDD(2)
  LSQ_RDD(4)
  LSQ_RDD(8)
  LSQ_RDD(16)
#undef LSQ_RDD
  return false;
}

bool resid_dd(hipStream_t st, const void* A, int a_f32, int64_t n, int64_t d, int64_t lda, const double* x,
              const double* y, double* part, double* r, double* scal) {
  if (n < 1 || d < 1) return false;
  bool ok;
  if (a_f32) {
    const bool vec = d % 4 == 0 && lda % 4 == 0 && ((uintptr_t)A % 16) == 0;
    ok = vec ? resid_dd_t<float, 4, true>(st, (const float*)A, n, d, lda, x, y, part)
             : resid_dd_t<float, 1, true>(st, (const float*)A, n, d, lda, x, y, part);
  } else {
    const bool vec = d % 2 == 0 && lda % 2 == 0 && ((uintptr_t)A % 16) == 0;
    ok = vec ? resid_dd_t<double, 2, false>(st, (const double*)A, n, d, lda, x, y, part)
             : resid_dd_t<double, 1, false>(st, (const double*)A, n, d, lda, x, y, part);
  }
  if (!ok) return false;
  double* part2 = part + (size_t)RDD_GRID * RDD_NW * (2 * d + 1);
  hipLaunchKernelGGL(k_resid_dd_seg, dim3((unsigned)((d + 1 + 63) / 64), RDD_SEG), dim3(64), 0, st, part,
                     (int64_t)RDD_GRID * RDD_NW, (int)d, part2);
  hipLaunchKernelGGL(k_resid_dd_final, dim3((unsigned)((d + 1 + 255) / 256)), dim3(256), 0, st, part2, (int)d,
                     r, scal);
  return true;
}

}  // namespace lsq
