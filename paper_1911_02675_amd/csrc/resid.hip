// Extra-precise residual for iterative refinement: r = A^T (y - A x) with the dot products a_j . x,
// the differences y_j - a_j . x and the accumulation over rows carried in double-double arithmetic
// (pairs hi + lo with |lo| <= u |hi|), rounded to FP64 once at the end.  Near the solution r is a
// small difference of large terms; computed in plain FP64 its error (about u times the sum of
// |q_j a_j|, amplified by kappa^2 through H_S^{-1}) sets a floor under the refinement's stop estimate,
// which the double-double form lowers by about 1/u.  The products are error-free (a product of two
// doubles is exactly p + fma(a, b, -p)), sums use Knuth's TwoSum.
//
// One wavefront per row at a time (64 lanes x VEC elements per step across the row), rows strided over
// the grid; every wavefront keeps its own (hi, lo) column sums and writes them as a partial, and the
// partials are added in a fixed order.
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

// acc += x (a double)
__device__ __forceinline__ dd dd_add_d(dd a, double x) {
  const dd s = two_sum(a.hi, x);
  const double lo = s.lo + a.lo;
  const double hi = s.hi + lo;
  return {hi, lo - (hi - s.hi)};
}

__device__ __forceinline__ double shfl_d(double v, int mask) { return __shfl_xor(v, mask, 64); }

constexpr int RDD_NT = 256;
constexpr int RDD_NW = RDD_NT / 64;

template <typename TA, int VEC>
__device__ __forceinline__ void rdd_load(const TA* p, double (&o)[VEC]);
template <>
__device__ __forceinline__ void rdd_load<float, 4>(const float* p, double (&o)[4]) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 v = __builtin_nontemporal_load((const f4*)p);
  o[0] = v[0];
  o[1] = v[1];
  o[2] = v[2];
  o[3] = v[3];
}
template <>
__device__ __forceinline__ void rdd_load<double, 2>(const double* p, double (&o)[2]) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2 v = __builtin_nontemporal_load((const d2*)p);
  o[0] = v[0];
  o[1] = v[1];
}
template <>
__device__ __forceinline__ void rdd_load<float, 1>(const float* p, double (&o)[1]) {
  o[0] = __builtin_nontemporal_load(p);
}
template <>
__device__ __forceinline__ void rdd_load<double, 1>(const double* p, double (&o)[1]) {
  o[0] = __builtin_nontemporal_load(p);
}

// NC chunks of VEC elements per lane; element (chunk c, lane l, u) is column (64 c + l) VEC + u.
// part: (gridDim.x * RDD_NW) rows of 2 d + 1 doubles: (hi, lo) per column, then sum q_j^2.
template <typename TA, int VEC, int NC>
__global__ __launch_bounds__(RDD_NT) void k_resid_dd(const TA* __restrict__ A, int64_t n, int d, int64_t lda,
                                                     const double* __restrict__ x, const double* __restrict__ y,
                                                     double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t gw = (int64_t)blockIdx.x * RDD_NW + wv, nw = (int64_t)gridDim.x * RDD_NW;
  double xv[NC][VEC];
  dd w[NC][VEC];
  bool ok[NC];
  int off[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int e0 = (64 * c + lane) * VEC;
    ok[c] = e0 < d;  // d is a multiple of VEC
    off[c] = ok[c] ? e0 : 0;
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      xv[c][u] = ok[c] ? x[e0 + u] : 0.0;
      w[c][u] = {0.0, 0.0};
    }
  }
  double qq = 0.0;
  for (int64_t r = gw; r < n; r += nw) {
    double a[NC][VEC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      rdd_load<TA, VEC>(A + r * lda + off[c], a[c]);
#pragma unroll
      for (int u = 0; u < VEC; ++u) a[c][u] = ok[c] ? a[c][u] : 0.0;
    }
    // s = a_r . x in double-double: error-free products, TwoSum accumulation
    dd s = {0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        const double p = a[c][u] * xv[c][u];
        const double pe = fma(a[c][u], xv[c][u], -p);
        const dd t = two_sum(s.hi, p);
        s.hi = t.hi;
        s.lo += t.lo + pe;
      }
    // across the wavefront (every lane ends with the same pair up to the order of the low parts)
#pragma unroll
    for (int mask = 1; mask < 64; mask <<= 1) {
      const dd o = {shfl_d(s.hi, mask), shfl_d(s.lo, mask)};
      s = dd_add(s, o);
    }
    // q = y_r - s
    dd q = two_sum(y[r], -s.hi);
    q.lo -= s.lo;
    {
      const double hi = q.hi + q.lo;
      q.lo = q.lo - (hi - q.hi);
      q.hi = hi;
    }
    qq = fma(q.hi, q.hi, qq);
    // w += q a_r (a_r exact): q.hi a is p + e exactly, q.lo a is below u of it
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        const double p = q.hi * a[c][u];
        const double pe = fma(q.hi, a[c][u], -p);
        const dd t = two_sum(w[c][u].hi, p);
        w[c][u].hi = t.hi;
        w[c][u].lo += t.lo + (pe + q.lo * a[c][u]);
      }
  }
  double* out = part + (gw) * (2 * (int64_t)d + 1);
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (ok[c]) {
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        const int e = (64 * c + lane) * VEC + u;
        out[2 * e] = w[c][u].hi;
        out[2 * e + 1] = w[c][u].lo;
      }
    }
  if (lane == 0) out[2 * d] = qq;  // lane 0 holds the same q for every row
}

// r[e] = round(sum over partials of (hi, lo)) in a fixed order; scal = sum of the q^2 partials.
__global__ __launch_bounds__(256) void k_resid_dd_reduce(const double* __restrict__ part, int64_t np, int d,
                                                         double* __restrict__ r, double* __restrict__ scal) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > d) return;
  const int64_t stride = 2 * (int64_t)d + 1;
  if (e == d) {
    double s = 0.0;
    for (int64_t k = 0; k < np; ++k) s += part[k * stride + 2 * d];
    if (scal) *scal = s;
    return;
  }
  dd acc = {0.0, 0.0};
  for (int64_t k = 0; k < np; ++k) acc = dd_add(acc, {part[k * stride + 2 * e], part[k * stride + 2 * e + 1]});
  r[e] = acc.hi + acc.lo;
}

constexpr int RDD_GRID = 512;  // 2048 wavefronts

size_t resid_dd_part_len(int64_t d) { return (size_t)RDD_GRID * RDD_NW * (2 * d + 1); }

template <typename TA, int VEC>
static bool resid_dd_t(hipStream_t st, const TA* A, int64_t n, int64_t d, int64_t lda, const double* x,
                       const double* y, double* part) {
  const int64_t nc = (d + 64 * VEC - 1) / (64 * VEC);
#define LSQ_RDD(NC)                                                                                  \
  if constexpr (64 * VEC * NC <= 1024) {                                                             \
    if (nc <= NC) {                                                                                  \
      hipLaunchKernelGGL((k_resid_dd<TA, VEC, NC>), dim3(RDD_GRID), dim3(RDD_NT), 0, st, A, n, (int)d, lda, \
                         x, y, part);                                                                \
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
  bool ok;
  if (a_f32) {
    const bool vec = d % 4 == 0 && lda % 4 == 0 && ((uintptr_t)A % 16) == 0;
    ok = vec ? resid_dd_t<float, 4>(st, (const float*)A, n, d, lda, x, y, part)
             : resid_dd_t<float, 1>(st, (const float*)A, n, d, lda, x, y, part);
  } else {
    const bool vec = d % 2 == 0 && lda % 2 == 0 && ((uintptr_t)A % 16) == 0;
    ok = vec ? resid_dd_t<double, 2>(st, (const double*)A, n, d, lda, x, y, part)
             : resid_dd_t<double, 1>(st, (const double*)A, n, d, lda, x, y, part);
  }
  if (!ok) return false;
  hipLaunchKernelGGL(k_resid_dd_reduce, dim3((unsigned)((d + 1 + 255) / 256)), dim3(256), 0, st, part,
                     (int64_t)RDD_GRID * RDD_NW, (int)d, r, scal);
  return true;
}

}  // namespace lsq
