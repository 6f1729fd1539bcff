// Iteration kernels: the fused pass over A and the small d-vector steps of PCG (Section 1.2) and
// IHS / Polyak-IHS (Section 1.1).
//
// Fused pass: every PCG step needs H p = A^T (A p) and p^T H p = ||A p||^2.  A row group of G lanes
// (a wavefront for d > 64) holds one row of A in registers, forms q_j = a_j . v with a butterfly
// reduction inside the group, and accumulates q_j a_j and q_j^2 without touching A again, so A is
// read from HBM exactly once per step and q is never stored.  Per-workgroup partial sums go to a
// small buffer and are reduced in a fixed order (no floating-point atomics: results are bitwise
// reproducible).
#include "internal.h"

namespace lsq {

// 16-byte (or scalar) loads of A with the non-temporal hint: A is streamed once per pass and
// must not evict the small vectors and partials from the caches (measured on MI355X: ~7.0 TB/s
// for non-temporal streaming reads against ~6.2 TB/s for ordinary loads).
typedef double lsq_d2v __attribute__((ext_vector_type(2)));
typedef float lsq_f4v __attribute__((ext_vector_type(4)));
template <typename T, int VEC>
struct VecLoad;
template <>
struct VecLoad<double, 2> {
  __device__ static void get(const double* p, double (&o)[2]) {
    const lsq_d2v v = __builtin_nontemporal_load((const lsq_d2v*)p);
    o[0] = v[0];
    o[1] = v[1];
  }
};
template <>
struct VecLoad<float, 4> {
  __device__ static void get(const float* p, float (&o)[4]) {
    const lsq_f4v v = __builtin_nontemporal_load((const lsq_f4v*)p);
    o[0] = v[0];
    o[1] = v[1];
    o[2] = v[2];
    o[3] = v[3];
  }
};
template <typename T>
struct VecLoad<T, 1> {
  __device__ static void get(const T* p, T (&o)[1]) { o[0] = __builtin_nontemporal_load(p); }
};

constexpr int FUSED_NT = 256;

// TA: storage type of A; TM: arithmetic type of the products; G lanes per row; NCH chunks of VEC
// contiguous elements per lane (d <= G * NCH * VEC); MODE 0: q = a.v, MODE 1: q = y_j - a.v.
template <typename TA, typename TM, int G, int NCH, int VEC, int MODE, int UNR, bool FULL>
__global__ __launch_bounds__(FUSED_NT) void k_fused(const TA* __restrict__ A, int64_t n, int d,
                                                    int64_t lda, const double* __restrict__ v,
                                                    const double* __restrict__ y,
                                                    int64_t rows_per_wg, double* __restrict__ part,
                                                    const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int NGRP = FUSED_NT / G;
  __shared__ double red[(FUSED_NT / 64) * 1024 + (FUSED_NT / 64)];
  const int tid = threadIdx.x;
  const int gl = tid % G, grp = tid / G;
  TM pv[NCH][VEC];
  TM wacc[NCH][VEC];
#pragma unroll
  for (int i = 0; i < NCH; ++i)
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      const int e = (gl + G * i) * VEC + u;
      pv[i][u] = e < d ? (TM)v[e] : (TM)0;
      wacc[i][u] = (TM)0;
    }
  TM sacc = (TM)0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min(n, r0 + rows_per_wg);
  int64_t r = r0 + grp;
  // Lanes whose chunk lies past d load from the row start instead and discard the value: the loads
  // are unconditional (no branches), so the compiler can issue all of them back to back.
  bool ok[NCH];
  int off[NCH];
#pragma unroll
  for (int i = 0; i < NCH; ++i) {
    const int e = (gl + G * i) * VEC;
    ok[i] = FULL || e < d;
    off[i] = ok[i] ? e : 0;
  }
  // UNR rows in flight per group
  for (; r + (UNR - 1) * NGRP < r1; r += UNR * NGRP) {
    TA a[UNR][NCH][VEC];
#pragma unroll
    for (int i = 0; i < NCH; ++i)
#pragma unroll
      for (int k = 0; k < UNR; ++k) {
        VecLoad<TA, VEC>::get(A + (r + k * NGRP) * lda + off[i], a[k][i]);
        if (!FULL) {
#pragma unroll
          for (int u = 0; u < VEC; ++u) a[k][i][u] = ok[i] ? a[k][i][u] : (TA)0;
        }
      }
    TM q[UNR];
#pragma unroll
    for (int k = 0; k < UNR; ++k) q[k] = (TM)0;
#pragma unroll
    for (int i = 0; i < NCH; ++i)
#pragma unroll
      for (int u = 0; u < VEC; ++u)
#pragma unroll
        for (int k = 0; k < UNR; ++k) q[k] = fma((TM)a[k][i][u], pv[i][u], q[k]);
#pragma unroll
    for (int k = 0; k < UNR; ++k) {
      q[k] = group_sum<G>(q[k]);
      if (MODE == 1) q[k] = (TM)(y[r + k * NGRP] - (double)q[k]);
    }
#pragma unroll
    for (int i = 0; i < NCH; ++i)
#pragma unroll
      for (int u = 0; u < VEC; ++u)
#pragma unroll
        for (int k = 0; k < UNR; ++k) wacc[i][u] = fma(q[k], (TM)a[k][i][u], wacc[i][u]);
    if (gl == 0)
#pragma unroll
      for (int k = 0; k < UNR; ++k) sacc = fma(q[k], q[k], sacc);
  }
  for (; r < r1; r += NGRP) {
    TA a0[NCH][VEC];
#pragma unroll
    for (int i = 0; i < NCH; ++i) {
      VecLoad<TA, VEC>::get(A + r * lda + off[i], a0[i]);
      if (!FULL) {
#pragma unroll
        for (int u = 0; u < VEC; ++u) a0[i][u] = ok[i] ? a0[i][u] : (TA)0;
      }
    }
    TM q0 = (TM)0;
#pragma unroll
    for (int i = 0; i < NCH; ++i)
#pragma unroll
      for (int u = 0; u < VEC; ++u) q0 = fma((TM)a0[i][u], pv[i][u], q0);
    q0 = group_sum<G>(q0);
    if (MODE == 1) q0 = (TM)(y[r] - (double)q0);
#pragma unroll
    for (int i = 0; i < NCH; ++i)
#pragma unroll
      for (int u = 0; u < VEC; ++u) wacc[i][u] = fma(q0, (TM)a0[i][u], wacc[i][u]);
    if (gl == 0) sacc = fma(q0, q0, sacc);
  }
  // combine the groups of a wavefront (they hold the same columns), then the wavefronts
  double wd[NCH][VEC];
#pragma unroll
  for (int i = 0; i < NCH; ++i)
#pragma unroll
    for (int u = 0; u < VEC; ++u) {
      double x = (double)wacc[i][u];
#pragma unroll
      for (int off = G; off < 64; off <<= 1) x += __shfl_xor(x, off, 64);
      wd[i][u] = x;
    }
  double sd = wave_sum((double)sacc);
  const int lane = tid & 63, wv = tid >> 6;
  if (lane < G) {
#pragma unroll
    for (int i = 0; i < NCH; ++i)
#pragma unroll
      for (int u = 0; u < VEC; ++u) {
        const int e = (lane + G * i) * VEC + u;
        if (e < d) red[wv * 1024 + e] = wd[i][u];
      }
  }
  if (lane == 0) red[(FUSED_NT / 64) * 1024 + wv] = sd;
  __syncthreads();
  double* out = part + (int64_t)blockIdx.x * (d + 1);
  for (int e = tid; e < d; e += FUSED_NT) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < FUSED_NT / 64; ++w) s += red[w * 1024 + e];
    out[e] = s;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < FUSED_NT / 64; ++w) s += red[(FUSED_NT / 64) * 1024 + w];
    out[d] = s;
  }
}

// Grid of the fused pass: groups_per_cu x CUs workgroups (oversubscribed: workgroups that finish
// early are replaced, which evens out the streaming across channels); small problems use fewer
// groups of at least 64 rows.  groups_per_cu is a tuning parameter (lsq_tune "fused_groups_per_cu").
static int g_num_cus = 0;
int g_fused_groups_per_cu = 8;

int fused_nwg(int64_t n, int64_t d) {
  (void)d;
  if (g_num_cus == 0) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      g_num_cus = cus;
    else
      g_num_cus = 256;
  }
  int64_t nwg = (n + 63) / 64;
  const int64_t cap = (int64_t)g_num_cus * g_fused_groups_per_cu;
  if (nwg > cap) nwg = cap;
  return (int)(nwg < 1 ? 1 : nwg);
}

template <typename TA, typename TM, int G, int NCH, int VEC>
static int fused_launch(hipStream_t st, const TA* A, int64_t n, int64_t d, int64_t lda, int mode,
                        const double* v, const double* y, double* part, int nwg, const int* done) {
  constexpr int UNR = 2;
  const int g = nwg;
  const int64_t rpw = (n + g - 1) / g;
  const bool full = d == (int64_t)G * NCH * VEC;
#define LSQ_FUSED_GO(M, F)                                                                         \
  hipLaunchKernelGGL((k_fused<TA, TM, G, NCH, VEC, M, UNR, F>), dim3(g), dim3(FUSED_NT), 0, st, A, n, \
                     (int)d, lda, v, y, rpw, part, done)
  if (mode == 0) {
    if (full) LSQ_FUSED_GO(0, true);
    else LSQ_FUSED_GO(0, false);
  } else {
    if (full) LSQ_FUSED_GO(1, true);
    else LSQ_FUSED_GO(1, false);
  }
#undef LSQ_FUSED_GO
  return g;
}

template <typename TA, typename TM, int VEC>
static int fused_dispatch(hipStream_t st, const TA* A, int64_t n, int64_t d, int64_t lda, int mode,
                           const double* v, const double* y, double* part, int nwg,
                           const int* done) {
  if (d <= 16 * VEC * 2) {
    if (d <= 16 * VEC)
      return fused_launch<TA, TM, 16, 1, VEC>(st, A, n, d, lda, mode, v, y, part, nwg, done);
    else
      return fused_launch<TA, TM, 16, 2, VEC>(st, A, n, d, lda, mode, v, y, part, nwg, done);
  }
  const int64_t nch = (d + 64 * VEC - 1) / (64 * VEC);
  if (nch <= 1)
    return fused_launch<TA, TM, 64, 1, VEC>(st, A, n, d, lda, mode, v, y, part, nwg, done);
  else if (nch <= 2)
    return fused_launch<TA, TM, 64, 2, VEC>(st, A, n, d, lda, mode, v, y, part, nwg, done);
  else if (nch <= 4)
    return fused_launch<TA, TM, 64, 4, VEC>(st, A, n, d, lda, mode, v, y, part, nwg, done);
  else if (nch <= 8)
    return fused_launch<TA, TM, 64, 8, VEC>(st, A, n, d, lda, mode, v, y, part, nwg, done);
  else
    return fused_launch<TA, TM, 64, 16, VEC>(st, A, n, d, lda, mode, v, y, part, nwg, done);
}

int fused_pass(hipStream_t st, const void* A, int a_f32, int f32_math, int64_t n, int64_t d,
               int64_t lda, int mode, const double* v, const double* y, double* part, int nwg,
               const int* done) {
  const uintptr_t addr = (uintptr_t)A;
  if (a_f32) {
    const bool vec = (addr % 16 == 0) && (lda % 4 == 0) && (d % 4 == 0);
    const float* Af = (const float*)A;
    if (f32_math) {
      if (vec) return fused_dispatch<float, float, 4>(st, Af, n, d, lda, mode, v, y, part, nwg, done);
      else return fused_dispatch<float, float, 1>(st, Af, n, d, lda, mode, v, y, part, nwg, done);
    } else {
      if (vec) return fused_dispatch<float, double, 4>(st, Af, n, d, lda, mode, v, y, part, nwg, done);
      else return fused_dispatch<float, double, 1>(st, Af, n, d, lda, mode, v, y, part, nwg, done);
    }
  } else {
    const bool vec = (addr % 16 == 0) && (lda % 2 == 0) && (d % 2 == 0);
    const double* Ad = (const double*)A;
    if (vec) return fused_dispatch<double, double, 2>(st, Ad, n, d, lda, mode, v, y, part, nwg, done);
    else return fused_dispatch<double, double, 1>(st, Ad, n, d, lda, mode, v, y, part, nwg, done);
  }
}

// --------------------------------------------------------------------------------------------------
// Fixed-order reduction of the per-workgroup partials.
// --------------------------------------------------------------------------------------------------
// Stage 1: workgroup (column block, split) sums rows [split*chunk, (split+1)*chunk) of the partials.
__global__ __launch_bounds__(256) void k_reduce_stage1(const double* __restrict__ part, int nwg,
                                                       int64_t d, double* __restrict__ part2,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[256];
  const int64_t width = d + 1;
  const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int ph = threadIdx.x >> 6;
  const int chunk = (nwg + REDUCE_SPLIT - 1) / REDUCE_SPLIT;
  const int g0 = blockIdx.y * chunk, g1 = min(nwg, g0 + chunk);
  double s = 0.0;
  if (c < width)
    for (int g = g0 + ph; g < g1; g += 4) s += part[(int64_t)g * width + c];
  const int cl = threadIdx.x & 63;
  sh[ph * 64 + cl] = s;
  __syncthreads();
  if (ph == 0 && c < width)
    part2[(int64_t)blockIdx.y * width + c] = ((sh[cl] + sh[64 + cl]) + sh[128 + cl]) + sh[192 + cl];
}

void reduce_stage1(hipStream_t st, const double* part, int nwg, int64_t d, double* part2,
                   const int* done) {
  hipLaunchKernelGGL(k_reduce_stage1, dim3((unsigned)((d + 1 + 63) / 64), REDUCE_SPLIT), dim3(256), 0, st,
                     part, nwg, d, part2, done);
}

// Stage 2 for one column: sum of the REDUCE_SPLIT rows, in order.
__device__ __forceinline__ double col2(const double* part2, int nrows, int64_t width, int64_t c) {
  double s = 0.0;
  for (int g = 0; g < nrows; ++g) s += part2[(int64_t)g * width + c];
  return s;
}

__global__ __launch_bounds__(256) void k_reduce_cols(const double* __restrict__ part2, int nrows,
                                                     int64_t d, double* __restrict__ out,
                                                     const int* __restrict__ done) {
  if (done && *done) return;
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c <= d) out[c] = col2(part2, nrows, d + 1, c);
}

void reduce_partials(hipStream_t st, const double* part, double* part2, int nwg, int64_t d,
                     double* out, const int* done) {
  reduce_stage1(st, part, nwg, d, part2, done);
  hipLaunchKernelGGL(k_reduce_cols, dim3((unsigned)((d + 1 + 255) / 256)), dim3(256), 0, st, part2,
                     REDUCE_SPLIT, d, out, done);
}

// alpha = rho / p^T H p;  x += alpha p;  r -= alpha H p  (H p and p^T H p from the stage-1 rows).
__global__ __launch_bounds__(256) void k_pcg_xr(const double* __restrict__ part2, int nrows, int64_t d,
                                                double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p, DevState* ds) {
  if (ds->done) return;
  const double rho = ds->rho;
  const int64_t width = d + 1;
  const double pHp = col2(part2, nrows, width, d);
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool bad = !(pHp > 0.0) || !isfinite(pHp);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ds->pHp = pHp;
    if (bad) ds->status = isfinite(pHp) ? (int)LSQ_ERR_RANK : (int)LSQ_ERR_NONFINITE;
  }
  if (bad) return;
  const double alpha = rho / pHp;
  if (blockIdx.x == 0 && threadIdx.x == 0) ds->alpha = alpha;
  if (c < d) {
    const double w = col2(part2, nrows, width, c);
    x[c] = fma(alpha, p[c], x[c]);
    r[c] = fma(-alpha, w, r[c]);
  }
}

void pcg_update_xr(hipStream_t st, const double* part2, int nrows, int64_t d, double* x, double* r,
                   const double* p, DevState* ds) {
  hipLaunchKernelGGL(k_pcg_xr, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, part2, nrows, d, x,
                     r, p, ds);
}

// --------------------------------------------------------------------------------------------------
// Preconditioner application rhat = W (W^T r) = R^{-1} R^{-T} r as two triangular GEMVs (one
// wavefront per output row), with per-workgroup partials of r . rhat.
// --------------------------------------------------------------------------------------------------
template <bool UPPER, bool DOT>
__global__ __launch_bounds__(256) void k_trigemv(const double* __restrict__ M, int64_t d,
                                                 const double* __restrict__ xin,
                                                 double* __restrict__ xout,
                                                 const double* __restrict__ rdot,
                                                 double* __restrict__ dotpart,
                                                 const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sh[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  double prod = 0.0;
  if (i < d) {
    const int64_t k0 = UPPER ? i : 0, k1 = UPPER ? d : i + 1;
    const double* row = M + i * d;
    double s = 0.0;
    for (int64_t k = k0 + lane; k < k1; k += 64) s = fma(row[k], xin[k], s);
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

void precond_apply(hipStream_t st, const double* W, const double* WT, int64_t d, const double* r,
                   double* u, double* rhat, double* dotpart, int* ndot, const int* done) {
  const unsigned nb = (unsigned)((d + 3) / 4);
  hipLaunchKernelGGL((k_trigemv<false, false>), dim3(nb), dim3(256), 0, st, WT, d, r, u, nullptr,
                     nullptr, done);
  hipLaunchKernelGGL((k_trigemv<true, true>), dim3(nb), dim3(256), 0, st, W, d, u, rhat, r, dotpart,
                     done);
  *ndot = (int)nb;
}

__device__ double block1024_sum(double v, double* sh) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < 16; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// rho' = r . rhat; beta = rho'/rho; p = rhat + beta p; stop-rule estimate and trace.
__global__ __launch_bounds__(1024) void k_pcg_p(int64_t d, const double* __restrict__ rhat,
                                                double* __restrict__ p,
                                                const double* __restrict__ dotpart, int ndot,
                                                DevState* ds, const double* __restrict__ x,
                                                const double* __restrict__ r,
                                                const double* __restrict__ xref,
                                                double* __restrict__ trace, int trace_len) {
  if (ds->done) return;
  __shared__ double sh[16];
  // read the state before any barrier: thread 0 rewrites it at the end
  const double rho = ds->rho, rho0 = ds->rho0, xrefb = ds->xrefb, tol = ds->tol;
  const int it = ds->iters + 1;
  double s = 0.0;
  for (int g = threadIdx.x; g < ndot; g += 1024) s += dotpart[g];
  const double rho_new = block1024_sum(s, sh);
  const double beta = rho_new / rho;
  for (int64_t c = threadIdx.x; c < d; c += 1024) p[c] = fma(beta, p[c], rhat[c]);
  const double proxy = 4.0 * sqrt(fmax(rho_new, 0.0) / rho0);
  double est = proxy;
  if (xref) {
    double e = 0.0;
    for (int64_t c = threadIdx.x; c < d; c += 1024) e += (x[c] - xref[c]) * r[c];
    e = block1024_sum(e, sh);
    est = sqrt(fmax(-e, 0.0) / xrefb);
  }
  if (threadIdx.x == 0) {
    ds->iters = it;
    ds->rho = rho_new;
    ds->est = est;
    if (trace && it < trace_len) trace[it] = est;
    if (!isfinite(rho_new)) {
      ds->status = (int)LSQ_ERR_NONFINITE;
      ds->done = 1;
    } else if (proxy <= tol) {
      ds->done = 1;
    }
    if (ds->status != 0) ds->done = 1;
  }
}

void pcg_update_p(hipStream_t st, int64_t d, const double* rhat, double* p, const double* dotpart,
                  int ndot, DevState* ds, const double* x, const double* r, const double* x_ref,
                  double* trace, int trace_len) {
  hipLaunchKernelGGL(k_pcg_p, dim3(1), dim3(1024), 0, st, d, rhat, p, dotpart, ndot, ds, x, r, x_ref,
                     trace, trace_len);
}

// rho_0 = r_0 . rhat_0, p_0 = rhat_0; trace[0].
__global__ __launch_bounds__(1024) void k_pcg_init(int64_t d, const double* __restrict__ rhat,
                                                   double* __restrict__ p,
                                                   const double* __restrict__ dotpart, int ndot,
                                                   DevState* ds, double tol,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ xref,
                                                   double* __restrict__ trace) {
  __shared__ double sh[16];
  const double xrefb = ds->xrefb;
  double s = 0.0;
  for (int g = threadIdx.x; g < ndot; g += 1024) s += dotpart[g];
  const double rho = block1024_sum(s, sh);
  for (int64_t c = threadIdx.x; c < d; c += 1024) p[c] = rhat[c];
  double est = 4.0;
  if (xref) {
    double e = 0.0;
    for (int64_t c = threadIdx.x; c < d; c += 1024) e += (x[c] - xref[c]) * r[c];
    e = block1024_sum(e, sh);
    est = sqrt(fmax(-e, 0.0) / xrefb);
  }
  if (threadIdx.x == 0) {
    ds->rho = rho;
    ds->rho0 = rho;
    ds->iters = 0;
    ds->status = 0;
    ds->tol = tol;
    ds->est = est;
    if (trace) trace[0] = est;
    ds->done = (rho > 0.0 && isfinite(rho)) ? 0 : 1;
    if (!isfinite(rho)) ds->status = (int)LSQ_ERR_NONFINITE;
  }
}

// ds->xrefb = x_ref . b (denominator of the exact-error trace).
__global__ __launch_bounds__(1024) void k_dot_state(int64_t d, const double* __restrict__ a,
                                                    const double* __restrict__ b, DevState* ds) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < d; c += 1024) s += a[c] * b[c];
  s = block1024_sum(s, sh);
  if (threadIdx.x == 0) ds->xrefb = s;
}

void dot_to_state(hipStream_t st, int64_t d, const double* a, const double* b, DevState* ds) {
  hipLaunchKernelGGL(k_dot_state, dim3(1), dim3(1024), 0, st, d, a, b, ds);
}

void pcg_init(hipStream_t st, int64_t d, const double* rhat, double* p, const double* dotpart,
              int ndot, DevState* ds, double tol, const double* x, const double* r,
              const double* x_ref, double* trace) {
  hipLaunchKernelGGL(k_pcg_init, dim3(1), dim3(1024), 0, st, d, rhat, p, dotpart, ndot, ds, tol, x, r,
                     x_ref, trace);
}

// --------------------------------------------------------------------------------------------------
// Small vector helpers.
// --------------------------------------------------------------------------------------------------
__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) dst[i] = src[i];
}
__global__ void k_zero(double* __restrict__ dst, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) dst[i] = 0.0;
}
__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, int64_t len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) y[i] = fma(a, x[i], y[i]);
}
void vec_copy(hipStream_t st, double* dst, const double* src, int64_t len) {
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, dst, src, len);
}
void vec_zero(hipStream_t st, double* dst, int64_t len) {
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, dst, len);
}
void vec_axpy(hipStream_t st, double* y, const double* x, double a, int64_t len) {
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, y, x, a, len);
}

// x_{t+1} = x_t + mu h + beta (x_t - x_{t-1}), with h = H_S^{-1} A^T (y - A x_t) = -H_S^{-1} grad f.
__global__ void k_ihs_update(int64_t d, double* __restrict__ x, double* __restrict__ xprev,
                             const double* __restrict__ h, double mu, double beta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d) return;
  const double xi = x[i];
  const double xn = fma(mu, h[i], xi) + beta * (xi - xprev[i]);
  xprev[i] = xi;
  x[i] = xn;
}
void ihs_update(hipStream_t st, int64_t d, double* x, double* xprev, const double* hinvg, double mu,
                double beta) {
  hipLaunchKernelGGL(k_ihs_update, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, d, x, xprev,
                     hinvg, mu, beta);
}

__global__ void k_err_from_resid(const double* scal, double denom, double* out) {
  if (threadIdx.x == 0) *out = sqrt(fmax(*scal, 0.0) / denom);
}
void error_from_resid(hipStream_t st, const double* scal, double denom, double* out) {
  hipLaunchKernelGGL(k_err_from_resid, dim3(1), dim3(64), 0, st, scal, denom, out);
}

}  // namespace lsq
