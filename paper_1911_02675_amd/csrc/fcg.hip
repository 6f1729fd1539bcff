// Flexible conjugate gradient with refreshed sketches (Section 1.2, analysed in Section 4): the
// d-vector steps of one iteration.  The sketch, the factorization, v_t = W W^T r_t and the pass
// H p_t = A^T (A p_t) are the solver's existing kernels; these two single-workgroup kernels do the
// conjugation against the window of earlier directions and the line-search step.
#include "internal.h"

namespace lsq {

constexpr int FCG_NT = 1024;
constexpr int FCG_NW = FCG_NT / 64;

// p_t = v - sum_{j = t-kt}^{t-1} c_j p_j with c_j = <v, H p_j> / <p_j, H p_j> (0 when that is not
// positive).  Direction j lives in ring slot j % K of P, HP and php.  Wavefront w forms the dot
// products of window entries w, w + 16, ...; then each thread subtracts the projections from its
// elements of v in increasing j and writes p_t into slot t % K (its own elements only, after reading
// them, so the slot of j = t - K may be reused).
__global__ __launch_bounds__(FCG_NT) void k_fcg_orth(const double* __restrict__ v, double* __restrict__ P,
                                                     const double* __restrict__ HP,
                                                     const double* __restrict__ php, int64_t d, int t,
                                                     int kt, int K) {
  __shared__ double c[FCG_MAX_WINDOW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = wv; i < kt; i += FCG_NW) {
    const int row = (t - kt + i) % K;
    const double* h = HP + (int64_t)row * d;
    double s = 0.0;
    for (int64_t e = lane; e < d; e += 64) s = fma(v[e], h[e], s);
    s = grp_sum<64>(s);
    if (lane == 0) {
      const double ph = php[row];
      c[i] = ph > 0.0 ? s / ph : 0.0;
    }
  }
  __syncthreads();
  double* p = P + (int64_t)(t % K) * d;
  for (int64_t e = tid; e < d; e += FCG_NT) {
    double x = v[e];
    for (int i = 0; i < kt; ++i) x = fma(-c[i], P[(int64_t)((t - kt + i) % K) * d + e], x);
    p[e] = x;
  }
}

// red = (H p_t, <p_t, H p_t>) from the fused pass.  alpha = <p_t, r_t> / <p_t, H p_t> (0 when that is
// not positive); x += alpha p_t; r -= alpha H p_t; H p_t and <p_t, H p_t> go to the ring slot.
__global__ __launch_bounds__(FCG_NT) void k_fcg_step(const double* __restrict__ p, const double* __restrict__ red,
                                                     int64_t d, double* __restrict__ x, double* __restrict__ r,
                                                     double* __restrict__ hp_slot, double* __restrict__ php_slot) {
  __shared__ double sh[FCG_NW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double s = 0.0;
  for (int64_t e = tid; e < d; e += FCG_NT) s = fma(p[e], r[e], s);
  s = grp_sum<64>(s);
  if (lane == 0) sh[wv] = s;
  __syncthreads();
  double pr = 0.0;
  for (int w = 0; w < FCG_NW; ++w) pr += sh[w];
  const double pHp = red[d];
  const double alpha = pHp > 0.0 ? pr / pHp : 0.0;
  for (int64_t e = tid; e < d; e += FCG_NT) {
    const double h = red[e];
    x[e] = fma(alpha, p[e], x[e]);
    r[e] = fma(-alpha, h, r[e]);
    hp_slot[e] = h;
  }
  if (tid == 0) *php_slot = pHp;
}

void fcg_orth(hipStream_t st, const double* v, double* P, const double* HP, const double* php, int64_t d,
              int t, int kt, int K) {
  hipLaunchKernelGGL(k_fcg_orth, dim3(1), dim3(FCG_NT), 0, st, v, P, HP, php, d, t, kt, K);
}

void fcg_step(hipStream_t st, const double* p, const double* red, int64_t d, double* x, double* r,
              double* hp_slot, double* php_slot) {
  hipLaunchKernelGGL(k_fcg_step, dim3(1), dim3(FCG_NT), 0, st, p, red, d, x, r, hp_slot, php_slot);
}

}  // namespace lsq
