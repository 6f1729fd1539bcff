// Shared device helpers of liblsq (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lsq.h"

#define LSQ_WAVE 64

namespace lsq {

// ---------------------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).  One round maps (c0, c1, c2, c3) to
// (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is bumped by the Weyl
// constants between rounds.
// ---------------------------------------------------------------------------------------------------
struct u64x4 {
  uint64_t x, y, z, w;
};

// The 128-bit product a b as (lo, hi).  On the device from four 32 x 32 + 64-bit multiply-adds on the
// 32-bit halves (schoolbook), which yields both halves together.
__host__ __device__ __forceinline__ void mul128(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint64_t a0 = (uint32_t)a, a1 = a >> 32, b0 = (uint32_t)b, b1 = b >> 32;
  const uint64_t t = a0 * b0;
  const uint64_t u = a1 * b0 + (t >> 32);
  const uint64_t v = a0 * b1 + (uint32_t)u;
  hi = a1 * b1 + ((u >> 32) + (v >> 32));
  lo = (v << 32) | (uint32_t)t;
#else
  const unsigned __int128 p = (unsigned __int128)a * b;
  lo = (uint64_t)p;
  hi = (uint64_t)(p >> 64);
#endif
}

// Philox4x64 with its state exposed, so that the ten rounds of one block can be evaluated in pieces
// (rounds [R0, R1) at a time) spread between other instructions.  Round r uses the key bumped r times
// by the Weyl constants.
struct PhiloxState {
  uint64_t c0, c1, c2, c3, k0, k1;
  template <int R0, int R1>
  __host__ __device__ __forceinline__ void rounds() {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = R0; r < R1; ++r) {
      const uint64_t kr0 = k0 + (uint64_t)r * W0, kr1 = k1 + (uint64_t)r * W1;
      uint64_t lo0, hi0, lo1, hi1;
      mul128(M0, c0, lo0, hi0);
      mul128(M1, c2, lo1, hi1);
      const uint64_t n0 = hi1 ^ c1 ^ kr0, n2 = hi0 ^ c3 ^ kr1;
      c0 = n0;
      c1 = lo1;
      c2 = n2;
      c3 = lo0;
    }
  }
};

__host__ __device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                        uint64_t c3, uint64_t k0, uint64_t k1) {
  PhiloxState s{c0, c1, c2, c3, k0, k1};
  s.rounds<0, 10>();
  return {s.c0, s.c1, s.c2, s.c3};
}

enum : uint64_t { TAG_SRHT = 1, TAG_SJLT = 2, TAG_GAUSS = 3 };
constexpr int MAX_SJLT_WORDS = 4096;
constexpr int MAX_SJLT_S = 32;

// Uniform target in [0, m) from the high 32 bits of a word (multiply-shift with rejection).
__device__ __forceinline__ bool sjlt_propose(uint64_t w, uint32_t m, uint32_t thr, uint32_t* h) {
  const uint64_t P = (w >> 32) * (uint64_t)m;
  *h = (uint32_t)(P >> 32);
  return (uint32_t)P >= thr;
}

// sin x and cos x for 0 <= x <= 2 pi (+ a few ulp) in FP64: Cody-Waite reduction x = k pi/2 + r with
// pi/2 split into three parts (33 + 33 + 53 bits, so k P1 and k P2 are exact for k <= 4 and x - k P1 is
// exact), then the Taylor series of sin and cos on |r| <= pi/4 to degree 17 and 18 (truncation below
// 1e-19), placed by the quadrant k mod 4.
__device__ __forceinline__ void sincos_0_2pi(double x, double& sn, double& cs) {
  const double P1 = 0x1.921fb54400000p+0, P2 = 0x1.0b4611a600000p-34, P3 = 0x1.3198a2e037073p-69;
  const double k = rint(x * 0.63661977236758134);  // 2 / pi
  double r = fma(-k, P1, x);
  r = fma(-k, P2, r);
  r = fma(-k, P3, r);
  const double z = r * r;
  double ps = -1.0 / 1307674368000.0 + z * (1.0 / 355687428096000.0);  // -1/15!, 1/17!
  ps = fma(z, ps, 1.0 / 6227020800.0);
  ps = fma(z, ps, -1.0 / 39916800.0);
  ps = fma(z, ps, 1.0 / 362880.0);
  ps = fma(z, ps, -1.0 / 5040.0);
  ps = fma(z, ps, 1.0 / 120.0);
  ps = fma(z, ps, -1.0 / 6.0);
  const double s = fma(r * z, ps, r);
  double pc = 1.0 / 20922789888000.0 + z * (-1.0 / 6402373705728000.0);  // 1/16!, -1/18!
  pc = fma(z, pc, -1.0 / 87178291200.0);
  pc = fma(z, pc, 1.0 / 479001600.0);
  pc = fma(z, pc, -1.0 / 3628800.0);
  pc = fma(z, pc, 1.0 / 40320.0);
  pc = fma(z, pc, -1.0 / 720.0);
  pc = fma(z, pc, 1.0 / 24.0);
  pc = fma(z, pc, -0.5);
  const double c = fma(z, pc, 1.0);
  // quadrant q: (sin, cos) = (s, c), (c, -s), (-s, -c), (-c, s) for q = 0, 1, 2, 3
  const int q = (int)k & 3;
  const double a = (q & 1) ? c : s, b = (q & 1) ? s : c;
  sn = a * ((q & 2) ? -1.0 : 1.0);
  cs = b * (((q + 1) & 2) ? -1.0 : 1.0);
}

// ln u for 2^-32 <= u <= 1 in FP64, without branches (u is never zero, negative, subnormal or special
// here): u = f 2^e with f in [sqrt(1/2), sqrt(2)) by frexp, ln u = e ln 2 + ln f with ln 2 split into 42 +
// 53 bits (e ln2_hi exact), and ln f = 2 atanh(s) = 2 (s + s^3/3 + ... + s^23/23), s = (f - 1)/(f + 1),
// |s| <= 0.172 (truncation below 1e-19).
__device__ __forceinline__ double log_unit(double u) {
  int e;
  double f = frexp(u, &e);  // [1/2, 1)
  const bool lo = f < 0.70710678118654752;
  f = lo ? 2.0 * f : f;
  e = lo ? e - 1 : e;
  const double sv = (f - 1.0) / (f + 1.0);
  const double z = sv * sv;
  double p = fma(z, 1.0 / 23.0, 1.0 / 21.0);
  p = fma(z, p, 1.0 / 19.0);
  p = fma(z, p, 1.0 / 17.0);
  p = fma(z, p, 1.0 / 15.0);
  p = fma(z, p, 1.0 / 13.0);
  p = fma(z, p, 1.0 / 11.0);
  p = fma(z, p, 1.0 / 9.0);
  p = fma(z, p, 1.0 / 7.0);
  p = fma(z, p, 1.0 / 5.0);
  p = fma(z, p, 1.0 / 3.0);
  const double lf = fma(2.0 * sv * z, p, 2.0 * sv);
  const double LN2_HI = 0x1.62e42fefa3800p-1, LN2_LO = 0x1.ef35793c76730p-45;
  return fma((double)e, LN2_HI, fma((double)e, LN2_LO, lf));
}

// Both standard normals of one 64-bit word by Box-Muller in FP64 (a = low 32 bits, b = high 32 bits):
// u1 = (a + 1) 2^-32 in (0, 1] and u2 = b 2^-32 are exact, r = sqrt(-2 ln u1), the angle 2 pi u2 is
// rounded to FP64 once, c = r cos(angle) (even columns), s = r sin(angle) (odd columns); ln by the
// reduction above, sqrt the device library's, sin and cos by sincos_0_2pi.
__device__ __forceinline__ void box_muller_pair_f64(uint64_t w, double& c, double& s) {
  const uint32_t a = (uint32_t)w, b = (uint32_t)(w >> 32);
  const double u1 = ((double)a + 1.0) * 0x1p-32;
  const double u2 = (double)b * 0x1p-32;
  const double r = sqrt(-2.0 * log_unit(u1));
  double sn, cs;
  sincos_0_2pi(2.0 * 3.141592653589793 * u2, sn, cs);
  c = r * cs;
  s = r * sn;
}

// ---------------------------------------------------------------------------------------------------
// Reductions.  All are fixed-order butterflies, so results are bitwise reproducible.
// ---------------------------------------------------------------------------------------------------
template <int WIDTH, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = WIDTH / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, WIDTH);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum<LSQ_WAVE>(v); }
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = LSQ_WAVE / 2; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, LSQ_WAVE));
  return v;
}

// Sums over aligned groups of G lanes, every lane of a group receiving the group's sum, without
// LDS: DPP quad permutations (xor 1, xor 2) and mirrors (8- and 16-lane groups, whose halves are
// already uniform), then the gfx950 permlane swaps across 16-lane rows (xor 16) and wave halves
// (xor 32).  Every lane adds the same two operands, so all lanes of a group hold identical bits.
// All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double xor16_sum(double v) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ __forceinline__ double xor32_sum(double v) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
// Lane l's value, uniform across the wavefront (two scalar reads).
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
template <int G>
__device__ __forceinline__ double grp_sum(double v) {
  if (G >= 2) v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  if (G >= 4) v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  if (G >= 8) v += dpp_d<0x141>(v);  // row_half_mirror
  if (G >= 16) v += dpp_d<0x140>(v); // row_mirror
  if (G >= 32) v = xor16_sum(v);
  if (G >= 64) v = xor32_sum(v);
  return v;
}

// Block-wide sum of K values per thread (NT threads, all active); every thread receives the K totals.
// scratch: at least (NT/64) * K + K doubles of shared memory.
template <int NT, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* scratch) {
  constexpr int NW = NT / LSQ_WAVE;
  const int lane = threadIdx.x & (LSQ_WAVE - 1), wv = threadIdx.x / LSQ_WAVE;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = grp_sum<LSQ_WAVE>(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) scratch[wv * K + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < NW; ++w) s += scratch[w * K + threadIdx.x];
    scratch[NW * K + threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = scratch[NW * K + k];
  __syncthreads();
}

// Device-side solver state shared by the iteration kernels.
struct DevState {
  int done;       // stop rule met (or fatal): later kernels of the queued iterations are no-ops
  int iters;      // iterations completed
  int status;     // lsq_status detected on the device (RANK, NONFINITE)
  int pad;
  double rho;     // r^T rhat
  double rho0;    // r_0^T rhat_0
  double alpha;
  double pHp;
  double est;     // current stop-rule estimate (or exact error)
  double tol;     // stop when est <= tol
  double xrefb;   // x_ref^T b (exact-error trace)
  double scal;    // scalar result of the last residual pass
};

}  // namespace lsq
