// Batched form of the fixed-sketch PCG solver (Section 1.2, with the sparse embedding of
// Section 2): many independent problems, each solved start to finish by one workgroup of a
// persistent kernel.
//
// A workgroup takes the next problem from a queue ordered by decreasing n*d (largest first) and
//   1. draws the SJLT of the problem (the counter-based draws of lsq_draw_sjlt), sorts the n*s
//      (target, row, sign) entries by target with a stable counting sort (per-wave histograms in
//      LDS, ballot multi-split scatter) and forms each row of S A as a sum over its bucket, in
//      draw order (no atomics on S A);
//   2. factors S A = Q R by blocked Householder QR: panels of 16 columns factored in registers
//      (one row per thread), the trailing update C <- C - V T^T V^T C on the FP64 matrix cores;
//      diag(R) > 0 and a relative pivot check;
//   3. forms W = R^{-1} blockwise (16 x 16 diagonal blocks by substitution, off-diagonal blocks on
//      the matrix cores);
//   4. runs PCG with the fixed preconditioner W W^T = (R^T R)^{-1}, inside FP64 iterative
//      refinement for the mixed form.  Each pass reads A once: q = A p and w = A^T q come from the
//      same rows while they sit in registers.
// No workgroup ever waits for another: the queue counter is the only shared state, and every loop
// is bounded, so the grid drains once the queue is empty.
//
// Each phase is a separate (not inlined) device function called once per problem, so that the
// register allocation of one phase does not constrain another; the workgroup's LDS is a file-scope
// object and global pointers carry the global address space, so those functions keep LDS and
// global instructions.
#include "internal.h"

#include <algorithm>

namespace lsq {

namespace {

constexpr int BT = 1024;          // threads per workgroup
constexpr int BNW = BT / 64;      // waves per workgroup
constexpr int B_DMAX = 256;       // largest d
constexpr int B_MMAX = 1024;      // largest m (one Householder row per thread)
constexpr int B_SEG = BNW;        // sort segments (one per wave)
constexpr int B_VR = B_DMAX + 2;  // stride of the per-wave reduction rows

#define LSQ_G __attribute__((address_space(1)))
#define LSQ_NOINLINE __attribute__((noinline))

typedef double lsq_b_d4 __attribute__((ext_vector_type(4)));
typedef double lsq_b_d2v __attribute__((ext_vector_type(2)));
typedef float lsq_b_f4v __attribute__((ext_vector_type(4)));

struct BatchLds {
  union {
    struct {
      uint32_t hist[B_SEG][B_MMAX];  // per-segment bucket counts, then running offsets
      uint32_t bstart[B_MMAX + 1];   // bucket starts in the sorted list
      uint32_t wtot[BNW];
      int draw_err;
    } sort;
    struct {
      double part[BT * 4];  // split-bucket partial sums of S A (overlays hist[] only)
    } red;
    struct {
      double T[16][16];  // compact-WY factor of the current panel
      double alpha[B_DMAX];
      double red[BNW * 16 + 16];
      double tot[16];
      double mx[BNW];
    } qr;
    struct {
      double red[BNW * B_VR];
      double x[B_DMAX], r[B_DMAX], p[B_DMAX], rh[B_DMAX], u[B_DMAX], dx[B_DMAX], w[B_DMAX];
      double sc[BNW + 4];
      double scal;
    } it;
  };
  int qidx;
};

__shared__ BatchLds g_L;

// Thread index behind an empty volatile asm: values derived from it are recomputed where they are
// used instead of being hoisted out of the problem and iteration loops.
__device__ __forceinline__ int b_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Wave-uniform copies (scalar registers) of values every lane already agrees on.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ lsq_b_d4 mfma16(double a, double b, lsq_b_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------------------------
// Loads of VEC contiguous elements of a row of A.  The vector form needs 16-byte alignment of the
// row start (A aligned, lda a multiple of VEC).  A chunk that straddles column d reads into the
// row's padding, which exists for every row but the last; the last row is therefore read from a
// zero-padded copy (`last`, made when the problem starts), selected by pointer so that the loads
// stay branch-free.  Elements at or past d are replaced by zero (the padding may hold anything).
// ---------------------------------------------------------------------------------------------
template <typename TA, int VEC>
struct RowLoad;

template <>
struct RowLoad<float, 4> {
  __device__ static void get(const float LSQ_G* p, float (&o)[4]) {
    const lsq_b_f4v v = __builtin_nontemporal_load((const lsq_b_f4v LSQ_G*)p);
    o[0] = v[0];
    o[1] = v[1];
    o[2] = v[2];
    o[3] = v[3];
  }
};
template <>
struct RowLoad<double, 2> {
  __device__ static void get(const double LSQ_G* p, double (&o)[2]) {
    const lsq_b_d2v v = __builtin_nontemporal_load((const lsq_b_d2v LSQ_G*)p);
    o[0] = v[0];
    o[1] = v[1];
  }
};
template <typename TA>
struct RowLoad<TA, 1> {
  __device__ static void get(const TA LSQ_G* p, TA (&o)[1]) { o[0] = __builtin_nontemporal_load(p); }
};

// chunk [c, c + VEC) of row `row`; `valid` false gives zeros (address clamped to the row start)
template <typename TA, int VEC>
__device__ __forceinline__ void load_chunk(const TA LSQ_G* A, int64_t lda, int64_t row, int64_t nlast,
                                           const TA LSQ_G* last, int c, int d, bool valid,
                                           TA (&o)[VEC]) {
  const TA LSQ_G* base = row == nlast ? last : A + row * lda;
  TA t[VEC];
  RowLoad<TA, VEC>::get(base + (valid ? c : 0), t);
#pragma unroll
  for (int e = 0; e < VEC; ++e) o[e] = (valid && c + e < d) ? t[e] : (TA)0;
}

// ---------------------------------------------------------------------------------------------
// Block-wide helpers (every thread receives the result).
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ double b_dot(const double* a, const double* b, int d, double* sc) {
  double s = 0.0;
  for (int c = b_tid(); c < d; c += BT) s = fma(a[c], b[c], s);
  double v[1] = {s};
  block_sum<BT, 1>(v, sc);
  return uni(v[0]);
}

__device__ __forceinline__ double b_max(double v, double* sc) {
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int tid = b_tid();
  if ((tid & 63) == 0) sc[tid >> 6] = v;
  __syncthreads();
  double m = 0.0;
  for (int q = 0; q < BNW; ++q) m = fmax(m, sc[q]);
  __syncthreads();
  return uni(m);
}

// 16 sums over the workgroup.  Within a wave a reduce-scatter butterfly (xor 8, 4, 2, 1 halve the
// values held per lane) leaves lane l with slot l & 15, then xor 16 and 32 finish the wave; 16
// threads add the per-wave rows in wave order.  The totals are also left in tot[].
__device__ __forceinline__ void block_sum16(double (&v)[16], double* red, double* tot) {
  const int tid = b_tid(), lane = tid & 63, wv = tid >> 6;
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
  double a8[8], a4[4], a2[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) a8[i] = (b3 ? v[i + 8] : v[i]) + __shfl_xor(b3 ? v[i] : v[i + 8], 8, 64);
#pragma unroll
  for (int i = 0; i < 4; ++i) a4[i] = (b2 ? a8[i + 4] : a8[i]) + __shfl_xor(b2 ? a8[i] : a8[i + 4], 4, 64);
#pragma unroll
  for (int i = 0; i < 2; ++i) a2[i] = (b1 ? a4[i + 2] : a4[i]) + __shfl_xor(b1 ? a4[i] : a4[i + 2], 2, 64);
  double a1 = (b0 ? a2[1] : a2[0]) + __shfl_xor(b0 ? a2[0] : a2[1], 1, 64);
  a1 += __shfl_xor(a1, 16, 64);
  a1 += __shfl_xor(a1, 32, 64);
  if (lane < 16) red[wv * 16 + lane] = a1;
  __syncthreads();
  if (tid < 16) {
    double t = 0.0;
    for (int q = 0; q < BNW; ++q) t += red[q * 16 + tid];
    tot[tid] = t;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = tot[i];
}

// ---------------------------------------------------------------------------------------------
// 1a. SJLT draws and the stable counting sort by target.  Keys are laid out entry-major: entry k
// of row j at position k n + j, the order of a scatter-add that adds entry 0 of every row, then
// entry 1, and so on.  On exit sorted[] holds row | sign << 31 bucket by bucket and
// g_L.sort.bstart[0..m] the bucket starts.  Returns 0 when a row exhausted its draw budget (the
// oracle raises in that case).
// ---------------------------------------------------------------------------------------------
LSQ_NOINLINE __device__ int b_sort(int64_t n, int m, int s, uint64_t seed, uint64_t t,
                                   uint32_t LSQ_G* keys, uint32_t LSQ_G* sorted) {
  auto& L = g_L.sort;
  const int tid = b_tid(), lane = tid & 63, wv = tid >> 6;
  const uint32_t thr = (uint32_t)((1ull << 32) % (uint64_t)m);
  if (tid == 0) L.draw_err = 0;
  for (int i = tid; i < B_SEG * m; i += BT) L.hist[i / m][i % m] = 0u;
  __syncthreads();
  // (a) draws: key = target | sign << 31
  for (int64_t j = tid; j < n; j += BT) {
    int cnt = 0;
    for (int c = 0; c < MAX_SJLT_WORDS / 4 && cnt < s; ++c) {
      const u64x4 w4 = philox4x64_10((uint64_t)j, TAG_SJLT, t, (uint64_t)c, seed, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint64_t wq = q == 0 ? w4.x : (q == 1 ? w4.y : (q == 2 ? w4.z : w4.w));
        uint32_t h;
        if (cnt < s && sjlt_propose(wq, (uint32_t)m, thr, &h)) {
          bool dup = false;
          for (int k = 0; k < cnt; ++k) dup |= (keys[(int64_t)k * n + j] & 0x3ffu) == h;
          if (!dup) {
            keys[(int64_t)cnt * n + j] = h | ((wq & 1ull) ? 0x80000000u : 0u);
            ++cnt;
          }
        }
      }
    }
    if (cnt < s) {
      for (int k = cnt; k < s; ++k) keys[(int64_t)k * n + j] = 0u;
      L.draw_err = 1;
    }
  }
  __syncthreads();
  // (b) per-segment histograms (segment q = positions [q len, (q + 1) len), walked by wave q)
  const int64_t P = (int64_t)s * n;
  const int64_t slen = (P + B_SEG - 1) / B_SEG;
  const int64_t s0 = min(P, (int64_t)wv * slen), s1 = min(P, s0 + slen);
  for (int64_t p = s0 + lane; p < s1; p += 64) atomicAdd(&L.hist[wv][keys[p] & 0x3ffu], 1u);
  __syncthreads();
  // (c) offsets: bucket-major, segment-minor exclusive scan
  uint32_t tot = 0;
  if (tid < m) {
    for (int q = 0; q < B_SEG; ++q) {
      const uint32_t c = L.hist[q][tid];
      L.hist[q][tid] = tot;
      tot += c;
    }
  }
  uint32_t inc = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(inc, off, 64);
    if (lane >= off) inc += o;
  }
  if (lane == 63) L.wtot[wv] = inc;
  __syncthreads();
  uint32_t wbase = 0;
  for (int q = 0; q < wv; ++q) wbase += L.wtot[q];
  const uint32_t excl = wbase + inc - tot;
  if (tid < m) {
    for (int q = 0; q < B_SEG; ++q) L.hist[q][tid] += excl;
    L.bstart[tid] = excl;
    if (tid == m - 1) L.bstart[m] = excl + tot;
  }
  __syncthreads();
  // (d) stable scatter: 64 entries at a time per wave, rank among equal targets from ballots
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t p0 = s0; p0 < s1; p0 += 64) {
    const int64_t p = p0 + lane;
    const bool valid = p < s1;
    const uint32_t key = valid ? keys[p] : 0u;
    const uint32_t h = key & 0x3ffu;
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 10; ++b) {
      const bool bit = (h >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      same &= bit ? bb : ~bb;
    }
    if (valid) {
      const uint32_t rank = (uint32_t)__popcll(same & below);
      const uint32_t cnt = (uint32_t)__popcll(same);
      const uint32_t at = L.hist[wv][h];
      const int64_t k = p / n, j = p - k * n;
      sorted[at + rank] = (uint32_t)j | (key & 0x80000000u);
      if (rank == cnt - 1) L.hist[wv][h] = at + cnt;
    }
  }
  __syncthreads();
  return uni(L.draw_err == 0 ? 1 : 0);
}

// ---------------------------------------------------------------------------------------------
// 1b. Segmented reduction of the sorted entries into S A (rows [0, m), columns [0, d), row stride
// dp), then zero padding of rows [m, mp) and columns [d, dp).  Bucket h holds the entries of
// target h in draw order; when m is small each bucket is split into F contiguous pieces summed by
// F lane groups and combined in piece order.  G lanes per row, NV chunks of VEC columns per lane.
// ---------------------------------------------------------------------------------------------
template <typename TA, int VEC, int G, int NV>
LSQ_NOINLINE __device__ void b_sjlt_reduce(const TA LSQ_G* __restrict__ A, int64_t lda, int64_t n,
                                           const TA LSQ_G* __restrict__ last, int d, int m, int mp,
                                           int dp, int s,
                                           const uint32_t LSQ_G* __restrict__ sorted,
                                           double LSQ_G* __restrict__ SA) {
  constexpr int NG = BT / G;
  constexpr int U = NV >= 4 ? 1 : 4 / NV;
  const double scale = 1.0 / sqrt((double)s);
  const int tid = b_tid();
  const int gl = tid % G, g = tid / G;
  int F = 1;
  while (F * 2 * m <= NG) F *= 2;
  const int TR = NG / F;
  const int64_t nlast = n - 1;
  int col[NV];
  bool cok[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    col[i] = (gl + G * i) * VEC;
    cok[i] = col[i] < d;
  }
  const uint32_t* bstart = g_L.sort.bstart;
  double* part = g_L.red.part;  // overlays only hist[], which is spent
  for (int h0 = 0; h0 < m; h0 += TR) {
    const int h = h0 + g / F, f = g % F;
    double acc[NV][VEC];
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[i][e] = 0.0;
    if (h < m) {
      const int64_t b0 = bstart[h], len = (int64_t)bstart[h + 1] - b0;
      const int64_t e0 = b0 + len * f / F, e1 = b0 + len * (f + 1) / F;
      for (int64_t e = e0; e < e1; e += U) {
        TA a[U][NV][VEC];
        double sg[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
          const bool ok = e + k < e1;
          const uint32_t key = sorted[ok ? e + k : e];  // e < e1 is a valid entry; masked below
          const int64_t j = (int64_t)(key & 0x7fffffffu);
          sg[k] = ok ? ((key >> 31) ? -scale : scale) : 0.0;
#pragma unroll
          for (int i = 0; i < NV; ++i)
            load_chunk<TA, VEC>(A, lda, j, nlast, last, col[i], d, ok && cok[i], a[k][i]);
        }
        // in entry order, so an unsplit bucket sums exactly like a sequential scatter-add
#pragma unroll
        for (int k = 0; k < U; ++k)
#pragma unroll
          for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int e2 = 0; e2 < VEC; ++e2)
              if (e + k < e1) acc[i][e2] += (double)a[k][i][e2] * sg[k];
      }
    }
    if (F == 1) {
      if (h < m) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
          for (int e = 0; e < VEC; ++e)
            if (col[i] + e < d) SA[(int64_t)h * dp + col[i] + e] = acc[i][e];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int e = 0; e < VEC; ++e) part[tid * (NV * VEC) + i * VEC + e] = acc[i][e];
      __syncthreads();
      if (f == 0 && h < m) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            double sum = 0.0;
            for (int q = 0; q < F; ++q) sum += part[((g + q) * G + gl) * (NV * VEC) + i * VEC + e];
            if (col[i] + e < d) SA[(int64_t)h * dp + col[i] + e] = sum;
          }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < (mp - m) * dp; i += BT) SA[(int64_t)m * dp + i] = 0.0;
  if (dp > d)
    for (int i = tid; i < m * (dp - d); i += BT) SA[(int64_t)(i / (dp - d)) * dp + d + i % (dp - d)] = 0.0;
  __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// 2. Householder QR of X = S A (mp x dp row-major, zero padded, m >= d), in place: on exit the
// upper triangle of X[0:d, 0:d] holds R up to row signs and g_L.qr.alpha[] its diagonal.
// ---------------------------------------------------------------------------------------------
LSQ_NOINLINE __device__ void b_qr(double LSQ_G* X, int m, int d, int mp, int dp, double LSQ_G* V) {
  auto& L = g_L.qr;
  const int tid = b_tid(), lane = tid & 63, wv = tid >> 6;
  const int r = tid;  // one row per thread (mp <= BT)
  const int li = lane & 15, lk = lane >> 4;
  for (int k0 = 0; k0 < d; k0 += 16) {
    const int bw = min(16, d - k0);
    double P[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) P[j] = (r >= k0 && r < m) ? X[(int64_t)r * dp + k0 + j] : 0.0;
    if (tid < 256) L.T[tid >> 4][tid & 15] = 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (j < bw) {
        const int diag = k0 + j;
        double s2[2] = {r > diag ? P[j] * P[j] : 0.0, r == diag ? P[j] : 0.0};
        block_sum<BT, 2>(s2, L.red);
        const double sigma = s2[0], x0 = s2[1];
        const double nrm = sqrt(x0 * x0 + sigma);
        const double alpha = nrm == 0.0 ? 0.0 : (x0 >= 0.0 ? -nrm : nrm);
        const double v0 = x0 - alpha;
        const double vtv = sigma + v0 * v0;
        const double tau = vtv > 0.0 ? 2.0 / vtv : 0.0;
        // rows above the diagonal hold final R entries of this panel column
        if (r >= k0 && r < diag) X[(int64_t)r * dp + diag] = P[j];
        if (r == diag) {
          X[(int64_t)diag * dp + diag] = alpha;
          L.alpha[diag] = alpha;
        }
        if (r < diag) P[j] = 0.0;
        else if (r == diag) P[j] = v0;
        // w[jj] = v_j^T col_jj (jj > j: update) or v_jj^T v_j (jj < j: column j of T)
        double w16[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) w16[jj] = jj == j ? 0.0 : P[j] * P[jj];
        block_sum16(w16, L.red, L.tot);
        if (tid == 0) {
          // T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j);  T[j, j] = tau_j
          for (int a = 0; a < j; ++a) {
            double acc = 0.0;
            for (int b = a; b < j; ++b) acc += L.T[a][b] * L.tot[b];
            L.T[a][j] = -tau * acc;
          }
          L.T[j][j] = tau;
        }
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
          if (jj > j) P[jj] -= tau * w16[jj] * P[j];
        __syncthreads();  // tot[] and red[] are rewritten by the next column
      }
    }
    if (r < mp) {
#pragma unroll
      for (int j = 0; j < 16; ++j) V[(int64_t)r * 16 + j] = P[j];
    }
    __syncthreads();
    // trailing update, one 16-column tile per wave: Z = V^T C, Y = T^T Z, C -= V Y
    const int nct = dp / 16 - (k0 / 16 + 1);
    for (int ct = wv; ct < nct; ct += BNW) {
      const int c0 = k0 + 16 + ct * 16;
      lsq_b_d4 Z = {0.0, 0.0, 0.0, 0.0};
      for (int rr = k0; rr < mp; rr += 16) {
        double av[4], bv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          av[q] = V[(int64_t)(rr + 4 * q + lk) * 16 + li];
          bv[q] = X[(int64_t)(rr + 4 * q + lk) * dp + c0 + li];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Z = mfma16(av[q], bv[q], Z);
      }
      lsq_b_d4 Y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q) Y = mfma16(L.T[4 * q + lk][li], Z[q], Y);
      for (int rb = k0; rb < mp; rb += 16) {
        lsq_b_d4 C;
        double av[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) C[v] = X[(int64_t)(rb + lk + 4 * v) * dp + c0 + li];
#pragma unroll
        for (int q = 0; q < 4; ++q) av[q] = -V[(int64_t)(rb + li) * 16 + 4 * q + lk];
#pragma unroll
        for (int q = 0; q < 4; ++q) C = mfma16(av[q], Y[q], C);
#pragma unroll
        for (int v = 0; v < 4; ++v) X[(int64_t)(rb + lk + 4 * v) * dp + c0 + li] = C[v];
      }
    }
    __syncthreads();
  }
}

// R (dp x dp, row-major) = diag(sign(alpha)) triu(X), identity on the padding; returns 0 when a
// pivot is not above 8 d eps max |alpha| (numerically rank deficient S A).  Optional copy Ru (d x d).
LSQ_NOINLINE __device__ int b_finish_r(const double LSQ_G* X, int d, int dp, double LSQ_G* R,
                                       double LSQ_G* Ru) {
  auto& L = g_L.qr;
  const int tid = b_tid();
  double mx = 0.0;
  for (int k = tid; k < d; k += BT) mx = fmax(mx, fabs(L.alpha[k]));
  mx = b_max(mx, L.mx);
  const double thr = 8.0 * (double)d * 2.220446049250313e-16 * mx;
  double bad = 0.0;
  for (int k = tid; k < d; k += BT) bad = fmax(bad, (fabs(L.alpha[k]) > thr) ? 0.0 : 1.0);
  bad = b_max(bad, L.mx);
  for (int i = tid; i < dp * dp; i += BT) {
    const int a = i / dp, b = i % dp;
    double v;
    if (a >= d || b >= d) v = (a == b) ? 1.0 : 0.0;
    else if (b < a) v = 0.0;
    else v = L.alpha[a] < 0.0 ? -X[(int64_t)a * dp + b] : X[(int64_t)a * dp + b];
    R[i] = v;
    if (Ru && a < d && b < d) Ru[(int64_t)a * d + b] = v;
  }
  __syncthreads();
  return bad == 0.0 ? 1 : 0;
}

// ---------------------------------------------------------------------------------------------
// 3. W = R^{-1} (dp x dp upper) and W^T, blockwise with 16 x 16 blocks.
// ---------------------------------------------------------------------------------------------
LSQ_NOINLINE __device__ void b_trinv(const double LSQ_G* R, int dp, double LSQ_G* W, double LSQ_G* WT) {
  const int tid = b_tid(), lane = tid & 63, wv = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nb = dp / 16;
  // zero the blocks below the diagonal
  for (int i = tid; i < dp * dp; i += BT) {
    const int a = i / dp, b = i % dp;
    if (a / 16 > b / 16) {
      W[i] = 0.0;
      WT[(int64_t)b * dp + a] = 0.0;
    }
  }
  // diagonal blocks: lane j < 16 of wave I computes column j of (R_II)^{-1} by back substitution
  if (wv < nb && lane < 16) {
    const int o = wv * 16, j = lane;
    double wc[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int k = i + 1; k < 16; ++k) s -= R[(int64_t)(o + i) * dp + o + k] * wc[k];
      wc[i] = i > j ? 0.0 : s / R[(int64_t)(o + i) * dp + o + i];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      W[(int64_t)(o + i) * dp + o + j] = wc[i];
      WT[(int64_t)(o + j) * dp + o + i] = wc[i];
    }
  }
  __syncthreads();
  // block column J (one wave): W_IJ = -W_II sum_{K=I+1..J} R_IK W_KJ for I = J-1 down to 0
  const int J = wv;
  if (J >= 1 && J < nb) {
    for (int I = J - 1; I >= 0; --I) {
      lsq_b_d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int K = I + 1; K <= J; ++K) {
        double av[4], bv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          av[q] = R[(int64_t)(16 * I + li) * dp + 16 * K + 4 * q + lk];
          bv[q] = W[(int64_t)(16 * K + 4 * q + lk) * dp + 16 * J + li];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc = mfma16(av[q], bv[q], acc);
      }
      lsq_b_d4 res = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < 4; ++q)
        res = mfma16(-W[(int64_t)(16 * I + li) * dp + 16 * I + 4 * q + lk], acc[q], res);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * I + lk + 4 * v, cl = 16 * J + li;
        W[(int64_t)row * dp + cl] = res[v];
        WT[(int64_t)cl * dp + row] = res[v];
      }
      // the next block row reads these entries back (other lanes of this wave)
      __threadfence_block();
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// 4. Iteration.
// Fused pass over all n rows of one problem by the whole workgroup:
//   MODE 0: q_j = a_j . v,          w = sum_j q_j a_j, scal = sum_j q_j^2   (H v and v^T H v)
//   MODE 1: q_j = y_j - a_j . v,    w = sum_j q_j a_j, scal = sum_j q_j^2   (A^T (y - A v))
// G lanes per row, NV chunks of VEC columns per lane (column of chunk i of lane g: (g + G i) VEC),
// FP64 arithmetic, U rows in flight per lane group.  v, w, scal, red in LDS.
// ---------------------------------------------------------------------------------------------
template <typename TA, int VEC, int G, int NV, int MODE>
__device__ __forceinline__ void b_fused(const TA LSQ_G* __restrict__ A, int64_t lda, int64_t n,
                                        const TA LSQ_G* __restrict__ last, int d,
                                        const double LSQ_G* __restrict__ y, const double* v, double* w,
                                        double* scal, double* red, bool has_last) {
  constexpr int RPW = 64 / G;    // rows per wave per step
  constexpr int RS = BNW * RPW;  // rows per workgroup step
  constexpr int U = NV >= 8 ? 1 : 8 / NV;  // rows in flight per lane group (U NV loads per lane)
  (void)last;
  const int tid = b_tid(), lane = tid & 63, wv = tid >> 6;
  const int gl = lane % G, rw = lane / G;
  double pv[NV][VEC], acc[NV][VEC];
  int col[NV];
  bool em[NV][VEC];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int c = (gl + G * i) * VEC;
    col[i] = c < d ? c : 0;  // chunks past d read the row start and are masked
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      em[i][e] = c + e < d;
      pv[i][e] = em[i][e] ? v[c + e] : 0.0;
      acc[i][e] = 0.0;
    }
  }
  double ss = 0.0;
  // rows [0, nm) are read with whole chunks; when d is not a multiple of VEC the matrix's last row's
  // straddling chunk would run past the matrix, so that row (when this block holds it) is read
  // element-wise at the end
  const int nm = (VEC > 1 && d % VEC != 0 && has_last) ? (int)n - 1 : (int)n;
  const int row0 = wv * RPW + rw;
  const int64_t kstep = (int64_t)RS * lda;
  // one row of the lane group: masked chunk values -> q -> accumulators
  auto row = [&](TA (&ak)[NV][VEC], double yk, bool ok) {
    double q = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        ak[i][e] = em[i][e] ? ak[i][e] : (TA)0;
        q = fma((double)ak[i][e], pv[i][e], q);
      }
    q = grp_sum<G>(q);
    if (MODE == 1) q = yk - q;
    q = ok ? q : 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[i][e] = fma(q, (double)ak[i][e], acc[i][e]);
    if (gl == 0) ss = fma(q, q, ss);
  };
  // Whole blocks of U * RS rows, loads rotated through the registers: as soon as row k of a block
  // is consumed its registers receive row k of the next block, so every lane keeps about U loads
  // in flight while it computes (the last block re-reads itself instead of running past the end).
  const int nblk = nm / (U * RS);
  const int64_t bstep = (int64_t)U * RS * lda;
  if (nblk > 0) {
    TA a[U][NV][VEC];
    double yk[U];
    const TA LSQ_G* pr = A + (int64_t)row0 * lda;
#pragma unroll
    for (int k = 0; k < U; ++k) {
#pragma unroll
      for (int i = 0; i < NV; ++i) RowLoad<TA, VEC>::get(pr + k * kstep + col[i], a[k][i]);
      yk[k] = MODE == 1 ? y[row0 + k * RS] : 0.0;
    }
    for (int b = 0; b < nblk; ++b) {
      const bool more = b + 1 < nblk;
      const TA LSQ_G* pn = more ? pr + bstep : pr;
      const int yn = (more ? b + 1 : b) * U * RS + row0;
#pragma unroll
      for (int k = 0; k < U; ++k) {
        row(a[k], yk[k], true);
#pragma unroll
        for (int i = 0; i < NV; ++i) RowLoad<TA, VEC>::get(pn + k * kstep + col[i], a[k][i]);
        yk[k] = MODE == 1 ? y[yn + k * RS] : 0.0;
      }
      pr = pn;
    }
  }
  // the remaining rows, U row steps at a time with masks (out-of-range rows read row 0)
  for (int r0 = nblk * U * RS; r0 < nm; r0 += U * RS) {
    TA a[U][NV][VEC];
    double yk[U];
    bool ok[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int r = r0 + k * RS + row0;
      ok[k] = r < nm;
      const TA LSQ_G* pk = A + (int64_t)(ok[k] ? r : 0) * lda;
#pragma unroll
      for (int i = 0; i < NV; ++i) RowLoad<TA, VEC>::get(pk + col[i], a[k][i]);
      yk[k] = MODE == 1 ? y[ok[k] ? r : 0] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) row(a[k], yk[k], ok[k]);
  }
  if (nm < n) {
    // last row by the first lane group of wave 0, element loads
    const bool act = wv == 0 && rw == 0;
    const TA LSQ_G* pl = A + (n - 1) * lda;
    TA a[NV][VEC];
    double q = 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        a[i][e] = (act && em[i][e]) ? pl[col[i] + e] : (TA)0;
        q = fma((double)a[i][e], pv[i][e], q);
      }
    q = grp_sum<G>(q);
    if (MODE == 1) q = (act ? y[n - 1] : 0.0) - q;
    q = act ? q : 0.0;
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[i][e] = fma(q, (double)a[i][e], acc[i][e]);
    if (gl == 0) ss = fma(q, q, ss);
  }
  // lanes with equal gl hold the same columns: fold them, then one row of LDS per wave
#pragma unroll
  for (int off = G; off < 64; off <<= 1)
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[i][e] += __shfl_xor(acc[i][e], off, 64);
  ss = wave_sum(ss);
  if (rw == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        if (em[i][e]) red[wv * B_VR + (gl + G * i) * VEC + e] = acc[i][e];
  }
  if (lane == 0) red[wv * B_VR + B_DMAX + 1] = ss;
  __syncthreads();
  for (int c = tid; c < d; c += BT) {
    double s = 0.0;
    for (int q = 0; q < BNW; ++q) s += red[q * B_VR + c];
    w[c] = s;
  }
  if (tid == BT - 1) {
    double s = 0.0;
    for (int q = 0; q < BNW; ++q) s += red[q * B_VR + B_DMAX + 1];
    *scal = s;
  }
  __syncthreads();
}

// rh = W (W^T r): two triangular GEMVs, a wave per output entry, four rows in flight per wave.
__device__ __forceinline__ void b_precond(const double LSQ_G* W, const double LSQ_G* WT, int d, int dp,
                                          const double* r, double* u, double* rh) {
  const int tid = b_tid(), lane = tid & 63, wv = tid >> 6;
  for (int i0 = wv; i0 < d; i0 += 4 * BNW) {
    double s[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + q * BNW;
      s[q] = 0.0;
      if (i < d)
        for (int k = lane; k <= i; k += 64) s[q] = fma(WT[(int64_t)i * dp + k], r[k], s[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double t = wave_sum(s[q]);
      const int i = i0 + q * BNW;
      if (lane == 0 && i < d) u[i] = t;
    }
  }
  __syncthreads();
  for (int i0 = wv; i0 < d; i0 += 4 * BNW) {
    double s[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + q * BNW;
      s[q] = 0.0;
      if (i < d)
        for (int k = i + lane; k < d; k += 64) s[q] = fma(W[(int64_t)i * dp + k], u[k], s[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double t = wave_sum(s[q]);
      const int i = i0 + q * BNW;
      if (lane == 0 && i < d) rh[i] = t;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------------
// Gangs: a problem above the gang size is solved by K workgroups together (K fixed by n d, so the
// result does not depend on the number of workgroups).  Member r streams rows [n r / K, n (r + 1) / K)
// in every pass and writes its partial A^T(.) and its sum of squares; after a barrier every member adds
// the K partials in rank order, so all members hold the same sums and take the same PCG steps.  The
// barrier is a counter in device memory (release fence, atomic add, acquire spin); its wait is bounded,
// and a wait that runs out marks the gang broken (the problem then reports LSQ_ERR_HIP) instead of
// hanging.  The K member tasks of a gang sit next to each other in the queue, so with at least K
// workgroups they are always taken by K workgroups that run at the same time.
// ---------------------------------------------------------------------------------------------
struct Gang {
  int K, rank, epoch;
  int LSQ_G* st;      // [0] barrier count, [1] leader slot, [2] setup status, [3] broken
  double LSQ_G* part;  // 2 x KMAX rows of pstride doubles
  int64_t pstride;
};

constexpr int B_GANG_SPIN = 1 << 22;  // barrier polls before the gang is declared broken

__device__ __forceinline__ void gang_barrier(Gang& g) {
  g.epoch += 1;  // every thread keeps the same count
  __threadfence();
  __syncthreads();
  if (b_tid() == 0) {
    atomicAdd((int*)g.st, 1);
    const int target = g.K * g.epoch;
    int spins = 0;
    while (__hip_atomic_load((int*)g.st, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      // a broken gang no longer waits (its result is discarded)
      if (__hip_atomic_load((int*)g.st + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      __builtin_amdgcn_s_sleep(8);
      if (++spins >= B_GANG_SPIN) {
        __hip_atomic_store((int*)g.st + 3, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __threadfence();
  __syncthreads();
}

// w (d values in LDS) and *scal of this member -> the sums over the gang's members, in rank order.
__device__ __forceinline__ void gang_reduce(Gang& g, double* w, double* scal, int d) {
  const int tid = b_tid();
  double LSQ_G* mine = g.part + ((int64_t)((g.epoch + 1) & 1) * BATCH_GANG_KMAX + g.rank) * g.pstride;
  for (int c = tid; c < d; c += BT) mine[c] = w[c];
  if (tid == BT - 1) mine[d] = *scal;
  gang_barrier(g);
  const double LSQ_G* all = g.part + (int64_t)(g.epoch & 1) * BATCH_GANG_KMAX * g.pstride;
  for (int c = tid; c <= d; c += BT) {
    double s = all[c];
    for (int k = 1; k < g.K; ++k) s += all[k * g.pstride + c];
    if (c < d)
      w[c] = s;
    else
      *scal = s;
  }
  __syncthreads();
}

// PCG (and the refinement loop of the mixed form) for one problem, with the stop rule of the
// single-problem solver: proxy 4 sqrt(rho_t / rho_0) <= tol.  Result written to *out.  With a gang,
// A and y are this member's row block (n rows, has_last when it holds the matrix's last row), every
// pass is followed by the gang's reduction, and only the leader writes x and *out.
struct PcgArgs {
  int64_t n, lda;
  int d, dp, mixed, max_iter, max_refine;
  double tol;
  bool has_last;
};

template <typename TA, int VEC, int G, int NV>
LSQ_NOINLINE __device__ void b_pcg(const TA LSQ_G* A, const TA LSQ_G* last, const double LSQ_G* yg,
                                   double LSQ_G* xg,
                                   const double LSQ_G* W, const double LSQ_G* WT, PcgArgs pa,
                                   BatchOut LSQ_G* out, Gang* gang) {
  auto& L = g_L.it;
  const int tid = b_tid();
  const int d = pa.d;
  double* x = L.x;
  double* r = L.r;
  double* p = L.p;
  double* rh = L.rh;
  double* dx = L.dx;
  double* w = L.w;
  for (int c = tid; c < d; c += BT) {
    x[c] = xg[c];
    dx[c] = 0.0;
  }
  __syncthreads();
  const int outer = pa.mixed ? pa.max_refine : 1;
  int total = 0, refinements = 0, status = 0;
  double est = 0.0, rho_b = -1.0;
  bool inner_done = false;
  for (int k = 0; k < outer; ++k) {
    b_fused<TA, VEC, G, NV, 1>(A, pa.lda, pa.n, last, d, yg, x, r, &L.scal, L.red, pa.has_last);
    if (gang) gang_reduce(*gang, r, &L.scal, d);
    b_precond(W, WT, d, pa.dp, r, L.u, rh);
    double rho = b_dot(r, rh, d, L.sc);
    double tol_in;
    if (pa.mixed) {
      if (rho_b < 0.0) rho_b = rho;
      est = rho_b > 0.0 ? 4.0 * sqrt(fmax(rho, 0.0) / rho_b) : 0.0;
      if (est <= pa.tol) break;
      refinements += 1;
      // the inner stop rule bounds the error of the correction relative to the current error
      const double rel = fmax(est / 4.0, 1e-300);
      tol_in = fmax(0.9 * pa.tol / rel, 1e-13);
    } else {
      tol_in = pa.tol;
    }
    if (!isfinite(rho)) {
      status = (int)LSQ_ERR_NONFINITE;
      break;
    }
    // the iterate being advanced: the correction dx (mixed) or x itself
    double* tgt = pa.mixed ? dx : x;
    for (int c = tid; c < d; c += BT) {
      p[c] = rh[c];
      dx[c] = 0.0;
    }
    __syncthreads();
    const double rho0 = rho;
    double proxy = rho0 > 0.0 ? 4.0 : 0.0;
    inner_done = !(rho0 > 0.0);
    int it = 0;
    while (!inner_done && it < pa.max_iter) {
      b_fused<TA, VEC, G, NV, 0>(A, pa.lda, pa.n, last, d, nullptr, p, w, &L.scal, L.red, pa.has_last);
      if (gang) gang_reduce(*gang, w, &L.scal, d);
      const double pHp = uni(L.scal);
      if (!(pHp > 0.0) || !isfinite(pHp)) {
        status = isfinite(pHp) ? (int)LSQ_ERR_RANK : (int)LSQ_ERR_NONFINITE;
        break;
      }
      const double alpha = rho / pHp;
      for (int c = tid; c < d; c += BT) {
        tgt[c] = fma(alpha, p[c], tgt[c]);
        r[c] = fma(-alpha, w[c], r[c]);
      }
      __syncthreads();
      b_precond(W, WT, d, pa.dp, r, L.u, rh);
      const double rho_new = b_dot(r, rh, d, L.sc);
      const double beta = rho_new / rho;
      for (int c = tid; c < d; c += BT) p[c] = fma(beta, p[c], rh[c]);
      __syncthreads();
      ++it;
      proxy = 4.0 * sqrt(fmax(rho_new, 0.0) / rho0);
      rho = rho_new;
      if (!isfinite(rho_new)) {
        status = (int)LSQ_ERR_NONFINITE;
        break;
      }
      if (proxy <= tol_in) inner_done = true;
    }
    total += it;
    if (!pa.mixed) est = proxy;
    if (status) break;
    if (pa.mixed) {
      for (int c = tid; c < d; c += BT) x[c] += dx[c];
      __syncthreads();
    }
  }
  const bool lead = !gang || gang->rank == 0;
  if (lead)
    for (int c = tid; c < d; c += BT) xg[c] = x[c];
  const bool conv = pa.mixed ? (est <= pa.tol) : inner_done;
  if (status == 0 && !conv) status = (int)LSQ_ERR_NOT_CONVERGED;
  if (gang && __hip_atomic_load((const int*)gang->st + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    status = (int)LSQ_ERR_HIP;  // a gang barrier ran out of time: the sums are not to be trusted
  if (lead && tid == 0) {
    out->status = status;
    out->iters = total;
    out->refinements = refinements;
    out->pad = 0;
    out->est = est;
  }
  __syncthreads();
}

// Column mapping of a problem: VEC elements per load, G lanes per row, NV chunks per lane.
struct Map {
  int vec, g, nv;
};

__device__ __forceinline__ Map choose_map(int a_f32, const void* A, int64_t lda, int d) {
  // few lanes per row (cheap row sums, all on the VALU) and up to 2 (FP32) or 4 (FP64) chunks per
  // lane, which keeps the row data, the accumulators and v in registers
  const bool al = ((uintptr_t)A % 16) == 0;
  Map mp;
  if (a_f32 && al && lda % 4 == 0) {
    const int c = (d + 3) / 4;
    mp.vec = 4;
    mp.g = c <= 4 ? 4 : (c <= 8 ? 8 : (c <= 32 ? 16 : 32));
    mp.nv = c <= 16 ? 1 : 2;
  } else if (!a_f32 && al && lda % 2 == 0) {
    const int c = (d + 1) / 2;
    mp.vec = 2;
    mp.g = c <= 8 ? 8 : (c <= 64 ? 16 : 32);
    mp.nv = c <= 16 ? 1 : (c <= 32 ? 2 : 4);
  } else {
    mp.vec = 1;
    mp.g = 64;
    mp.nv = 4;
  }
  return mp;
}

#define LSQ_B_FOR_MAPS(TA, MACRO)                  \
  if constexpr (sizeof(TA) == 4) {                \
    if (mapv.vec == 4) {                          \
      if (mapv.g == 4)                            \
        MACRO(TA, 4, 4, 1)                        \
      else if (mapv.g == 8)                       \
        MACRO(TA, 4, 8, 1)                        \
      else if (mapv.g == 16 && mapv.nv == 1)      \
        MACRO(TA, 4, 16, 1)                       \
      else if (mapv.g == 16)                      \
        MACRO(TA, 4, 16, 2)                       \
      else                                        \
        MACRO(TA, 4, 32, 2)                       \
    } else {                                      \
      MACRO(TA, 1, 64, 4)                         \
    }                                             \
  } else {                                        \
    if (mapv.vec == 2) {                          \
      if (mapv.g == 8)                            \
        MACRO(TA, 2, 8, 1)                        \
      else if (mapv.g == 16 && mapv.nv == 1)      \
        MACRO(TA, 2, 16, 1)                       \
      else if (mapv.g == 16 && mapv.nv == 2)      \
        MACRO(TA, 2, 16, 2)                       \
      else if (mapv.g == 16)                      \
        MACRO(TA, 2, 16, 4)                       \
      else                                        \
        MACRO(TA, 2, 32, 4)                       \
    } else {                                      \
      MACRO(TA, 1, 64, 4)                         \
    }                                             \
  }

// Iterations of problem pd on this workgroup's row block (the whole matrix when gang is null).
__device__ __forceinline__ void b_iterate(const BatchArgs& a, const BatchDesc& pd, const Map& mapv,
                                          const double LSQ_G* W, const double LSQ_G* WT, double LSQ_G* last,
                                          BatchOut LSQ_G* out, Gang* gang) {
  const int d = pd.d;
  const int K = gang ? gang->K : 1, rank = gang ? gang->rank : 0;
  const int64_t r0 = pd.n * rank / K, r1 = pd.n * (rank + 1) / K;
  PcgArgs pa;
  pa.n = r1 - r0;
  pa.lda = pd.lda;
  pa.d = d;
  pa.dp = (d + 15) & ~15;
  pa.mixed = a.mixed;
  pa.max_iter = a.max_iter;
  pa.max_refine = a.max_refine;
  pa.tol = a.tol;
  pa.has_last = rank == K - 1;
#define LSQ_B_PCG(T_, V_, G_, N_)                                                                       \
  b_pcg<T_, V_, G_, N_>((const T_ LSQ_G*)pd.A + r0 * pd.lda, (const T_ LSQ_G*)last,                     \
                        (const double LSQ_G*)pd.y + r0, (double LSQ_G*)pd.x, W, WT, pa, out, gang);
  if (pd.a_f32) {
    LSQ_B_FOR_MAPS(float, LSQ_B_PCG)
  } else {
    LSQ_B_FOR_MAPS(double, LSQ_B_PCG)
  }
#undef LSQ_B_PCG
}

__device__ __forceinline__ void b_solve(const BatchArgs& a, const BatchTask tk, int slot) {
  const uint64_t t_start = wall_clock64();
  const int q = tk.q;
  const BatchDesc pd = a.descs[q];
  const int d = pd.d, m = pd.m;
  const int dp = (d + 15) & ~15, mp = (m + 15) & ~15;
  BatchOut LSQ_G* out = (BatchOut LSQ_G*)(a.out + pd.idx);
  const Map mapv = choose_map(pd.a_f32, pd.A, pd.lda, d);
  Gang gang;
  Gang* gp = nullptr;
  if (tk.K > 1) {
    gang.K = tk.K;
    gang.rank = tk.rank;
    gang.epoch = 0;
    gang.st = (int LSQ_G*)(a.gstate + 4 * (int64_t)tk.gang);
    gang.part = (double LSQ_G*)(a.gpart + (int64_t)tk.gang * 2 * BATCH_GANG_KMAX * a.gpart_stride);
    gang.pstride = a.gpart_stride;
    gp = &gang;
  }
  if (gp && tk.rank > 0) {
    // a member: the leader's factorization, then this member's rows
    gang_barrier(gang);
    const int ok = __hip_atomic_load((const int*)gang.st + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int lslot = __hip_atomic_load((const int*)gang.st + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ok != 1) return;  // the leader reports the failure
    const double LSQ_G* W = (const double LSQ_G*)(a.W + (int64_t)lslot * a.r_stride);
    const double LSQ_G* WT = (const double LSQ_G*)(a.WT + (int64_t)lslot * a.r_stride);
    b_iterate(a, pd, mapv, W, WT, (double LSQ_G*)(a.last + (int64_t)slot * a.last_stride), out, gp);
    return;
  }
  uint32_t LSQ_G* keys = (uint32_t LSQ_G*)(a.keys + (int64_t)slot * a.keys_stride);
  uint32_t LSQ_G* sorted = (uint32_t LSQ_G*)(a.sorted + (int64_t)slot * a.keys_stride);
  double LSQ_G* SA = (double LSQ_G*)(a.SA + (int64_t)slot * a.sa_stride);
  double LSQ_G* V = (double LSQ_G*)(a.V + (int64_t)slot * a.v_stride);
  double LSQ_G* R = (double LSQ_G*)(a.R + (int64_t)slot * a.r_stride);
  double LSQ_G* W = (double LSQ_G*)(a.W + (int64_t)slot * a.r_stride);
  double LSQ_G* WT = (double LSQ_G*)(a.WT + (int64_t)slot * a.r_stride);
  // zero-padded copy of the last row of A (see load_chunk)
  double LSQ_G* last = (double LSQ_G*)(a.last + (int64_t)slot * a.last_stride);
  for (int c = b_tid(); c < B_DMAX; c += BT) {
    if (pd.a_f32) {
      const float LSQ_G* Af = (const float LSQ_G*)pd.A + (pd.n - 1) * pd.lda;
      ((float LSQ_G*)last)[c] = c < d ? Af[c] : 0.0f;
    } else {
      const double LSQ_G* Ad = (const double LSQ_G*)pd.A + (pd.n - 1) * pd.lda;
      last[c] = c < d ? Ad[c] : 0.0;
    }
  }
  if (gp && b_tid() == 0) gang.st[1] = slot;  // published by the barrier after the factorization
  __syncthreads();
  if (b_tid() == 0) out->t_start = t_start;
  // 1. sketch
  const int drew = b_sort(pd.n, m, pd.s, pd.seed, pd.t, keys, sorted);
#define LSQ_B_RED(T_, V_, G_, N_) \
  b_sjlt_reduce<T_, V_, G_, N_>((const T_ LSQ_G*)pd.A, pd.lda, pd.n, (const T_ LSQ_G*)last, d, m, mp, dp, \
                                pd.s, sorted, SA);
  if (pd.a_f32) {
    LSQ_B_FOR_MAPS(float, LSQ_B_RED)
  } else {
    LSQ_B_FOR_MAPS(double, LSQ_B_RED)
  }
#undef LSQ_B_RED
  if (b_tid() == 0) out->t_sketch = wall_clock64();
  // 2. factor
  b_qr(SA, m, d, mp, dp, V);
  const int full_rank = b_finish_r(SA, d, dp, R, (double LSQ_G*)pd.R);
  if (!drew || !full_rank) {
    if (b_tid() == 0) {
      out->status = drew ? (int)LSQ_ERR_RANK : (int)LSQ_ERR_INVALID_ARG;
      out->iters = 0;
      out->refinements = 0;
      out->pad = 0;
      out->est = 0.0;
      out->t_factor = out->t_end = wall_clock64();
    }
    if (gp) {
      if (b_tid() == 0) gang.st[2] = 2;
      gang_barrier(gang);  // releases the members, who then leave
    }
    __syncthreads();
    return;
  }
  // 3. W = R^{-1};  4. iterate
  b_trinv(R, dp, W, WT);
  if (b_tid() == 0) out->t_factor = wall_clock64();
  if (gp) {
    if (b_tid() == 0) gang.st[2] = 1;
    gang_barrier(gang);  // W, W^T and the leader's slot to the members
  }
  b_iterate(a, pd, mapv, W, WT, last, out, gp);
  if (b_tid() == 0) out->t_end = wall_clock64();
}

}  // namespace

int g_batched_slots = 0;
int64_t g_batched_gang_unit = 8 << 20;

__global__ __launch_bounds__(BT) void k_batched(const BatchArgs a) {
  const int ntasks = a.ntasks;
  for (;;) {
    if (b_tid() == 0) g_L.qidx = atomicAdd(a.queue, 1);
    __syncthreads();
    const int q = uni(g_L.qidx);
    __syncthreads();
    if (q >= ntasks) break;
    b_solve(a, a.tasks[q], blockIdx.x);
  }
}

__global__ void k_batch_reset(int* queue, BatchOut* out, int count, int* gstate, int ngangs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 4 * ngangs) gstate[i] = 0;
  if (i == 0) *queue = 0;
  if (i < count) {
    out[i].status = -1;
    out[i].iters = 0;
    out[i].refinements = 0;
    out[i].pad = 0;
    out[i].est = 0.0;
    out[i].t_start = out[i].t_sketch = out[i].t_factor = out[i].t_end = 0;
  }
}

void batched_launch(hipStream_t st, const BatchArgs& a, int slots) {
  const int nr = std::max(a.count, 4 * a.ngangs);
  hipLaunchKernelGGL(k_batch_reset, dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, st, a.queue, a.out,
                     a.count, a.gstate, a.ngangs);
  hipLaunchKernelGGL(k_batched, dim3((unsigned)slots), dim3(BT), 0, st, a);
}

}  // namespace lsq
