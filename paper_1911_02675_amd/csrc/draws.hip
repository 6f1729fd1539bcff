// Random draws of the three embeddings (Section 2), as pure functions of (seed, t, index).
// SRHT row subset: "uniformly at random without replacement" is realised as the m smallest
// (64-bit key, row) pairs, found by a 4-digit radix select and an order-preserving compaction.
#include "internal.h"

namespace lsq {

// ------------------------------------------------------------------------------------------------
// SRHT signs and keys
// ------------------------------------------------------------------------------------------------
__global__ void k_srht_draw(uint64_t seed, uint64_t t, int64_t N, int8_t* __restrict__ signs,
                            uint64_t* __restrict__ keys) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const u64x4 w = philox4x64_10((uint64_t)j, TAG_SRHT, t, 0, seed, 0);
  if (signs) signs[j] = (w.x >> 63) ? (int8_t)-1 : (int8_t)1;
  if (keys) keys[j] = w.y;
}

void launch_srht_draw(hipStream_t st, uint64_t seed, uint64_t t, int64_t N, int8_t* signs,
                      uint64_t* keys) {
  const int nt = 256;
  hipLaunchKernelGGL(k_srht_draw, dim3((unsigned)((N + nt - 1) / nt)), dim3(nt), 0, st, seed, t, N,
                     signs, keys);
}

// ------------------------------------------------------------------------------------------------
// Block-level exclusive scan of one int per thread (NT threads).
// ------------------------------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(inc, off, 64);
    if (lane >= off) inc += o;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < NT / 64; ++w) {
      const int c = sh[w];
      sh[w] = run;
      run += c;
    }
    sh[NT / 64] = run;
  }
  __syncthreads();
  const int ex = inc - v + sh[wv];
  if (total) *total = sh[NT / 64];
  __syncthreads();
  return ex;
}

// ------------------------------------------------------------------------------------------------
// Radix select of the m-th smallest key: four 16-bit digits, most significant first.
// ------------------------------------------------------------------------------------------------
struct SelState {
  uint64_t prefix;   // fixed high bits so far
  int64_t need;      // how many of the keys matching `prefix` still have to be taken
  int64_t jthresh;   // among keys == prefix (after 4 levels), take those with j <= jthresh
  int64_t eqcount;   // number of keys equal to the final prefix
};

__global__ void k_sel_init(SelState* s, int64_t m, int* hist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 65536) hist[i] = 0;
  if (i == 0) {
    s->prefix = 0;
    s->need = m;
    s->jthresh = INT64_MAX;
    s->eqcount = 0;
  }
}

__global__ void k_sel_hist(const uint64_t* __restrict__ keys, int64_t N, int level,
                           const SelState* __restrict__ s, int* __restrict__ hist) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const uint64_t k = keys[j];
  const int shift = 48 - 16 * level;
  if (level > 0 && (k >> (shift + 16)) != (s->prefix >> (shift + 16))) return;
  atomicAdd(&hist[(k >> shift) & 0xFFFF], 1);
}

// One workgroup of 1024 threads: locate the digit where the running count crosses `need`.
__global__ __launch_bounds__(1024) void k_sel_pick(int level, SelState* s, int* hist) {
  __shared__ int sh[17];
  const int tid = threadIdx.x;
  int loc = 0;
  for (int b = 0; b < 64; ++b) loc += hist[tid * 64 + b];
  int total;
  const int ex = block_excl_scan<1024>(loc, sh, &total);
  const int64_t need = s->need;
  __syncthreads();
  if ((int64_t)ex < need && need <= (int64_t)(ex + loc)) {
    int run = ex;
    for (int b = 0; b < 64; ++b) {
      const int c = hist[tid * 64 + b];
      if (need <= (int64_t)(run + c)) {
        const int digit = tid * 64 + b;
        const int shift = 48 - 16 * level;
        s->prefix |= ((uint64_t)digit) << shift;
        s->need = need - run;
        s->eqcount = c;
        break;
      }
      run += c;
    }
  }
  __syncthreads();
  for (int b = 0; b < 64; ++b) hist[tid * 64 + b] = 0;
}

// Rare path: several keys equal the m-th key and only some are taken -> take the smallest rows.
__global__ __launch_bounds__(1024) void k_sel_ties(const uint64_t* __restrict__ keys, int64_t N,
                                                   SelState* s) {
  __shared__ int sh[17];
  if (s->need >= s->eqcount) return;  // all equal keys are taken (the usual case)
  const uint64_t K = s->prefix;
  int64_t need = s->need;
  for (int64_t base = 0; base < N; base += 1024) {
    const int64_t j = base + threadIdx.x;
    const int eq = (j < N && keys[j] == K) ? 1 : 0;
    int tot;
    const int ex = block_excl_scan<1024>(eq, sh, &tot);
    if (eq && ex + 1 == need) s->jthresh = j;
    need -= tot;
    __syncthreads();
    if (need <= 0) break;
  }
}

constexpr int CMP_CHUNK = 4096;  // keys per workgroup in the compaction (256 threads x 16)

__device__ __forceinline__ bool sel_pred(uint64_t k, int64_t j, const SelState& s) {
  return k < s.prefix || (k == s.prefix && j <= s.jthresh);
}

__global__ __launch_bounds__(256) void k_cmp_count(const uint64_t* __restrict__ keys, int64_t N,
                                                   const SelState* __restrict__ sp,
                                                   int* __restrict__ bcount) {
  __shared__ int sh[5];
  const SelState s = *sp;
  const int64_t base = (int64_t)blockIdx.x * CMP_CHUNK + threadIdx.x * 16;
  int c = 0;
  for (int i = 0; i < 16; ++i) {
    const int64_t j = base + i;
    if (j < N && sel_pred(keys[j], j, s)) ++c;
  }
  int tot;
  block_excl_scan<256>(c, sh, &tot);
  if (threadIdx.x == 0) bcount[blockIdx.x] = tot;
}

// Single workgroup exclusive scan of `len` ints in place (len up to a few hundred thousand).
__global__ __launch_bounds__(1024) void k_scan_small(int* __restrict__ a, int64_t len) {
  __shared__ int sh[17];
  int carry = 0;
  for (int64_t base = 0; base < len; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int v = i < len ? a[i] : 0;
    int tot;
    const int ex = block_excl_scan<1024>(v, sh, &tot);
    if (i < len) a[i] = ex + carry;
    carry += tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_cmp_write(const uint64_t* __restrict__ keys, int64_t N,
                                                   const SelState* __restrict__ sp,
                                                   const int* __restrict__ boff,
                                                   int64_t* __restrict__ rows, int64_t m) {
  __shared__ int sh[5];
  const SelState s = *sp;
  const int64_t base = (int64_t)blockIdx.x * CMP_CHUNK + threadIdx.x * 16;
  int c = 0;
  for (int i = 0; i < 16; ++i) {
    const int64_t j = base + i;
    if (j < N && sel_pred(keys[j], j, s)) ++c;
  }
  int pos = block_excl_scan<256>(c, sh, nullptr) + boff[blockIdx.x];
  for (int i = 0; i < 16; ++i) {
    const int64_t j = base + i;
    if (j < N && sel_pred(keys[j], j, s)) {
      if (pos < m) rows[pos] = j;
      ++pos;
    }
  }
}

size_t srht_select_bcount_len(int64_t N) { return (size_t)((N + CMP_CHUNK - 1) / CMP_CHUNK) + 1; }

void srht_select(hipStream_t st, const uint64_t* keys, int64_t N, int64_t m, int64_t* rows,
                 SelectScratch sc) {
  SelState* s = (SelState*)sc.state;
  hipLaunchKernelGGL(k_sel_init, dim3(256), dim3(256), 0, st, s, m, sc.hist);
  const unsigned nb = (unsigned)((N + 255) / 256);
  for (int level = 0; level < 4; ++level) {
    hipLaunchKernelGGL(k_sel_hist, dim3(nb), dim3(256), 0, st, keys, N, level, s, sc.hist);
    hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(1024), 0, st, level, s, sc.hist);
  }
  hipLaunchKernelGGL(k_sel_ties, dim3(1), dim3(1024), 0, st, keys, N, s);
  const int64_t nblk = (N + CMP_CHUNK - 1) / CMP_CHUNK;
  hipLaunchKernelGGL(k_cmp_count, dim3((unsigned)nblk), dim3(256), 0, st, keys, N, s, sc.bcount);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, sc.bcount, nblk);
  hipLaunchKernelGGL(k_cmp_write, dim3((unsigned)nblk), dim3(256), 0, st, keys, N, s, sc.bcount,
                     rows, m);
}

// ------------------------------------------------------------------------------------------------
// SJLT targets and signs: one thread per row of A.
// ------------------------------------------------------------------------------------------------
__global__ void k_sjlt_draw(uint64_t seed, uint64_t t, int64_t n, uint32_t m, int s,
                            int32_t* __restrict__ targets, int8_t* __restrict__ signs,
                            int* __restrict__ err) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t thr = (uint32_t)((1ull << 32) % m);
  uint32_t tg[MAX_SJLT_S];
  int cnt = 0;
  for (int c = 0; c < MAX_SJLT_WORDS / 4 && cnt < s; ++c) {
    const u64x4 w4 = philox4x64_10((uint64_t)j, TAG_SJLT, t, (uint64_t)c, seed, 0);
    const uint64_t ws[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (cnt >= s) break;
      uint32_t h;
      if (!sjlt_propose(ws[q], m, thr, &h)) continue;
      bool dup = false;
      for (int k = 0; k < cnt; ++k) dup |= (tg[k] == h);
      if (dup) continue;
      tg[cnt] = h;
      targets[j * s + cnt] = (int32_t)h;
      signs[j * s + cnt] = (ws[q] & 1ull) ? (int8_t)-1 : (int8_t)1;
      ++cnt;
    }
  }
  if (cnt < s) {
    // keep every target a valid row index so later passes stay in bounds; the call reports an error
    for (int k = cnt; k < s; ++k) {
      targets[j * s + k] = 0;
      signs[j * s + k] = 1;
    }
    atomicOr(err, 1);
  }
}

void launch_sjlt_draw(hipStream_t st, uint64_t seed, uint64_t t, int64_t n, int64_t m, int s,
                      int32_t* targets, int8_t* signs, int* err) {
  const int nt = 256;
  hipLaunchKernelGGL(k_sjlt_draw, dim3((unsigned)((n + nt - 1) / nt)), dim3(nt), 0, st, seed, t, n,
                     (uint32_t)m, s, targets, signs, err);
}

// ------------------------------------------------------------------------------------------------
// Gaussian entries (unscaled standard normals, FP64, the values of the FP64 sketch), one thread per
// entry: for the parity checks of the draws.
// ------------------------------------------------------------------------------------------------
__global__ void k_gauss_draw(uint64_t seed, uint64_t t, int64_t m, int64_t j0, int64_t ncols,
                             double* __restrict__ G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * ncols) return;
  const int64_t i = idx / ncols, c = idx % ncols, j = j0 + c;
  const u64x4 w = philox4x64_10((uint64_t)(j >> 3), TAG_GAUSS, t, (uint64_t)i, seed, 0);
  const int q = (int)(j & 7), p = q >> 1;
  const uint64_t word = p == 0 ? w.x : p == 1 ? w.y : p == 2 ? w.z : w.w;
  double cs, sn;
  box_muller_pair_f64(word, cs, sn);
  G[idx] = (q & 1) ? sn : cs;
}

// The Gaussian embedding's standard normals transposed: Gt[j m + i] = g(i, j), j < n, i < m (the n x m
// matrix whose columns are the rows of the unscaled embedding), FP64 as in the FP64 sketch.  One thread
// per (i, 8 consecutive j): one Philox block gives the 8 values; consecutive threads write consecutive i.
__global__ void k_gauss_draw_t(uint64_t seed, uint64_t t, int64_t n, int64_t m, double* __restrict__ Gt) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = (n + 7) / 8;
  if (idx >= nb * m) return;
  const int64_t i = idx % m, jb = idx / m;
  const u64x4 w = philox4x64_10((uint64_t)jb, TAG_GAUSS, t, (uint64_t)i, seed, 0);
  const uint64_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    double cs, sn;
    box_muller_pair_f64(ws[p], cs, sn);
    const int64_t j = 8 * jb + 2 * p;
    if (j < n) Gt[j * m + i] = cs;
    if (j + 1 < n) Gt[(j + 1) * m + i] = sn;
  }
}

void launch_gauss_draw_t(hipStream_t st, uint64_t seed, uint64_t t, int64_t n, int64_t m, double* Gt) {
  const int64_t tot = (n + 7) / 8 * m;
  hipLaunchKernelGGL(k_gauss_draw_t, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, seed, t, n, m, Gt);
}

void launch_gauss_draw(hipStream_t st, uint64_t seed, uint64_t t, int64_t m, int64_t j0,
                       int64_t ncols, double* G) {
  const int64_t tot = m * ncols;
  hipLaunchKernelGGL(k_gauss_draw, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, seed, t,
                     m, j0, ncols, G);
}

// ------------------------------------------------------------------------------------------------
// Device-wide exclusive scan of int32 (tiles of 4096, then a single-workgroup scan of tile sums).
// ------------------------------------------------------------------------------------------------
constexpr int SCAN_TILE = 4096;

__global__ __launch_bounds__(256) void k_scan_tiles(const int* __restrict__ in, int* __restrict__ out,
                                                    int64_t len, int* __restrict__ tsum) {
  __shared__ int sh[5];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 16;
  int v[16];
  int c = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    v[i] = (base + i < len) ? in[base + i] : 0;
    c += v[i];
  }
  int tot;
  int run = block_excl_scan<256>(c, sh, &tot);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (base + i < len) out[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_add(int* __restrict__ out, int64_t len,
                                                  const int* __restrict__ tsum) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 16;
  const int add = tsum[blockIdx.x];
#pragma unroll
  for (int i = 0; i < 16; ++i)
    if (base + i < len) out[base + i] += add;
}

size_t scan_tmp_len(int64_t len) { return (size_t)((len + SCAN_TILE - 1) / SCAN_TILE) + 1; }

void exclusive_scan_i32(hipStream_t st, const int* in, int* out, int64_t len, int* tmp) {
  const int64_t nt = (len + SCAN_TILE - 1) / SCAN_TILE;
  if (nt == 0) return;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(256), 0, st, in, out, len, tmp);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, tmp, nt);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(256), 0, st, out, len, tmp);
}

}  // namespace lsq
