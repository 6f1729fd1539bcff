// Internal launcher interface between the kernels (*.hip) and the host driver (api.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace lsq {

// ---- device helpers shared by the kernels ------------------------------------------------------
// Workgroup barrier for data exchanged through LDS only: this wavefront's LDS accesses complete
// (lgkmcnt), then s_barrier; loads from global memory stay in flight (__syncthreads also drains them).
// The empty asm statements keep the compiler from moving memory accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt unconstrained
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// s_waitcnt vmcnt(N): at most N of this wavefront's vector memory instructions (global loads, stores and
// global-to-LDS loads, in issue order) still outstanding; expcnt and lgkmcnt unconstrained.
template <int N>
__device__ __forceinline__ void vm_wait() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}

// Four 16-byte LDS reads at base + 0, 1, 2, 3 x STRIDE bytes, waited for inside the same statement.
// For LDS that global-to-LDS loads fill: the compiler cannot tell which of those loads an ordinary LDS
// read depends on and waits for all of them (vmcnt(0)), which would drain the loads issued ahead; the
// caller orders these reads after the loads they need (vm_wait + barrier) itself.
template <int O0, int O1, int O2, int O3>
__device__ __forceinline__ void lds_read4_b128_at(uint32_t base, int4& a, int4& b, int4& c, int4& e) {
  static_assert(O0 >= 0 && O1 < 65536 && O2 < 65536 && O3 < 65536, "ds_read offset range");
  asm volatile(
      "ds_read_b128 %0, %4 offset:%5\n\t"
      "ds_read_b128 %1, %4 offset:%6\n\t"
      "ds_read_b128 %2, %4 offset:%7\n\t"
      "ds_read_b128 %3, %4 offset:%8\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a), "=&v"(b), "=&v"(c), "=&v"(e)
      : "v"(base), "i"(O0), "i"(O1), "i"(O2), "i"(O3)
      : "memory");
}
template <int STRIDE>
__device__ __forceinline__ void lds_read4_b128(uint32_t base, int4& a, int4& b, int4& c, int4& e) {
  lds_read4_b128_at<0, STRIDE, 2 * STRIDE, 3 * STRIDE>(base, a, b, c, e);
}
template <int O0, int O1>
__device__ __forceinline__ void lds_read2_b128_at(uint32_t base, int4& a, int4& b) {
  static_assert(O0 >= 0 && O1 < 65536, "ds_read offset range");
  asm volatile(
      "ds_read_b128 %0, %2 offset:%3\n\t"
      "ds_read_b128 %1, %2 offset:%4\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a), "=&v"(b)
      : "v"(base), "i"(O0), "i"(O1)
      : "memory");
}

// F values (F = 8 or 16) of 4 or 8 bytes at base + k 64 elements, k < F (ds_read2st64: two per
// instruction), waited for inside the statement; and the matching writes (not waited for: the next
// lds_barrier drains them).  Same purpose as lds_read4_b128.
typedef uint32_t lds_u2 __attribute__((ext_vector_type(2)));
typedef uint64_t lds_q2 __attribute__((ext_vector_type(2)));
template <typename V>
__device__ __forceinline__ void lds_read8_st64(uint32_t base, V (&x)[4]);
template <>
__device__ __forceinline__ void lds_read8_st64<lds_u2>(uint32_t base, lds_u2 (&x)[4]) {
  asm volatile(
      "ds_read2st64_b32 %0, %4 offset1:1\n\t"
      "ds_read2st64_b32 %1, %4 offset0:2 offset1:3\n\t"
      "ds_read2st64_b32 %2, %4 offset0:4 offset1:5\n\t"
      "ds_read2st64_b32 %3, %4 offset0:6 offset1:7\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3])
      : "v"(base)
      : "memory");
}
template <>
__device__ __forceinline__ void lds_read8_st64<lds_q2>(uint32_t base, lds_q2 (&x)[4]) {
  asm volatile(
      "ds_read2st64_b64 %0, %4 offset1:1\n\t"
      "ds_read2st64_b64 %1, %4 offset0:2 offset1:3\n\t"
      "ds_read2st64_b64 %2, %4 offset0:4 offset1:5\n\t"
      "ds_read2st64_b64 %3, %4 offset0:6 offset1:7\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3])
      : "v"(base)
      : "memory");
}
template <typename V>
__device__ __forceinline__ void lds_read16_st64(uint32_t base, V (&x)[8]);
template <>
__device__ __forceinline__ void lds_read16_st64<lds_u2>(uint32_t base, lds_u2 (&x)[8]) {
  asm volatile(
      "ds_read2st64_b32 %0, %8 offset1:1\n\t"
      "ds_read2st64_b32 %1, %8 offset0:2 offset1:3\n\t"
      "ds_read2st64_b32 %2, %8 offset0:4 offset1:5\n\t"
      "ds_read2st64_b32 %3, %8 offset0:6 offset1:7\n\t"
      "ds_read2st64_b32 %4, %8 offset0:8 offset1:9\n\t"
      "ds_read2st64_b32 %5, %8 offset0:10 offset1:11\n\t"
      "ds_read2st64_b32 %6, %8 offset0:12 offset1:13\n\t"
      "ds_read2st64_b32 %7, %8 offset0:14 offset1:15\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(x[4]), "=&v"(x[5]), "=&v"(x[6]), "=&v"(x[7])
      : "v"(base)
      : "memory");
}
template <>
__device__ __forceinline__ void lds_read16_st64<lds_q2>(uint32_t base, lds_q2 (&x)[8]) {
  asm volatile(
      "ds_read2st64_b64 %0, %8 offset1:1\n\t"
      "ds_read2st64_b64 %1, %8 offset0:2 offset1:3\n\t"
      "ds_read2st64_b64 %2, %8 offset0:4 offset1:5\n\t"
      "ds_read2st64_b64 %3, %8 offset0:6 offset1:7\n\t"
      "ds_read2st64_b64 %4, %8 offset0:8 offset1:9\n\t"
      "ds_read2st64_b64 %5, %8 offset0:10 offset1:11\n\t"
      "ds_read2st64_b64 %6, %8 offset0:12 offset1:13\n\t"
      "ds_read2st64_b64 %7, %8 offset0:14 offset1:15\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(x[4]), "=&v"(x[5]), "=&v"(x[6]), "=&v"(x[7])
      : "v"(base)
      : "memory");
}
// one pair write: values a, b at base + (2 k) and (2 k + 1) x 64 elements
template <int K>
__device__ __forceinline__ void lds_write2_st64(uint32_t base, uint32_t a, uint32_t b) {
  asm volatile("ds_write2st64_b32 %0, %1, %2 offset0:%3 offset1:%4" : : "v"(base), "v"(a), "v"(b), "i"(2 * K),
               "i"(2 * K + 1) : "memory");
}
template <int K>
__device__ __forceinline__ void lds_write2_st64(uint32_t base, uint64_t a, uint64_t b) {
  asm volatile("ds_write2st64_b64 %0, %1, %2 offset0:%3 offset1:%4" : : "v"(base), "v"(a), "v"(b), "i"(2 * K),
               "i"(2 * K + 1) : "memory");
}

// ---- draws.hip ----------------------------------------------------------------------------------
// Per padded row j < N: sign (int8 +-1) and 64-bit selection key (SRHT specification).
void launch_srht_draw(hipStream_t st, uint64_t seed, uint64_t t, int64_t N, int8_t* signs,
                      uint64_t* keys);
// Scratch for srht_select (device): hist 65536 ints, sel state, block counts.
struct SelectScratch {
  int* hist;       // 65536
  int* bcount;     // nblocks(N) + 1
  void* state;     // SelState
};
size_t srht_select_bcount_len(int64_t N);
// rows (device int64, m entries, increasing) = the m padded rows with the smallest (key, j).
void srht_select(hipStream_t st, const uint64_t* keys, int64_t N, int64_t m, int64_t* rows,
                 SelectScratch sc);
// s targets and signs per row of A, in draw order; err set to 1 if a row exhausts its draws.
void launch_sjlt_draw(hipStream_t st, uint64_t seed, uint64_t t, int64_t n, int64_t m, int s,
                      int32_t* targets, int8_t* signs, int* err);
void launch_gauss_draw(hipStream_t st, uint64_t seed, uint64_t t, int64_t m, int64_t j0,
                       int64_t ncols, double* G);
// Gt (n x m, row-major FP32) = the unscaled normals transposed, Gt[j m + i] = g(i, j).
void launch_gauss_draw_t(hipStream_t st, uint64_t seed, uint64_t t, int64_t n, int64_t m, double* Gt);
// Exclusive prefix sum of len int32 values; tmp needs scan_tmp_len(len) ints.
size_t scan_tmp_len(int64_t len);
void exclusive_scan_i32(hipStream_t st, const int* in, int* out, int64_t len, int* tmp);

// ---- sketch.hip ---------------------------------------------------------------------------------
// Column slices of 128 bytes: 256-row Walsh-Hadamard blocks (N rows when N is smaller), then the
// remaining high bits are summed directly for the selected rows only.
struct SrhtPlan {
  int64_t N, N1, N2, m;
  int nneeded;             // buckets T is sized for: min(N1, m), at least the distinct k_lo selected
  int passb = 0;           // form of pass B for large buckets (lsq_set_option "srht_passb")
};
size_t srht_tbuf_bytes(int64_t N2, int64_t nneeded, int64_t d, int compute_f32);
// Groups the selected rows by k_lo: slot (N1 ints, -1 if unused), order (m ints), bstart (N1+1 ints).
// The count of distinct k_lo is left on the device (nneeded_dev); the host sizes T for min(N1, m) buckets.
void srht_plan_groups(hipStream_t st, const int64_t* rows, int64_t m, int64_t N1, int* slot,
                      int* order, int* bstart, int* nneeded_dev);
size_t srht_partial_bytes(int64_t N2, int64_t m, int64_t d);
// With gpart (N2 rows of d + 1 doubles) and y, pass A also leaves A^T y in the fused pass's partial layout
// (column d: sum of y^2) when it takes its vector form; returns whether it did.
bool srht_apply(hipStream_t st, const void* A, int a_f32, int64_t n, int64_t d, int64_t lda,
                int compute_f32, const SrhtPlan& plan, const int8_t* signs, const int64_t* rows,
                const int* slot, const int* order, const int* bstart, void* tbuf, double* partial,
                double* SA, int64_t ldsa, const double* y = nullptr, double* gpart = nullptr);

struct SjltScratch {
  int32_t* targets;  // n*s
  int8_t* signs;     // n*s
  int* cnt;          // m * nblk
  int* off;          // m * nblk
  int* scan_tmp;
  uint32_t* sorted;  // n*s entries (row << 1 | negative)
  int* bstart;       // m + 1 (bucket starts, = off[h * nblk])
  int* err;
};
int64_t sjlt_nblk(int64_t n);
void sjlt_apply(hipStream_t st, uint64_t seed, uint64_t t, const void* A, int a_f32, int64_t n,
                int64_t d, int64_t lda, int64_t m, int s, SjltScratch sc, double* SA, int64_t ldsa);

// Gaussian sketch SA = G A with G generated in registers (FP64 matrix cores; bf16 split on request).
// The workspace (partials) holds the FP64 partial sums and, for the BF16 form at d >= the planes
// threshold, the three BF16 terms of one chunk of rows of A after them.
size_t gauss_partial_bytes(int64_t m, int64_t d, int64_t n, int bf16);
void gauss_apply(hipStream_t st, uint64_t seed, uint64_t t, const void* A, int a_f32, int64_t n,
                 int64_t d, int64_t lda, int64_t m, int bf16, double* partials, double* SA,
                 int64_t ldsa);

// ---- factor.hip ---------------------------------------------------------------------------------
// Householder QR of SA (m x d, row-major) -> R (d x d row-major, positive diagonal).  X: m*d doubles of
// scratch.  status: device int, set to LSQ_ERR_RANK on a zero pivot.
void householder_qr(hipStream_t st, const double* SA, int64_t m, int64_t d, int64_t lds, double* X,
                    double* R, int* status);
// W = R^{-1} and WT = W^T (both d x d row-major).  scratch: trinv_scratch_len(d) doubles.
size_t trinv_scratch_len(int64_t d);
void tri_inverse(hipStream_t st, const double* R, int64_t d, double* W, double* WT, double* scratch);
// W = R^{-1} for an n x n upper R (row-major, ld n) into W (n x n); scratch: trinv_scratch_len(n) doubles.
void tri_inverse_padded(hipStream_t st, const double* R, int64_t n, double* W, double* scratch);
// status |= 1 when some |R_kk| <= 8 d eps max |R_jj|.
// flag (device int, cleared by the caller) = 1 when X (m x d, row stride ld) holds a NaN or an infinity.
void nonfinite_scan(hipStream_t st, const double* X, int64_t m, int64_t d, int64_t ld, int* flag);
// out[0] (device) = max |R_ii| / min |R_ii| of the d x d row-major R (a lower estimate of kappa(R)).
void diag_spread(hipStream_t st, const double* R, int64_t d, double* out);
void qr_rank_check(hipStream_t st, const double* R, int64_t d, int* status);

// ---- chol.hip -----------------------------------------------------------------------------------
// CholeskyQR2 of SA (m x d) -> R (d x d).  flags: 2 device ints, hflags: their pinned host mirror.
// Returns 0 on success, 1 when the first Cholesky broke down or its diagonal spread exceeds 1e7 (then
// R is not written and the caller uses a robust path).  trinv_scratch: trinv_scratch_len(padded d).
int64_t cholqr_padded(int64_t d);
size_t cholqr_scratch_len(int64_t m, int64_t d);
int cholqr_factor(hipStream_t st, const double* SA, int64_t m, int64_t d, int64_t lds, double* scratch,
                  double* R, int* flags, int* hflags, double* trinv_scratch, int passes = 2);
// Spread of diag(R) of the first CholeskyQR pass up to which the automatic form stops after that pass.
constexpr double CHOLQR_ONE_PASS_SPREAD = 2e5;
// Shifted CholeskyQR3 (any full-rank SA up to kappa ~ 1/u).  flags: 1 device int.
int cholqr3_shifted(hipStream_t st, const double* SA, int64_t m, int64_t d, int64_t lds, double* scratch,
                    double* R, int* flags, double* trinv_scratch);
// Haar embedding helpers.  W (dp x dp, dp = cholqr_padded(md)) = R^{-1} for R^T R = scale Z (Z: md x md
// symmetric positive definite, row-major); flag set on a non-positive pivot.  scratch:
// spd_inverse_scratch_len(md) doubles; trinv_scratch: trinv_scratch_len(dp).
size_t spd_inverse_scratch_len(int64_t md);
void spd_chol_inverse(hipStream_t st, const double* Z, int64_t md, double scale, double* scratch, double* W,
                      int* flag, double* trinv_scratch);
// SA = scale W^T Y for W upper triangular (m x m used, ld ldw) and Y (m x d, row-major).
void haar_apply(hipStream_t st, const double* W, int64_t ldw, const double* Y, int64_t m, int64_t d, double scale,
                double* SA, int64_t ldsa);
// ---- svd.hip ------------------------------------------------------------------------------------
// One-sided Jacobi SVD of the d x d R (overwritten by Sigma V^T): W = V Sigma^+ and WT = W^T (dense),
// singular values below rtol * sigma_max dropped.  Returns the number kept.  scratch: svd_scratch_len(d)
// doubles; flags / hflags: 2 device ints and their pinned mirror.  *sweeps: Jacobi sweeps run.
constexpr int SVD_MAX_SWEEPS = 40;
constexpr double SVD_RTOL = 1e-12;  // singular values below rtol * sigma_max are dropped
// rhat = W W^T r with the preconditioner's shape: triangular W (precond_apply) or dense W (the SVD form:
// two full GEMVs, the same dot-product partials for r . rhat).
void precond_apply_any(hipStream_t st, const double* W, const double* WT, int64_t d, const double* r, double* u,
                       double* rhat, double* dotpart, int* ndot, const int* done, int dense);
size_t svd_scratch_len(int64_t d);
int svd_precond(hipStream_t st, double* R, int64_t d, double rtol, double* scratch, double* W, double* WT,
                int* flags, int* hflags, int* sweeps);
// ---- qrcp.hip -----------------------------------------------------------------------------------
// Column-pivoted Householder QR of S A (m x d): R (d x d) = R_pivoted P^T, W = P [R11^{-1}; 0] and WT = W^T
// (dense), R11 the leading r x r block with |R_kk| > rtol |R_00|.  Returns r.  scratch:
// qrcp_scratch_len(m, d) doubles; trinv_scratch: trinv_scratch_len(d); flags / hflags: 1 device int and its
// pinned mirror.
size_t qrcp_scratch_len(int64_t m, int64_t d);
int qrcp_precond(hipStream_t st, const double* SA, int64_t m, int64_t d, int64_t lds, double rtol, double* scratch,
                 double* trinv_scratch, double* R, double* W, double* WT, int* flags, int* hflags);
constexpr int64_t QR_M_MAX = 8192;       // Householder QR: rows held in registers
constexpr int64_t FACTOR_M_MAX = 65536;  // any factorization

// ---- iter.hip -----------------------------------------------------------------------------------
int fused_nwg(int64_t n, int64_t d);
// Launch-shape tuning (lsq_tune; set from the autotuner's table).  None changes the method: each selects
// a grid or a kernel form that computes the same sums (in another fixed order at most).
extern int g_srht_fold8_rows_f32;   // SRHT pass B: 8-point fold from this many selected rows per bucket (FP32 T)
extern int g_srht_fold8_rows_f64;   // the same for an FP64 intermediate
extern int g_srht_stream_rows_f32;  // SRHT pass B: the streamed form from this many rows per bucket (FP32 T)
extern int g_srht_stream_rows_f64;  // the same for an FP64 intermediate
extern int g_srht_passa_wgs;        // SRHT pass A: workgroups aimed at (0: by the transform precision)
extern int g_srht_passb_wgs;        // LDS-staged SRHT pass B: workgroups aimed at when splitting j_hi
extern int g_gauss_wgs;             // Gaussian sketch: workgroups aimed at when splitting n
extern int g_gauss_planes_min_d;    // BF16 Gaussian sketch: smallest d taking the planes form
extern int g_gauss_planes_wgs;      // ... its workgroups per launch aimed at (one per compute unit)
extern int g_gauss_chunk_rows;      // ... rows of A per chunk (0: planes of about 1 GiB)
extern int g_gram_wgs;              // CholeskyQR Gram kernel: workgroups aimed at when splitting m
extern int g_fused_groups_per_cu;   // tuning: fused-pass workgroups per CU
extern int g_batched_slots;         // tuning: batched-kernel workgroups (0 = one per CU)
// Bare streaming read of the first bytes / 16 whole 16-byte vectors of buf (device, 16-byte aligned) by
// `groups` workgroups, each writing its sum to out[group] (for measuring the read ceiling).
void stream_read(hipStream_t st, const void* buf, int64_t bytes, int groups, float* out);
void stream_copy(hipStream_t st, const void* src, void* dst, int64_t bytes, int groups);
// Partial sums are reduced in two fixed-order stages: nwg rows -> REDUCE_SPLIT rows -> 1.
constexpr int REDUCE_SPLIT = 32;
void reduce_stage1(hipStream_t st, const double* part, int nwg, int64_t d, double* part2,
                   const int* done);
// mode 0: part[g] = (sum_j (a_j.v) a_j, sum_j (a_j.v)^2), mode 1: with q_j = y_j - a_j.v.
// part: nwg * (d + 1) doubles.  done: optional device flag (skip when set).
// Returns the number of workgroups launched (= partial rows to reduce), at most nwg.
int fused_pass(hipStream_t st, const void* A, int a_f32, int f32_math, int64_t n, int64_t d,
               int64_t lda, int mode, const double* v, const double* y, double* part, int nwg,
               const int* done);
// out[c] = sum_g part[g][c] for c <= d (fixed order); part2: REDUCE_SPLIT * (d + 1) scratch.
void reduce_partials(hipStream_t st, const double* part, double* part2, int nwg, int64_t d,
                     double* out, const int* done);
// PCG building blocks (see iter.hip for the exact steps).
// part2: the REDUCE_SPLIT rows left by reduce_stage1.
void pcg_update_xr(hipStream_t st, const double* part2, int nrows, int64_t d, double* x, double* r,
                   const double* p, DevState* ds);
void precond_apply(hipStream_t st, const double* W, const double* WT, int64_t d, const double* r,
                   double* u, double* rhat, double* dotpart, int* ndot, const int* done);
void pcg_update_p(hipStream_t st, int64_t d, const double* rhat, double* p, const double* dotpart,
                  int ndot, DevState* ds, const double* x, const double* r, const double* x_ref,
                  double* trace, int trace_len);
void pcg_init(hipStream_t st, int64_t d, const double* rhat, double* p, const double* dotpart,
              int ndot, DevState* ds, double tol, const double* x, const double* r,
              const double* x_ref, double* trace);
void dot_to_state(hipStream_t st, int64_t d, const double* a, const double* b, DevState* ds);
void vec_copy(hipStream_t st, double* dst, const double* src, int64_t len);
void vec_zero(hipStream_t st, double* dst, int64_t len);
void vec_axpy(hipStream_t st, double* y, const double* x, double a, int64_t len);
// IHS: x_new = x - mu * hinvg + beta (x - xprev); xprev <- x; x <- x_new.
void ihs_update(hipStream_t st, int64_t d, double* x, double* xprev, const double* hinvg, double mu,
                double beta);
// out = sqrt(a[0] / b) style scalar helpers evaluated on the device
void error_from_resid(hipStream_t st, const double* scal, double denom, double* out);

// ---- noalloc.hip ------------------------------------------------------------------------------
// A file-scope device array of NOALLOC_DOUBLES doubles (8 MiB) per device for lsq_fused_pass_noalloc;
// noalloc_scratch returns its address on device dev (the current device), looked up once per device.
constexpr size_t NOALLOC_DOUBLES = (size_t)1 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch(int dev, double** out);

// ---- resid.hip ----------------------------------------------------------------------------------
// r = A^T (y - A x) in double-double, rounded once; scal (optional) = ||y - A x||^2.  part:
// resid_dd_part_len(d) doubles.  Returns false when d is beyond the kernel's chunk limit (d <= 1024).
size_t resid_dd_part_len(int64_t d);
bool resid_dd(hipStream_t st, const void* A, int a_f32, int64_t n, int64_t d, int64_t lda, const double* x,
              const double* y, double* part, double* r, double* scal);

// ---- fcg.hip ------------------------------------------------------------------------------------
// Ring of K directions (P, HP: K x d; php: K) for the flexible CG window; see fcg.hip.
constexpr int FCG_MAX_WINDOW = 1024;
void fcg_orth(hipStream_t st, const double* v, double* P, const double* HP, const double* php, int64_t d,
              int t, int kt, int K);
void fcg_step(hipStream_t st, const double* p, const double* red, int64_t d, double* x, double* r,
              double* hp_slot, double* php_slot);

// ---- batched form (batched.hip) ----
// One problem of a batch, in queue order (largest n*d first).
struct BatchDesc {
  const void* A;
  const double* y;
  double* x;        // in: x_0, out: solution (d entries)
  double* R;        // optional copy of R (d x d row-major), may be null
  int64_t n, lda;
  int32_t d, m, s, a_f32;
  uint64_t seed, t;
  int32_t idx, pad;  // position in the caller's arrays
};
struct BatchOut {
  int32_t status, iters, refinements, pad;
  double est;
  uint64_t t_start, t_sketch, t_factor, t_end;  // device wall clock at the phase boundaries
};
// One entry of the work queue: problem q (position in the table), member `rank` of a gang of K
// workgroups (K = 1: the problem alone), gang index (-1 for K = 1).
struct BatchTask {
  int32_t q, rank, K, gang;
};
constexpr int BATCH_GANG_KMAX = 4;  // workgroups per problem at most
// Kernel arguments: the problem table, the task queue (ntasks entries), results, queue counter, solver
// options, the per-slot workspace (slot = workgroup index; strides in elements) and the per-gang state
// (gstate: 4 ints per gang, barrier count, leader slot, setup status, broken flag; gpart: 2 x KMAX
// partial rows of gpart_stride doubles per gang).
struct BatchArgs {
  const BatchDesc* descs;
  const BatchTask* tasks;
  BatchOut* out;
  int* queue;
  int count, ntasks, ngangs, mixed, max_iter, max_refine;
  double tol;
  uint32_t *keys, *sorted;
  double *SA, *V, *R, *W, *WT, *last;
  int64_t keys_stride, sa_stride, v_stride, r_stride, last_stride;
  int* gstate;
  double* gpart;
  int64_t gpart_stride;
};
extern int64_t g_batched_gang_unit;  // elements (n d) per gang member; 0: no gangs
// Resets the queue and the results, then launches the persistent kernel with `slots` workgroups.
void batched_launch(hipStream_t st, const BatchArgs& a, int slots);

}  // namespace lsq
