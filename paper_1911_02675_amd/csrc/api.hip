// Host driver and C ABI of liblsq (declared in include/lsq.h).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

using namespace lsq;

static thread_local std::string g_err;

static lsq_status fail(lsq_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(LSQ_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

#define CHK(expr)                                                                             \
  do {                                                                                        \
    lsq_status s_ = (expr);                                                                   \
    if (s_ != LSQ_OK) return s_;                                                              \
  } while (0)

struct EvPair {
  hipEvent_t a, b;
};

struct lsq_ctx {
  hipStream_t st = nullptr;
  int dev = 0;
  std::map<std::string, std::pair<void*, size_t>> bufs;
  DevState* ds = nullptr;   // device
  DevState* hds = nullptr;  // pinned host mirror
  int* dflags = nullptr;    // device ints: [0] factor status, [1] SJLT draw error, [2] SRHT buckets used,
                            // [4], [5] CholeskyQR breakdown / spread flags
  int* hflags = nullptr;    // pinned host mirror (8 ints)
  hipEvent_t ev[6] = {};
  std::vector<EvPair> fused_ev;  // events around fused passes of the current call
  size_t fused_used = 0;
  double fused_total_ms = 0.0, fused_last_ms = 0.0;
  int64_t fused_count = 0;
  double last_rate = -1.0;  // contraction per PCG iteration seen in the previous loop (batch sizing)
  // batched form: private stream (capture is not possible on the legacy default stream), the
  // instantiated graph and the launch configuration it was captured for, pinned result buffer
  hipStream_t bst = nullptr;
  hipGraph_t bgraph = nullptr;
  hipGraphExec_t bexec = nullptr;
  std::vector<unsigned char> bkey;
  void* bhost = nullptr;
  size_t bhost_bytes = 0;
  hipEvent_t bev[3] = {};
  double* hx = nullptr;  // pinned host copy of a starting point (mixed solve)
  size_t hx_len = 0;
  int w_dense = 0;        // the last factorization's W is dense (SVD form) rather than triangular
  int svd_rank = 0, svd_sweeps = 0;
  // numerics options of this context (lsq_set_option)
  int factor_mode = 0;    // 0 CholeskyQR, second pass when needed, with fallbacks; 1 Householder; 2 SVD;
                          // 3 column-pivoted QR; 4 CholeskyQR2 always; 5 one pass always (fallbacks of 0)
  int srht_passb = 0;     // SRHT pass B form for large buckets
  double* noalloc = nullptr;  // this device's static array for lsq_fused_pass_noalloc
  int sketch_upgrade = 1; // mixed form: an FP32 SRHT is retaken in FP64 when diag(R) spreads beyond 1e6
};
constexpr double SKETCH_UPGRADE_SPREAD = 1e6;

// Per-call trace on stderr when the environment variable LSQ_LOG is set to a non-zero value.
static bool log_on() {
  static const int on = [] {
    const char* v = getenv("LSQ_LOG");
    return v && *v && strcmp(v, "0") != 0 ? 1 : 0;
  }();
  return on != 0;
}
#define LSQ_TRACE(...)                     \
  do {                                     \
    if (log_on()) {                        \
      fprintf(stderr, "[lsq] " __VA_ARGS__); \
      fputc('\n', stderr);                 \
      fflush(stderr);                      \
    }                                      \
  } while (0)

// ------------------------------------------------------------------------------------------------
// workspace
// ------------------------------------------------------------------------------------------------
static lsq_status ws(lsq_ctx* c, const char* name, size_t bytes, void** out) {
  if (bytes == 0) bytes = 16;
  auto& b = c->bufs[name];
  if (b.second < bytes) {
    if (b.first) {
      HIPCHK(hipStreamSynchronize(c->st));
      HIPCHK(hipFree(b.first));
      b.first = nullptr;
      b.second = 0;
    }
    const size_t cap = bytes + bytes / 8 + 256;
    if (hipMalloc(&b.first, cap) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LSQ_ERR_NOMEM, std::string("workspace allocation failed: ") + name);
    }
    b.second = cap;
  }
  *out = b.first;
  return LSQ_OK;
}

template <typename T>
static lsq_status wsT(lsq_ctx* c, const char* name, size_t count, T** out) {
  void* p;
  CHK(ws(c, name, count * sizeof(T), &p));
  *out = (T*)p;
  return LSQ_OK;
}

static lsq_status sync_state(lsq_ctx* c) {
  HIPCHK(hipMemcpyAsync(c->hds, c->ds, sizeof(DevState), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return LSQ_OK;
}

static int64_t next_pow2(int64_t n) {
  int64_t N = 1;
  while (N < n) N <<= 1;
  return N;
}

// ------------------------------------------------------------------------------------------------
// validation
// ------------------------------------------------------------------------------------------------
static lsq_status check_problem(const lsq_ctx* c, const lsq_problem* p) {
  if (!c) return fail(LSQ_ERR_INVALID_ARG, "null context");
  if (!p || !p->A || !p->y) return fail(LSQ_ERR_INVALID_ARG, "null problem, A or y");
  if (p->d < 1 || p->n < p->d) return fail(LSQ_ERR_INVALID_ARG, "need n >= d >= 1");
  if (p->lda < p->d) return fail(LSQ_ERR_INVALID_ARG, "lda < d");
  if (p->a_dtype != LSQ_F64 && p->a_dtype != LSQ_F32)
    return fail(LSQ_ERR_INVALID_ARG, "a_dtype must be LSQ_F64 or LSQ_F32");
  if (p->d > 1024) return fail(LSQ_ERR_UNSUPPORTED, "d > 1024 is not implemented");
  if (p->n >= (int64_t)1 << 31) return fail(LSQ_ERR_UNSUPPORTED, "n >= 2^31 is not implemented");
  return LSQ_OK;
}

static lsq_status check_sketch(const lsq_ctx* c, const lsq_problem* p, const lsq_sketch_desc* s,
                               bool need_factor) {
  if (!s) return fail(LSQ_ERR_INVALID_ARG, "null sketch descriptor");
  if (s->m < 1) return fail(LSQ_ERR_INVALID_ARG, "m < 1");
  if (need_factor && s->m < p->d) return fail(LSQ_ERR_INVALID_ARG, "m < d: S A cannot have full rank");
  if (need_factor && s->m > FACTOR_M_MAX) return fail(LSQ_ERR_UNSUPPORTED, "m > 65536 is not implemented");
  if (need_factor && c->factor_mode == 1 && s->m > QR_M_MAX)
    return fail(LSQ_ERR_UNSUPPORTED, "Householder QR limited to m <= 8192");
  switch (s->kind) {
    case LSQ_SRHT:
      if (s->m > next_pow2(p->n)) return fail(LSQ_ERR_INVALID_ARG, "SRHT needs m <= N");
      if (s->compute != LSQ_F64 && s->compute != LSQ_F32)
        return fail(LSQ_ERR_INVALID_ARG, "SRHT compute must be LSQ_F64 or LSQ_F32");
      break;
    case LSQ_SJLT:
      if (s->s < 1 || s->s > s->m || s->s > MAX_SJLT_S)
        return fail(LSQ_ERR_INVALID_ARG, "SJLT needs 1 <= s <= min(m, 32)");
      if (s->m > 16384) return fail(LSQ_ERR_UNSUPPORTED, "SJLT with m > 16384 is not implemented");
      if ((int64_t)p->n * s->s >= ((int64_t)1 << 31))
        return fail(LSQ_ERR_UNSUPPORTED, "SJLT with n*s >= 2^31 is not implemented");
      break;
    case LSQ_GAUSSIAN:
      if (s->compute != LSQ_F64 && s->compute != LSQ_BF16 && s->compute != LSQ_F32)
        return fail(LSQ_ERR_INVALID_ARG, "Gaussian compute must be LSQ_F64, LSQ_F32 or LSQ_BF16");
      break;
    case LSQ_HAAR:
      if (s->compute != LSQ_F64) return fail(LSQ_ERR_INVALID_ARG, "Haar compute must be LSQ_F64");
      if (s->m > p->n) return fail(LSQ_ERR_INVALID_ARG, "Haar needs m <= n");
      // one Cholesky of the draws' Gram keeps the rows orthonormal to about u kappa(g)^2, and
      // kappa(g) <= (1 + sqrt(m/n)) / (1 - sqrt(m/n)) <= 3 for m <= n/4
      if (s->m > 1024 || 4 * s->m > p->n)
        return fail(LSQ_ERR_UNSUPPORTED, "Haar embedding limited to m <= min(1024, n/4)");
      break;
    default:
      return fail(LSQ_ERR_INVALID_ARG, "unknown sketch kind");
  }
  return LSQ_OK;
}

// ------------------------------------------------------------------------------------------------
// sketch
// ------------------------------------------------------------------------------------------------
// grad (optional): for an SRHT sketch whose first pass takes the vector form, *grad points at the N2
// partial rows of A^T y left by that pass and *grad_rows = N2; otherwise *grad = nullptr.
static lsq_status do_sketch(lsq_ctx* c, const lsq_problem* p, const lsq_sketch_desc* s, uint64_t t,
                            double* SA, int64_t ldsa, double** grad = nullptr, int* grad_rows = nullptr) {
  if (grad) *grad = nullptr;
  const hipStream_t st = c->st;
  const int a_f32 = p->a_dtype == LSQ_F32;
  if (s->kind == LSQ_SRHT) {
    const int64_t N = next_pow2(p->n);
    int8_t* signs;
    uint64_t* keys;
    int64_t* rows;
    int *hist, *bcount, *slot, *order, *bstart;
    void* state;
    CHK(wsT(c, "srht_signs", N, &signs));
    CHK(wsT(c, "srht_keys", N, &keys));
    CHK(wsT(c, "srht_rows", s->m, &rows));
    CHK(wsT(c, "sel_hist", 65536, &hist));
    CHK(wsT(c, "sel_bcount", srht_select_bcount_len(N), &bcount));
    CHK(ws(c, "sel_state", 64, &state));
    launch_srht_draw(st, s->seed, t, N, signs, keys);
    srht_select(st, keys, N, s->m, rows, SelectScratch{hist, bcount, state});
    SrhtPlan plan;
    plan.N = N;
    plan.N1 = N < 256 ? N : 256;
    plan.N2 = N / plan.N1;
    plan.m = s->m;
    plan.passb = c->srht_passb;
    CHK(wsT(c, "srht_slot", plan.N1, &slot));
    CHK(wsT(c, "srht_order", s->m, &order));
    CHK(wsT(c, "srht_bstart", plan.N1 + 1, &bstart));
    srht_plan_groups(st, rows, s->m, plan.N1, slot, order, bstart, c->dflags + 2);
    // T is sized for every bucket a selected row can fall in (the count of distinct buckets stays on the
    // device, so the sketch needs no host round trip)
    plan.nneeded = (int)std::min<int64_t>(plan.N1, s->m);
    const int cf32 = s->compute == LSQ_F32;
    void* tbuf;
    CHK(ws(c, "srht_tbuf", srht_tbuf_bytes(plan.N2, plan.nneeded, p->d, cf32), &tbuf));
    double* partial;
    CHK(wsT(c, "srht_partial", srht_partial_bytes(plan.N2, s->m, p->d) / sizeof(double), &partial));
    double* gpart = nullptr;
    if (grad) CHK(wsT(c, "srht_grad", (size_t)plan.N2 * (p->d + 1), &gpart));
    if (srht_apply(st, p->A, a_f32, p->n, p->d, p->lda, cf32, plan, signs, rows, slot, order, bstart, tbuf,
                   partial, SA, ldsa, p->y, gpart)) {
      *grad = gpart;
      *grad_rows = (int)plan.N2;
    }
  } else if (s->kind == LSQ_SJLT) {
    SjltScratch sc;
    const int64_t nblk = sjlt_nblk(p->n);
    const int64_t ns = p->n * s->s;
    CHK(wsT(c, "sjlt_targets", ns, &sc.targets));
    CHK(wsT(c, "sjlt_signs", ns, &sc.signs));
    CHK(wsT(c, "sjlt_cnt", s->m * nblk, &sc.cnt));
    CHK(wsT(c, "sjlt_off", s->m * nblk, &sc.off));
    CHK(wsT(c, "sjlt_scan", scan_tmp_len(s->m * nblk), &sc.scan_tmp));
    CHK(wsT(c, "sjlt_sorted", ns, &sc.sorted));
    CHK(wsT(c, "sjlt_bstart", s->m + 1, &sc.bstart));
    sc.err = c->dflags + 1;
    HIPCHK(hipMemsetAsync(sc.err, 0, sizeof(int), st));
    sjlt_apply(st, s->seed, t, p->A, a_f32, p->n, p->d, p->lda, s->m, s->s, sc, SA, ldsa);
    HIPCHK(hipMemcpyAsync(c->hflags + 1, c->dflags + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (c->hflags[1]) return fail(LSQ_ERR_INVALID_ARG, "SJLT draw limit exhausted (s too close to m)");
  } else if (s->kind == LSQ_HAAR) {
    // S = Q^T for the positive-diagonal QR g^T = Q R_g of the unscaled Gaussian draws g (m x n), without
    // forming Q: S A = R_g^{-T} (g A), R_g^T R_g = g g^T.  With the Gaussian sketch G_s = g / sqrt(m):
    // Y = G_s A and Z = G_s g^T (the Gaussian sketch of the drawn n x m matrix g^T), so g A = sqrt(m) Y
    // and g g^T = sqrt(m) Z.
    const int64_t m = s->m, n = p->n, d = p->d, mp = cholqr_padded(m);
    double* Gt;
    double *Y, *Z, *W, *scr, *tscr, *part;
    CHK(wsT(c, "haar_gt", (size_t)n * m, &Gt));
    CHK(wsT(c, "haar_y", (size_t)m * d, &Y));
    CHK(wsT(c, "haar_z", (size_t)m * m, &Z));
    CHK(wsT(c, "haar_w", (size_t)mp * mp, &W));
    CHK(wsT(c, "haar_scr", spd_inverse_scratch_len(m), &scr));
    CHK(wsT(c, "haar_tscr", trinv_scratch_len(mp), &tscr));
    const size_t pb = std::max(gauss_partial_bytes(m, d, n, 0), gauss_partial_bytes(m, m, n, 0));
    CHK(wsT(c, "gauss_part", pb / sizeof(double) + 1, &part));
    launch_gauss_draw_t(st, s->seed, t, n, m, Gt);
    gauss_apply(st, s->seed, t, p->A, a_f32, n, d, p->lda, m, 0, part, Y, d);
    gauss_apply(st, s->seed, t, Gt, 0, n, m, m, m, 0, part, Z, m);
    HIPCHK(hipMemsetAsync(c->dflags + 6, 0, sizeof(int), st));
    const double rm = sqrt((double)m);
    spd_chol_inverse(st, Z, m, rm, scr, W, c->dflags + 6, tscr);
    haar_apply(st, W, mp, Y, m, d, rm, SA, ldsa);
    HIPCHK(hipMemcpyAsync(c->hflags + 6, c->dflags + 6, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (c->hflags[6]) return fail(LSQ_ERR_RANK, "Haar embedding: the Gram of the Gaussian draws is not positive definite");
  } else {
    double* part;
    const int bf16 = s->compute == LSQ_BF16;
    CHK(wsT(c, "gauss_part", gauss_partial_bytes(s->m, p->d, p->n, bf16) / sizeof(double) + 1, &part));
    gauss_apply(st, s->seed, t, p->A, a_f32, p->n, p->d, p->lda, s->m, bf16, part, SA, ldsa);
  }
  HIPCHK(hipGetLastError());
  return LSQ_OK;
}

// Factor S A -> R, W = R^{-1}, W^T.  CholeskyQR (Gram matrices on the matrix cores): the Cholesky factor
// of H_S when the spread of its diagonal is small, CholeskyQR2 when it is larger, Householder QR (m <= 8192)
// or shifted CholeskyQR3 (larger m) when the first Cholesky is not usable; the other forms by the context's
// option "factor".
static lsq_status do_factor(lsq_ctx* c, const double* SA, int64_t m, int64_t d, int64_t lds,
                            double* R, double* W, double* WT, bool pcg = false) {
  const hipStream_t st = c->st;
  double* tscr;
  CHK(wsT(c, "trinv", trinv_scratch_len(cholqr_padded(d)), &tscr));
  c->w_dense = 0;
  // A NaN or an infinity in A (or in a caller's S A) reaches S A: report it as such rather than as the
  // breakdown it would cause in the factorization
  HIPCHK(hipMemsetAsync(c->dflags + 7, 0, sizeof(int), st));
  nonfinite_scan(st, SA, m, d, lds, c->dflags + 7);
  HIPCHK(hipMemcpyAsync(c->hflags + 7, c->dflags + 7, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (c->hflags[7]) return fail(LSQ_ERR_NONFINITE, "S A holds a NaN or an infinity (non-finite values in A)");
  if (c->factor_mode == 3) {
    // column-pivoted QR: the basic solution on the kept columns for a rank-deficient S A
    double* qs;
    CHK(wsT(c, "qrcp", qrcp_scratch_len(m, d), &qs));
    c->svd_rank = qrcp_precond(st, SA, m, d, lds, SVD_RTOL, qs, tscr, R, W, WT, c->dflags + 6, c->hflags + 6);
    HIPCHK(hipGetLastError());
    c->w_dense = 1;
    if (c->svd_rank < 1) return fail(LSQ_ERR_RANK, "S A is zero");
    return LSQ_OK;
  }
  if (c->factor_mode == 2) {
    // SVD form: R by Householder QR (m <= 8192; a zero pivot is allowed, rank deficiency is handled by
    // the truncation) or CholeskyQR2, then one-sided Jacobi on R
    if (m <= QR_M_MAX) {
      double* X;
      CHK(wsT(c, "qr_x", (size_t)m * d + (size_t)d * d, &X));
      householder_qr(st, SA, m, d, lds, X, R, c->dflags);
    } else {
      double* cs;
      CHK(wsT(c, "cholqr", cholqr_scratch_len(m, d), &cs));
      if (cholqr_factor(st, SA, m, d, lds, cs, R, c->dflags + 4, c->hflags + 4, tscr) != 0)
        return fail(LSQ_ERR_UNSUPPORTED, "SVD form above m = 8192 needs a full-rank, moderately conditioned S A");
    }
    double* vs;
    CHK(wsT(c, "svd", svd_scratch_len(d), &vs));
    c->svd_rank = svd_precond(st, R, d, SVD_RTOL, vs, W, WT, c->dflags + 6, c->hflags + 6, &c->svd_sweeps);
    HIPCHK(hipGetLastError());
    c->w_dense = 1;
    if (c->svd_rank < 1) return fail(LSQ_ERR_RANK, "S A is zero");
    return LSQ_OK;
  }
  bool done = false;
  if (c->factor_mode == 0 || c->factor_mode == 4 || c->factor_mode == 5) {
    double* cs;
    CHK(wsT(c, "cholqr", cholqr_scratch_len(m, d), &cs));
    // one pass or two by the first factor's spread for PCG, whose answer the preconditioner's last digits do
    // not change; two for the others (IHS and FCG iterates are defined by H_S^{-1} itself)
    const int passes = c->factor_mode == 4 ? 2 : (c->factor_mode == 5 ? 1 : (pcg ? 0 : 2));
    if (cholqr_factor(st, SA, m, d, lds, cs, R, c->dflags + 4, c->hflags + 4, tscr, passes) == 0) {
      done = true;
    } else if (m > QR_M_MAX) {
      // the shift regularises the first pass; a breakdown in the later passes means rank deficiency
      cholqr3_shifted(st, SA, m, d, lds, cs, R, c->dflags + 4, tscr);
      HIPCHK(hipMemcpyAsync(c->hflags + 4, c->dflags + 4, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (c->hflags[4]) return fail(LSQ_ERR_RANK, "S A is numerically rank deficient (Cholesky breakdown)");
      done = true;
    }
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipMemsetAsync(c->dflags, 0, sizeof(int), st));
  if (done) {
    qr_rank_check(st, R, d, c->dflags);
  } else {
    if (m > QR_M_MAX) return fail(LSQ_ERR_UNSUPPORTED, "Householder QR limited to m <= 8192");
    double* X;
    CHK(wsT(c, "qr_x", (size_t)m * d + (size_t)d * d, &X));
    householder_qr(st, SA, m, d, lds, X, R, c->dflags);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->hflags, c->dflags, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (c->hflags[0]) return fail(LSQ_ERR_RANK, "S A is numerically rank deficient (zero pivot in R)");
  tri_inverse(st, R, d, W, WT, tscr);
  HIPCHK(hipGetLastError());
  return LSQ_OK;
}

static EvPair* fused_event(lsq_ctx* c) {
  if (c->fused_used == c->fused_ev.size()) {
    EvPair e;
    // device-scope release: timing events must not add system-scope cache flushes between kernels
    if (hipEventCreateWithFlags(&e.a, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&e.b, hipEventDisableSystemFence) != hipSuccess)
      return nullptr;
    c->fused_ev.push_back(e);
  }
  return &c->fused_ev[c->fused_used++];
}

// Sum the first `count` recorded fused-pass event pairs (the stream has been synchronised).
static void fused_account(lsq_ctx* c, size_t first, size_t count) {
  for (size_t i = first; i < first + count && i < c->fused_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->fused_ev[i].a, c->fused_ev[i].b) == hipSuccess) {
      c->fused_total_ms += ms;
      c->fused_last_ms = ms;
      c->fused_count += 1;
    }
  }
}

struct SolveBufs {
  double *r, *rhat, *u, *p, *part, *part2, *dotpart, *red, *dx;
  int nwg;
};

static lsq_status solve_bufs(lsq_ctx* c, int64_t n, int64_t d, SolveBufs* b) {
  b->nwg = fused_nwg(n, d);
  CHK(wsT(c, "v_r", d, &b->r));
  CHK(wsT(c, "v_rhat", d, &b->rhat));
  CHK(wsT(c, "v_u", d, &b->u));
  CHK(wsT(c, "v_p", d, &b->p));
  CHK(wsT(c, "v_dx", d, &b->dx));
  CHK(wsT(c, "v_red", d + 1, &b->red));
  CHK(wsT(c, "part", (size_t)b->nwg * (d + 1), &b->part));
  CHK(wsT(c, "part2", (size_t)REDUCE_SPLIT * (d + 1), &b->part2));
  CHK(wsT(c, "dotpart", (d + 3) / 4 + 1, &b->dotpart));
  return LSQ_OK;
}

// PCG iterations on H z = r_0 from the state prepared by pcg_init (r, rhat, p already set).
// z accumulates the iterate.  Returns the number of iterations run; fused passes are timed.
static lsq_status pcg_loop(lsq_ctx* c, const lsq_problem* pr, int f32_math, const double* W,
                           const double* WT, SolveBufs& b, double* z, int max_iter, int check_every,
                           const double* x_ref, double* trace, int trace_len, int* iters_out) {
  const int64_t d = pr->d;
  const int a_f32 = pr->a_dtype == LSQ_F32;
  const size_t ev0 = c->fused_used;
  int it = 0;
  CHK(sync_state(c));
  bool done = c->hds->done != 0;
  // Batches of iterations are queued between host checks of the device stop flag.  After the first
  // batch the remaining count is predicted from the observed contraction of the stop-rule estimate,
  // so that almost no iterations are queued past convergence.
  double prev_proxy = -1.0;
  int prev_it = 0;
  const double tol = c->hds->tol;
  while (!done && it < max_iter) {
    int k = std::min(check_every, max_iter - it);
    const double proxy = c->hds->rho0 > 0.0 ? 4.0 * sqrt(fmax(c->hds->rho, 0.0) / c->hds->rho0) : 0.0;
    double rate = -1.0;
    if (prev_proxy > 0.0 && proxy > 0.0 && proxy < prev_proxy && it > prev_it)
      rate = pow(proxy / prev_proxy, 1.0 / (it - prev_it));
    else if (it == 0)
      rate = c->last_rate;  // first batch: the rate of the previous solve on this context
    if (tol > 0.0 && proxy > 0.0 && rate > 0.0 && rate < 1.0) {
      const double need = ceil(log(tol / proxy) / log(rate));
      if (need >= 1.0 && need < k) k = (int)need;
      if (it > 0) c->last_rate = rate;
    }
    prev_proxy = proxy;
    prev_it = it;
    for (int q = 0; q < k; ++q) {
      EvPair* e = fused_event(c);
      if (e) HIPCHK(hipEventRecord(e->a, c->st));
      const int ng_ = fused_pass(c->st, pr->A, a_f32, f32_math, pr->n, d, pr->lda, 0, b.p, nullptr, b.part, b.nwg,
                 &c->ds->done);
      if (e) HIPCHK(hipEventRecord(e->b, c->st));
      reduce_stage1(c->st, b.part, ng_, d, b.part2, &c->ds->done);
      pcg_update_xr(c->st, b.part2, REDUCE_SPLIT, d, z, b.r, b.p, c->ds);
      int ndot;
      precond_apply_any(c->st, W, WT, d, b.r, b.u, b.rhat, b.dotpart, &ndot, &c->ds->done, c->w_dense);
      pcg_update_p(c->st, d, b.rhat, b.p, b.dotpart, ndot, c->ds, z, b.r, x_ref, trace, trace_len);
    }
    HIPCHK(hipGetLastError());
    CHK(sync_state(c));
    it += k;
    done = c->hds->done != 0;
  }
  *iters_out = c->hds->iters;
  fused_account(c, ev0, (size_t)c->hds->iters);
  c->fused_used = ev0;  // recycle the events
  return LSQ_OK;
}

// ------------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------------
extern "C" {

const char* lsq_version(void) { return "liblsq 0.1 (gfx950)"; }

const char* lsq_status_string(lsq_status s) {
  switch (s) {
    case LSQ_OK: return "ok";
    case LSQ_ERR_INVALID_ARG: return "invalid argument";
    case LSQ_ERR_RANK: return "rank deficient or breakdown";
    case LSQ_ERR_NOT_CONVERGED: return "not converged";
    case LSQ_ERR_NONFINITE: return "non-finite value";
    case LSQ_ERR_HIP: return "HIP runtime error";
    case LSQ_ERR_NOMEM: return "out of device memory";
    case LSQ_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* lsq_last_error(void) { return g_err.c_str(); }

lsq_status lsq_create(lsq_ctx** out, void* stream) {
  if (!out) return fail(LSQ_ERR_INVALID_ARG, "null output pointer");
  lsq_ctx* c = new lsq_ctx();
  c->st = (hipStream_t)stream;
  if (hipGetDevice(&c->dev) != hipSuccess) {
    delete c;
    return fail(LSQ_ERR_HIP, "hipGetDevice failed");
  }
  bool ok = hipMalloc(&c->ds, sizeof(DevState)) == hipSuccess &&
            hipHostMalloc(&c->hds, sizeof(DevState), hipHostMallocDefault) == hipSuccess &&
            hipMalloc(&c->dflags, 8 * sizeof(int)) == hipSuccess &&
            hipHostMalloc(&c->hflags, 8 * sizeof(int), hipHostMallocDefault) == hipSuccess;
  for (int i = 0; ok && i < 6; ++i) ok = hipEventCreate(&c->ev[i]) == hipSuccess;
  if (!ok) {
    lsq_destroy(c);
    return fail(LSQ_ERR_HIP, "context allocation failed");
  }
  hipMemset(c->ds, 0, sizeof(DevState));
  hipMemset(c->dflags, 0, 8 * sizeof(int));
  // the allocation-free entry point's array: its address on this (current) device, once per device
  if (noalloc_scratch(c->dev, &c->noalloc) != hipSuccess) {
    lsq_destroy(c);
    return fail(LSQ_ERR_HIP, "hipGetSymbolAddress of the static partials array failed");
  }
  *out = c;
  return LSQ_OK;
}

void lsq_destroy(lsq_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  else (void)hipDeviceSynchronize();
  for (auto& kv : c->bufs)
    if (kv.second.first) (void)hipFree(kv.second.first);
  for (auto& e : c->fused_ev) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (int i = 0; i < 6; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  for (int i = 0; i < 3; ++i)
    if (c->bev[i]) (void)hipEventDestroy(c->bev[i]);
  if (c->bexec) (void)hipGraphExecDestroy(c->bexec);
  if (c->bgraph) (void)hipGraphDestroy(c->bgraph);
  if (c->bst) {
    (void)hipStreamSynchronize(c->bst);
    (void)hipStreamDestroy(c->bst);
  }
  if (c->bhost) (void)hipHostFree(c->bhost);
  if (c->ds) (void)hipFree(c->ds);
  if (c->dflags) (void)hipFree(c->dflags);
  if (c->hds) (void)hipHostFree(c->hds);
  if (c->hx) (void)hipHostFree(c->hx);
  if (c->hflags) (void)hipHostFree(c->hflags);
  delete c;
}

lsq_status lsq_sketch(lsq_ctx* c, const lsq_problem* p, const lsq_sketch_desc* s, void* SA,
                      int64_t ldsa, int32_t sa_dtype) {
  CHK(check_problem(c, p));
  CHK(check_sketch(c, p, s, false));
  if (!SA) return fail(LSQ_ERR_INVALID_ARG, "null SA");
  if (ldsa < p->d) return fail(LSQ_ERR_INVALID_ARG, "ldsa < d");
  if (sa_dtype != LSQ_F64) return fail(LSQ_ERR_INVALID_ARG, "sa_dtype must be LSQ_F64");
  CHK(do_sketch(c, p, s, s->t, (double*)SA, ldsa));
  HIPCHK(hipStreamSynchronize(c->st));
  return LSQ_OK;
}

lsq_status lsq_factor(lsq_ctx* c, const double* SA, int64_t m, int64_t d, int64_t lds, double* R,
                      double* W) {
  if (!c || !SA) return fail(LSQ_ERR_INVALID_ARG, "null context or SA");
  if (d < 1 || m < d || lds < d) return fail(LSQ_ERR_INVALID_ARG, "need m >= d >= 1 and lds >= d");
  if (d > 1024 || m > FACTOR_M_MAX) return fail(LSQ_ERR_UNSUPPORTED, "factor limited to d <= 1024, m <= 65536");
  double *Rb, *Wb, *WTb;
  CHK(wsT(c, "f_R", (size_t)d * d, &Rb));
  CHK(wsT(c, "f_W", (size_t)d * d, &Wb));
  CHK(wsT(c, "f_WT", (size_t)d * d, &WTb));
  CHK(do_factor(c, SA, m, d, lds, Rb, Wb, WTb));
  if (R) HIPCHK(hipMemcpyAsync(R, Rb, sizeof(double) * d * d, hipMemcpyDeviceToDevice, c->st));
  if (W) HIPCHK(hipMemcpyAsync(W, Wb, sizeof(double) * d * d, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return LSQ_OK;
}

lsq_status lsq_fused_pass(lsq_ctx* c, const lsq_problem* p, int32_t mode, int32_t f32_math,
                          const double* v, double* w, double* scal) {
  CHK(check_problem(c, p));
  if (!v || !w || !scal) return fail(LSQ_ERR_INVALID_ARG, "null v, w or scal");
  if (mode < 0 || mode > 2) return fail(LSQ_ERR_INVALID_ARG, "mode must be 0, 1 or 2");
  if (f32_math && (p->a_dtype != LSQ_F32 || mode == 2))
    return fail(LSQ_ERR_INVALID_ARG, "f32_math needs an FP32 matrix and mode 0 or 1");
  if (mode == 2) {
    double* part;
    CHK(wsT(c, "resid_dd", resid_dd_part_len(p->d), &part));
    if (!resid_dd(c->st, p->A, p->a_dtype == LSQ_F32, p->n, p->d, p->lda, v, p->y, part, w, scal))
      return fail(LSQ_ERR_UNSUPPORTED, "double-double residual limited to d <= 1024");
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return LSQ_OK;
  }
  SolveBufs b;
  CHK(solve_bufs(c, p->n, p->d, &b));
  EvPair* e = fused_event(c);
  const size_t ev0 = c->fused_used - 1;
  if (e) HIPCHK(hipEventRecord(e->a, c->st));
  const int ng_ = fused_pass(c->st, p->A, p->a_dtype == LSQ_F32, f32_math, p->n, p->d, p->lda, mode, v, p->y, b.part,
             b.nwg, nullptr);
  if (e) HIPCHK(hipEventRecord(e->b, c->st));
  reduce_partials(c->st, b.part, b.part2, ng_, p->d, b.red, nullptr);
  vec_copy(c->st, w, b.red, p->d);
  vec_copy(c->st, scal, b.red + p->d, 1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  if (e) fused_account(c, ev0, 1);
  c->fused_used = ev0;
  return LSQ_OK;
}

lsq_status lsq_fused_pass_noalloc(lsq_ctx* c, const lsq_problem* p, int32_t mode, int32_t f32_math,
                                  const double* v, double* w, double* scal) {
  CHK(check_problem(c, p));
  if (!v || !w || !scal) return fail(LSQ_ERR_INVALID_ARG, "null v, w or scal");
  if (mode == 2)
    return fail(LSQ_ERR_UNSUPPORTED, "lsq_fused_pass_noalloc: mode 2 (double-double) needs more partials than "
                                     "the static array holds; use lsq_fused_pass");
  if (mode != 0 && mode != 1) return fail(LSQ_ERR_INVALID_ARG, "mode must be 0 or 1");
  if (f32_math && p->a_dtype != LSQ_F32) return fail(LSQ_ERR_INVALID_ARG, "f32_math needs an FP32 matrix");
  if (!c->noalloc) return fail(LSQ_ERR_HIP, "static partials array not available on this device");
  // partials (one row of d + 1 per workgroup), the REDUCE_SPLIT rows of the first reduction stage and
  // the reduced row, all inside the array: the workgroup count is capped to what fits
  const int64_t width = p->d + 1;
  const int64_t rows_fit = (int64_t)NOALLOC_DOUBLES / width - (REDUCE_SPLIT + 1);
  if (rows_fit < 1) return fail(LSQ_ERR_UNSUPPORTED, "lsq_fused_pass_noalloc: d too large for the static array");
  const int nwg = (int)std::min<int64_t>(fused_nwg(p->n, p->d), rows_fit);
  double* part = c->noalloc;
  double* part2 = part + (size_t)nwg * width;
  double* red = part2 + (size_t)REDUCE_SPLIT * width;
  const int ng_ = fused_pass(c->st, p->A, p->a_dtype == LSQ_F32, f32_math, p->n, p->d, p->lda, mode, v, p->y, part,
                             nwg, nullptr);
  reduce_partials(c->st, part, part2, ng_, p->d, red, nullptr);
  vec_copy(c->st, w, red, p->d);
  vec_copy(c->st, scal, red + p->d, 1);
  HIPCHK(hipGetLastError());
  return LSQ_OK;
}

lsq_status lsq_copy_bandwidth(lsq_ctx* c, const void* src, void* dst, int64_t bytes, int32_t reps, double* gbs) {
  if (!c || !src || !dst || !gbs) return fail(LSQ_ERR_INVALID_ARG, "null context, buffer or output");
  if (bytes < 16 || reps < 1) return fail(LSQ_ERR_INVALID_ARG, "need bytes >= 16 and reps >= 1");
  if ((uintptr_t)src % 16 || (uintptr_t)dst % 16) return fail(LSQ_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
  const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
  if (s0 < d0 + (uintptr_t)bytes && d0 < s0 + (uintptr_t)bytes)
    return fail(LSQ_ERR_INVALID_ARG, "source and destination overlap");
  int cus = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->dev));
  double best = 0.0;
  for (int gpc : {4, 8, 16}) {
    const int groups = std::max(cus, 1) * gpc;
    stream_copy(c->st, src, dst, bytes, groups);  // warm-up
    HIPCHK(hipEventRecord(c->ev[4], c->st));
    for (int r = 0; r < reps; ++r) stream_copy(c->st, src, dst, bytes, groups);
    HIPCHK(hipEventRecord(c->ev[5], c->st));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(c->ev[5]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[4], c->ev[5]));
    const double rate = 2.0 * (double)(bytes / 16 * 16) * reps / (ms * 1e-3) / 1e9;
    best = std::max(best, rate);
  }
  *gbs = best;
  return LSQ_OK;
}

lsq_status lsq_read_bandwidth(lsq_ctx* c, const void* buf, int64_t bytes, int32_t reps, double* gbs) {
  if (!c || !buf || !gbs) return fail(LSQ_ERR_INVALID_ARG, "null context, buffer or output");
  if (bytes < 16 || reps < 1) return fail(LSQ_ERR_INVALID_ARG, "need bytes >= 16 and reps >= 1");
  if ((uintptr_t)buf % 16) return fail(LSQ_ERR_INVALID_ARG, "buffer must be 16-byte aligned");
  int cus = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->dev));
  double best = 0.0;
  for (int gpc : {4, 8, 16}) {
    const int groups = std::max(cus, 1) * gpc;
    float* out;
    CHK(wsT(c, "read_probe", (size_t)groups, &out));
    stream_read(c->st, buf, bytes, groups, out);  // warm-up
    HIPCHK(hipEventRecord(c->ev[4], c->st));
    for (int r = 0; r < reps; ++r) stream_read(c->st, buf, bytes, groups, out);
    HIPCHK(hipEventRecord(c->ev[5], c->st));
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(c->ev[5]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[4], c->ev[5]));
    const double rate = (double)(bytes / 16 * 16) * reps / (ms * 1e-3) / 1e9;
    best = std::max(best, rate);
  }
  *gbs = best;
  return LSQ_OK;
}

lsq_status lsq_fused_pass_timing(lsq_ctx* c, int32_t reset, double* last_ms, double* avg_ms,
                                 int64_t* launches) {
  if (!c) return fail(LSQ_ERR_INVALID_ARG, "null context");
  if (last_ms) *last_ms = c->fused_last_ms;
  if (avg_ms) *avg_ms = c->fused_count ? c->fused_total_ms / c->fused_count : 0.0;
  if (launches) *launches = c->fused_count;
  if (reset) {
    c->fused_total_ms = 0.0;
    c->fused_count = 0;
  }
  return LSQ_OK;
}

// Solve the correction system H z = s (s = A^T (y - A x) held in b.r) with PCG from z = 0 and the
// relative tolerance tol_in; returns iterations.  b.rhat / b.p / dotpart prepared here.
static lsq_status inner_pcg(lsq_ctx* c, const lsq_problem* p, int f32_math, const double* W,
                            const double* WT, SolveBufs& b, double* z, double tol_in, int max_iter,
                            int check_every, const double* x_ref, double* trace, int trace_len,
                            int* iters) {
  int ndot;
  precond_apply_any(c->st, W, WT, p->d, b.r, b.u, b.rhat, b.dotpart, &ndot, nullptr, c->w_dense);
  pcg_init(c->st, p->d, b.rhat, b.p, b.dotpart, ndot, c->ds, tol_in, z, b.r, x_ref, trace);
  HIPCHK(hipGetLastError());
  return pcg_loop(c, p, f32_math, W, WT, b, z, max_iter, check_every, x_ref, trace, trace_len, iters);
}

lsq_status lsq_pcg_solve(lsq_ctx* c, const lsq_problem* p, const lsq_sketch_desc* s,
                         const lsq_pcg_opts* o, double* x, double* err_trace, lsq_info* info) {
  CHK(check_problem(c, p));
  CHK(check_sketch(c, p, s, true));
  if (!o || !x) return fail(LSQ_ERR_INVALID_ARG, "null options or x");
  if (o->max_iter < 1) return fail(LSQ_ERR_INVALID_ARG, "max_iter < 1");
  if (!(o->tol > 0.0) && o->stop_rule == 0) return fail(LSQ_ERR_INVALID_ARG, "tol must be > 0");
  if (o->mixed && o->max_refine < 1) return fail(LSQ_ERR_INVALID_ARG, "max_refine < 1");
  if (o->inner_f32 && (!o->mixed || p->a_dtype != LSQ_F32))
    return fail(LSQ_ERR_INVALID_ARG, "inner_f32 needs mixed = 1 and an FP32 matrix");
  const hipStream_t st = c->st;
  const int64_t d = p->d, m = s->m;
  const int check_every = o->check_every > 0 ? o->check_every : 8;
  double *SA, *R, *W, *WT;
  CHK(wsT(c, "SA", (size_t)m * d, &SA));
  CHK(wsT(c, "f_R", (size_t)d * d, &R));
  CHK(wsT(c, "f_W", (size_t)d * d, &W));
  CHK(wsT(c, "f_WT", (size_t)d * d, &WT));
  SolveBufs b;
  CHK(solve_bufs(c, p->n, d, &b));
  const double a_bytes = (double)p->n * d * (p->a_dtype == LSQ_F32 ? 4.0 : 8.0);

  // From x_0 = 0 the first gradient is A^T y, which the SRHT's first pass forms while it streams A
  // (do_sketch), saving a pass.
  if (c->hx_len < (size_t)d) {
    if (c->hx) HIPCHK(hipHostFree(c->hx));
    c->hx = nullptr;
    c->hx_len = 0;
    HIPCHK(hipHostMalloc(&c->hx, sizeof(double) * d, hipHostMallocDefault));
    c->hx_len = d;
  }
  HIPCHK(hipMemcpyAsync(c->hx, x, sizeof(double) * d, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  bool x0_zero = true;
  for (int64_t i = 0; i < d && x0_zero; ++i) x0_zero = c->hx[i] == 0.0;
  double* grad = nullptr;
  int grad_rows = 0;

  HIPCHK(hipEventRecord(c->ev[0], st));
  CHK(do_sketch(c, p, s, s->t, SA, d, x0_zero || o->x_ref ? &grad : nullptr, &grad_rows));
  HIPCHK(hipEventRecord(c->ev[1], st));
  CHK(do_factor(c, SA, m, d, d, R, W, WT, true));
  if (o->mixed && s->kind == LSQ_SRHT && s->compute == LSQ_F32 && c->sketch_upgrade) {
    // An FP32 transform perturbs S A by about its single-precision rounding; once kappa(A) approaches
    // 1/u32 that visibly weakens the preconditioner (at kappa = 1e8, 37 PCG iterations instead of 17).
    // The spread of diag(R), about kappa / 25, decides: above 1e6 the sketch is taken again with an FP64
    // transform of the same FP32 A.
    double* spr;
    CHK(wsT(c, "diag_spread", 1, &spr));
    diag_spread(st, R, d, spr);
    HIPCHK(hipMemcpyAsync(c->hx, spr, sizeof(double), hipMemcpyDeviceToHost, st));  // (x_0 was read above)
    HIPCHK(hipStreamSynchronize(st));
    const double spread = c->hx[0];
    if (spread > SKETCH_UPGRADE_SPREAD) {
      LSQ_TRACE("diag(R) spread %.3e > %.1e: FP32 transform replaced by an FP64 one", spread, SKETCH_UPGRADE_SPREAD);
      lsq_sketch_desc s64 = *s;
      s64.compute = LSQ_F64;
      CHK(do_sketch(c, p, &s64, s64.t, SA, d, x0_zero || o->x_ref ? &grad : nullptr, &grad_rows));
      HIPCHK(hipEventRecord(c->ev[1], st));
      CHK(do_factor(c, SA, m, d, d, R, W, WT, true));
    }
  }
  HIPCHK(hipEventRecord(c->ev[2], st));

  const int a_f32 = p->a_dtype == LSQ_F32;
  const double tol = o->stop_rule == 1 ? -1.0 : o->tol;
  int total_iters = 0, refinements = 0;
  double est = 0.0, passes = 0.0;
  const int trace_len = o->max_iter + 1;

  if (o->x_ref) {
    // x_ref^T b with b = A^T y: one residual pass at v = 0 (or the first pass's partials)
    if (grad) {
      reduce_partials(st, grad, b.part2, grad_rows, d, b.red, nullptr);
    } else {
      vec_zero(st, b.dx, d);
      const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 1, b.dx, p->y, b.part, b.nwg, nullptr);
      reduce_partials(st, b.part, b.part2, ng_, d, b.red, nullptr);
      passes += 1;
    }
    dot_to_state(st, d, o->x_ref, b.red, c->ds);
  }

  bool measured_ok = false;
  if (!o->mixed && o->stop_rule == 1) {
    // exactly max_iter PCG iterations from r_0 = A^T (y - A x_0)
    if (grad && x0_zero) {
      reduce_partials(st, grad, b.part2, grad_rows, d, b.r, nullptr);
    } else {
      const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 1, x, p->y, b.part, b.nwg, nullptr);
      reduce_partials(st, b.part, b.part2, ng_, d, b.r, nullptr);
      passes += 1;
    }
    int it = 0;
    CHK(inner_pcg(c, p, 0, W, WT, b, x, tol, o->max_iter, check_every, o->x_ref, err_trace, trace_len,
                  &it));
    total_iters = it;
    passes += it;
    est = c->hds->est;
  } else {
    // PCG on the correction system H dx = r from an accurate residual r = A^T (y - A x), then x += dx
    // and a new residual in double-double arithmetic (rounded once) measures the result.  PCG's
    // recursively updated residual drifts from the true one by about u kappa(A) relative to its start,
    // so near the FP64 conditioning floor it reports progress that x no longer makes; the measured
    // residual exposes that, and the next correction starts from it (residual replacement).  The plain
    // form (FP64 A as given, FP64 arithmetic) and the mixed form (FP32 storage of A read into FP64
    // registers, or FP32 arithmetic with inner_f32) share this loop; the plain form's first correction
    // accumulates into x itself, so that its error trace follows the iterates.
    double rho_b = -1.0, est_meas_prev = -1.0, est_exact = -1.0;
    const double floor_in = o->inner_f32 ? 1e-6 : 1e-13;
    const int max_steps = std::max(o->max_refine, 1);
    double* rpart;
    CHK(wsT(c, "resid_dd", resid_dd_part_len(d), &rpart));
    if (d > 1024) return fail(LSQ_ERR_UNSUPPORTED, "double-double residual limited to d <= 1024");
    // From x_0 = 0 the first residual is A^T y, with no cancellation: FP64 products and sums (the SRHT's
    // first pass, or one plain pass) give it to working accuracy.  Any other start takes the
    // double-double residual from the outset.
    double est_carried = -1.0;
    for (int k = 0; k <= max_steps; ++k) {
      // After a correction solved from an accurate residual (k >= 2: the first check, k = 1, measures
      // the PCG's own drift and is always taken), the new error estimate is the old one times the
      // correction solve's relative reduction; the rounding inside that solve is relative to the
      // correction, so the carried value stands in for one more residual.
      if (k >= 2 && o->stop_rule == 0 && !o->x_ref && est_carried >= 0.0 && est_carried <= o->tol) {
        est = est_carried;
        LSQ_TRACE("pcg step %d: carried estimate %.3e <= tol, done", k, est);
        measured_ok = true;
        break;
      }
      const bool measured = !(k == 0 && x0_zero);
      if (k == 0 && x0_zero && grad) {
        reduce_partials(st, grad, b.part2, grad_rows, d, b.r, nullptr);
      } else if (k == 0 && x0_zero) {
        const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 1, x, p->y, b.part, b.nwg, nullptr);
        reduce_partials(st, b.part, b.part2, ng_, d, b.r, nullptr);
        passes += 1;
      } else if (!resid_dd(st, p->A, a_f32, p->n, d, p->lda, x, p->y, rpart, b.r, nullptr)) {
        return fail(LSQ_ERR_UNSUPPORTED, "double-double residual limited to d <= 1024");
      } else {
        passes += 1;
      }
      int ndot;
      precond_apply_any(st, W, WT, d, b.r, b.u, b.rhat, b.dotpart, &ndot, nullptr, c->w_dense);
      // (with x_ref: the exact error of x, from this residual)
      pcg_init(st, d, b.rhat, b.p, b.dotpart, ndot, c->ds, 1.0, x, b.r, o->x_ref, nullptr);
      CHK(sync_state(c));
      if (c->hds->status) break;  // a non-finite residual
      if (o->x_ref) est_exact = c->hds->est;
      const double rho_s = c->hds->rho0;
      if (rho_b < 0.0) rho_b = rho_s;  // relative to the starting residual (x_0 = 0: to ||A x*||)
      est = rho_b > 0.0 ? 4.0 * sqrt(fmax(rho_s, 0.0) / rho_b) : 0.0;
      LSQ_TRACE("pcg step %d: %s residual, estimate %.3e (carried %.3e)", k,
                measured ? "measured" : "first", est, est_carried);
      if (o->stop_rule == 0 && est <= o->tol) {
        measured_ok = true;
        break;
      }
      if (o->stop_rule == 1 && k > 0) break;
      if (k == max_steps) break;  // budget of corrections spent
      // a measured residual that did not halve since the last one: x is at the attainable accuracy
      if (measured && est_meas_prev > 0.0 && est > 0.5 * est_meas_prev) {
        LSQ_TRACE("pcg step %d: no progress since the last measured residual (%.3e), stop", k, est_meas_prev);
        break;
      }
      if (measured) est_meas_prev = est;
      refinements += 1;
      // the inner stop rule bounds the error of the correction relative to the current error, whose
      // estimate is est = 4 sqrt(rho_s / rho_b): asking 0.9 tol / (est / 4) of it lands at 0.9 tol
      const double rel = fmax(est / 4.0, 1e-300);
      const double tol_in = o->stop_rule == 1 ? -1.0 : fmax(0.9 * o->tol / rel, floor_in);
      const bool direct = !o->mixed && k == 0;  // the plain form's first correction: into x
      double* z = direct ? x : b.dx;
      if (!direct) vec_zero(st, b.dx, d);
      int it = 0;
      CHK(inner_pcg(c, p, o->inner_f32, W, WT, b, z, tol_in, o->max_iter, check_every,
                    direct ? o->x_ref : nullptr, direct ? err_trace : nullptr, direct ? trace_len : 0, &it));
      total_iters += it;
      passes += it;
      LSQ_TRACE("pcg step %d: correction solve to %.3e relative: %d iterations, its estimate %.3e%s", k, tol_in,
                it, c->hds->est, c->hds->done ? "" : " (budget spent)");
      if (c->hds->status) break;
      est_carried = est * (c->hds->est / 4.0);
      if (!direct) vec_axpy(st, x, b.dx, 1.0, d);
      if (!c->hds->done && o->stop_rule == 0) break;  // the iteration budget ended this solve
    }
    if (o->x_ref && est_exact >= 0.0) est = est_exact;
  }
  HIPCHK(hipEventRecord(c->ev[3], st));
  HIPCHK(hipStreamSynchronize(st));
  const int dev_status = c->hds->status;
  if (info) {
    float ms;
    info->iters = total_iters;
    info->refinements = refinements;
    info->est_rel_err = est;
    hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    info->t_sketch_ms = ms;
    hipEventElapsedTime(&ms, c->ev[1], c->ev[2]);
    info->t_factor_ms = ms;
    hipEventElapsedTime(&ms, c->ev[2], c->ev[3]);
    info->t_iter_ms = ms;
    hipEventElapsedTime(&ms, c->ev[0], c->ev[3]);
    info->t_total_ms = ms;
    info->bytes_streamed = passes * a_bytes;
    info->mu = 0.0;
    info->pad_ = 0;
    info->t_start_ms = 0.0;
  }
  lsq_status ret = LSQ_OK;
  if (dev_status == LSQ_ERR_RANK) ret = fail(LSQ_ERR_RANK, "breakdown: p^T H p <= 0");
  else if (dev_status == LSQ_ERR_NONFINITE) ret = fail(LSQ_ERR_NONFINITE, "non-finite value in PCG");
  else if (o->stop_rule == 0 && !measured_ok)
    ret = fail(LSQ_ERR_NOT_CONVERGED, "the measured residual did not meet the tolerance within the budget");
  if (info) info->status = ret;
  return ret;
}

// Section 6's iteration model: T(m) = ceil(log(4 / eps) / log(m / d)), eps = tol^2 (rho = d/m).
static int msize_iterations(int64_t m, int64_t d, double tol) {
  if (m <= d) return 1 << 30;
  return (int)ceil(log(4.0 / (tol * tol)) / log((double)m / (double)d));
}

// Candidate sketch sizes: 1.5 d .. 64 d (multiples of 64 for d >= 64), above d, within the
// factorization's limit and the embedding's own (m <= N for the SRHT, 16384 for the SJLT, min(1024, n/4)
// for Haar).
static std::vector<int64_t> msize_candidates(int64_t n, int64_t d, int kind) {
  int64_t hi = FACTOR_M_MAX;
  if (kind == LSQ_SRHT) hi = std::min(hi, next_pow2(n));
  if (kind == LSQ_SJLT) hi = std::min<int64_t>(hi, 16384);
  if (kind == LSQ_HAAR) hi = std::min<int64_t>(std::min<int64_t>(hi, 1024), n / 4);
  std::vector<int64_t> out;
  for (double f : {1.5, 2.0, 3.0, 4.0, 5.0, 6.0, 8.0, 10.0, 12.0, 16.0, 24.0, 32.0, 40.0, 48.0, 64.0}) {
    const int64_t m = d >= 64 ? (int64_t)llround(f * d / 64.0) * 64 : (int64_t)llround(f * d);
    if (m > d && m <= hi && std::find(out.begin(), out.end(), m) == out.end()) out.push_back(m);
  }
  return out;
}

lsq_status lsq_choose_sketch_size(lsq_ctx* c, const lsq_problem* p, const lsq_sketch_desc* s, double tol,
                                  double extra_passes, int32_t reps, lsq_msize_entry* table, int32_t capacity,
                                  int32_t* count, int64_t* m_best, double* t_pass_ms) {
  CHK(check_problem(c, p));
  if (!s || !m_best) return fail(LSQ_ERR_INVALID_ARG, "null descriptor or output");
  if (!(tol > 0.0 && tol < 1.0)) return fail(LSQ_ERR_INVALID_ARG, "tol must lie in (0, 1)");
  if (reps < 1 || extra_passes < 0.0) return fail(LSQ_ERR_INVALID_ARG, "need reps >= 1, extra_passes >= 0");
  if (table && capacity < 1) return fail(LSQ_ERR_INVALID_ARG, "table without capacity");
  const int64_t n = p->n, d = p->d;
  const std::vector<int64_t> cand = msize_candidates(n, d, s->kind);
  if (cand.empty()) return fail(LSQ_ERR_UNSUPPORTED, "no sketch size between d and the embedding's limit");
  if (table && capacity < (int32_t)cand.size()) return fail(LSQ_ERR_INVALID_ARG, "table capacity below the candidate count");
  const hipStream_t st = c->st;
  double *SA, *R, *W, *WT, *spr;
  CHK(wsT(c, "SA", (size_t)cand.back() * d, &SA));
  CHK(wsT(c, "f_R", (size_t)d * d, &R));
  CHK(wsT(c, "f_W", (size_t)d * d, &W));
  CHK(wsT(c, "f_WT", (size_t)d * d, &WT));
  CHK(wsT(c, "diag_spread", 1, &spr));
  // one fused pass (H v), the unit of the iteration term
  SolveBufs b;
  CHK(solve_bufs(c, n, d, &b));
  vec_zero(st, b.p, d);
  double t_pass = 1e300;
  for (int r = 0; r <= 3; ++r) {
    HIPCHK(hipEventRecord(c->ev[4], st));
    const int ng_ = fused_pass(st, p->A, p->a_dtype == LSQ_F32, 0, n, d, p->lda, 0, b.p, nullptr, b.part, b.nwg, nullptr);
    HIPCHK(hipEventRecord(c->ev[5], st));
    reduce_partials(st, b.part, b.part2, ng_, d, b.red, nullptr);
    HIPCHK(hipEventSynchronize(c->ev[5]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->ev[4], c->ev[5]));
    if (r > 0) t_pass = std::min(t_pass, (double)ms);  // the first launch is a warm-up
  }
  int64_t best = -1;
  double best_pred = 1e300;
  for (size_t i = 0; i < cand.size(); ++i) {
    lsq_sketch_desc sd = *s;
    sd.m = cand[i];
    CHK(check_sketch(c, p, &sd, true));
    double ts = 1e300, tf = 1e300;
    for (int r = 0; r <= reps; ++r) {
      HIPCHK(hipEventRecord(c->ev[0], st));
      CHK(do_sketch(c, p, &sd, sd.t, SA, d));
      HIPCHK(hipEventRecord(c->ev[1], st));
      CHK(do_factor(c, SA, sd.m, d, d, R, W, WT, true));
      HIPCHK(hipEventRecord(c->ev[2], st));
      HIPCHK(hipEventSynchronize(c->ev[2]));
      float a = 0.f, f = 0.f;
      HIPCHK(hipEventElapsedTime(&a, c->ev[0], c->ev[1]));
      HIPCHK(hipEventElapsedTime(&f, c->ev[1], c->ev[2]));
      if (r > 0 || reps == 0) {  // the first round also loads code and grows the workspace
        ts = std::min(ts, (double)a);
        tf = std::min(tf, (double)f);
      }
    }
    diag_spread(st, R, d, spr);
    HIPCHK(hipMemcpyAsync(c->hflags, spr, sizeof(double), hipMemcpyDeviceToHost, st));  // (8 pinned ints)
    HIPCHK(hipStreamSynchronize(st));
    double spread;
    memcpy(&spread, c->hflags, sizeof(double));
    const int T = msize_iterations(sd.m, d, tol);
    const double pred = ts + tf + (T + extra_passes) * t_pass;
    LSQ_TRACE("sketch size %lld: sketch %.3f ms factor %.3f ms T %d predicted %.2f ms (diag spread %.2e)",
              (long long)sd.m, ts, tf, T, pred, spread);
    if (table) {
      table[i].m = sd.m;
      table[i].iters = T;
      table[i].pad_ = 0;
      table[i].t_sketch_ms = ts;
      table[i].t_factor_ms = tf;
      table[i].predicted_ms = pred;
      table[i].r_spread = spread;
    }
    if (pred < best_pred) {  // ties keep the smaller m
      best_pred = pred;
      best = sd.m;
    }
  }
  if (count) *count = (int32_t)cand.size();
  if (t_pass_ms) *t_pass_ms = t_pass;
  *m_best = best;
  return LSQ_OK;
}

lsq_status lsq_ihs_solve(lsq_ctx* c, const lsq_problem* p, const lsq_sketch_desc* s,
                         const lsq_ihs_opts* o, double* x, double* err_trace, lsq_info* info) {
  CHK(check_problem(c, p));
  CHK(check_sketch(c, p, s, true));
  if (!o || !x) return fail(LSQ_ERR_INVALID_ARG, "null options or x");
  if (o->iters < 0) return fail(LSQ_ERR_INVALID_ARG, "iters < 0");
  if (err_trace && !o->x_ref) return fail(LSQ_ERR_INVALID_ARG, "err_trace needs x_ref");
  const int64_t d = p->d, m = s->m;
  double mu = o->mu;
  if (o->mu_rule == 0) {
    if (s->kind == LSQ_GAUSSIAN) {
      if (m < d + 4) return fail(LSQ_ERR_INVALID_ARG, "Gaussian step rule needs m >= d + 4");
      const double md = (double)m, dd = (double)d;
      const double t1 = md / (md - dd - 1.0);
      const double t2 = md * md * (md - 1.0) / ((md - dd) * (md - dd - 1.0) * (md - dd - 3.0));
      mu = t1 / t2;
    } else if (s->kind == LSQ_SRHT) {
      if (m <= d) return fail(LSQ_ERR_INVALID_ARG, "SRHT step rule needs m > d");
      const double N = (double)next_pow2(p->n), md = (double)m, dd = (double)d;
      const double t1 = (N - dd) / (md - dd);
      const double t2 = (N - dd) * (dd * dd + md * N - 2.0 * dd * md) / ((md - dd) * (md - dd) * (md - dd));
      mu = (N / md) * t1 / t2;
    } else if (s->kind == LSQ_HAAR) {
      // Section 2's Haar theta's (orthonormal rows, no rescaling)
      if (m <= d) return fail(LSQ_ERR_INVALID_ARG, "Haar step rule needs m > d");
      const double nn = (double)p->n, md = (double)m, dd = (double)d;
      const double t1 = (nn - dd) / (md - dd);
      const double t2 = (nn - dd) * (dd * dd + md * nn - 2.0 * dd * md) / ((md - dd) * (md - dd) * (md - dd));
      mu = t1 / t2;
    } else {
      return fail(LSQ_ERR_INVALID_ARG, "the SJLT has no closed-form step: use mu_rule = 1");
    }
  } else if (o->mu_rule == 2 || o->mu_rule == 3) {
    // Theorem 3.2 with rho = d/m: IHS step (1 - rho)^2 / (1 + rho); Polyak mu = (1 - rho)^2, beta = rho
    if (m <= d) return fail(LSQ_ERR_INVALID_ARG, "the fixed-sketch rules need m > d");
    const double rho = (double)d / (double)m;
    mu = o->mu_rule == 2 ? (1.0 - rho) * (1.0 - rho) / (1.0 + rho) : (1.0 - rho) * (1.0 - rho);
  } else if (o->mu_rule != 1) {
    return fail(LSQ_ERR_INVALID_ARG, "mu_rule must be 0, 1, 2 or 3");
  }
  const double beta = o->mu_rule == 3 ? (double)d / (double)m : o->beta;
  const hipStream_t st = c->st;
  const int a_f32 = p->a_dtype == LSQ_F32;
  double *SA, *R, *W, *WT, *xprev, *diff, *errv;
  CHK(wsT(c, "SA", (size_t)m * d, &SA));
  CHK(wsT(c, "f_R", (size_t)d * d, &R));
  CHK(wsT(c, "f_W", (size_t)d * d, &W));
  CHK(wsT(c, "f_WT", (size_t)d * d, &WT));
  CHK(wsT(c, "ihs_xprev", d, &xprev));
  CHK(wsT(c, "ihs_diff", d, &diff));
  CHK(wsT(c, "ihs_err", 1, &errv));
  SolveBufs b;
  CHK(solve_bufs(c, p->n, d, &b));
  double ax2 = 0.0;
  auto error_at = [&](int t) -> lsq_status {
    // err_trace[t] = ||A (x - x_ref)|| / ||A x_ref||
    vec_copy(st, diff, x, d);
    vec_axpy(st, diff, o->x_ref, -1.0, d);
    const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 0, diff, nullptr, b.part, b.nwg, nullptr);
    reduce_partials(st, b.part, b.part2, ng_, d, b.red, nullptr);
    error_from_resid(st, b.red + d, ax2, err_trace + t);
    HIPCHK(hipGetLastError());
    return LSQ_OK;
  };
  if (err_trace) {
    const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 0, o->x_ref, nullptr, b.part, b.nwg, nullptr);
    reduce_partials(st, b.part, b.part2, ng_, d, b.red, nullptr);
    HIPCHK(hipMemcpyAsync(c->hflags, b.red + d, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    memcpy(&ax2, c->hflags, sizeof(double));
    CHK(error_at(0));
  }
  double t_sketch = 0.0, t_factor = 0.0, t_iter = 0.0;
  HIPCHK(hipEventRecord(c->ev[4], st));
  vec_copy(st, xprev, x, d);
  for (int t = 0; t < o->iters; ++t) {
    if (t == 0 || o->refresh) {
      float ms;
      HIPCHK(hipEventRecord(c->ev[0], st));
      CHK(do_sketch(c, p, s, s->t + (o->refresh ? (uint64_t)t : 0), SA, d));
      HIPCHK(hipEventRecord(c->ev[1], st));
      CHK(do_factor(c, SA, m, d, d, R, W, WT));
      HIPCHK(hipEventRecord(c->ev[2], st));
      HIPCHK(hipEventSynchronize(c->ev[2]));
      hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
      t_sketch += ms;
      hipEventElapsedTime(&ms, c->ev[1], c->ev[2]);
      t_factor += ms;
    }
    HIPCHK(hipEventRecord(c->ev[0], st));
    const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 1, x, p->y, b.part, b.nwg, nullptr);
    reduce_partials(st, b.part, b.part2, ng_, d, b.r, nullptr);
    int ndot;
    precond_apply_any(st, W, WT, d, b.r, b.u, b.rhat, b.dotpart, &ndot, nullptr, c->w_dense);
    ihs_update(st, d, x, xprev, b.rhat, mu, beta);
    HIPCHK(hipEventRecord(c->ev[1], st));
    HIPCHK(hipEventSynchronize(c->ev[1]));
    float ms;
    hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    t_iter += ms;
    if (err_trace) CHK(error_at(t + 1));
  }
  HIPCHK(hipEventRecord(c->ev[5], st));
  HIPCHK(hipStreamSynchronize(st));
  if (info) {
    float ms;
    info->iters = o->iters;
    info->refinements = 0;
    info->est_rel_err = 0.0;
    if (err_trace && o->iters >= 0) {
      double e;
      hipMemcpy(&e, err_trace + o->iters, sizeof(double), hipMemcpyDeviceToHost);
      info->est_rel_err = e;
    }
    info->t_sketch_ms = t_sketch;
    info->t_factor_ms = t_factor;
    info->t_iter_ms = t_iter;
    hipEventElapsedTime(&ms, c->ev[4], c->ev[5]);
    info->t_total_ms = ms;
    info->bytes_streamed = (double)o->iters * p->n * d * (a_f32 ? 4.0 : 8.0);
    info->mu = mu;
    info->status = LSQ_OK;
    info->pad_ = 0;
    info->t_start_ms = 0.0;
  }
  return LSQ_OK;
}

lsq_status lsq_fcg_solve(lsq_ctx* c, const lsq_problem* p, const lsq_sketch_desc* s,
                         const lsq_fcg_opts* o, double* x, double* err_trace, lsq_info* info) {
  CHK(check_problem(c, p));
  CHK(check_sketch(c, p, s, true));
  if (!o || !x) return fail(LSQ_ERR_INVALID_ARG, "null options or x");
  if (o->iters < 0) return fail(LSQ_ERR_INVALID_ARG, "iters < 0");
  if (o->window < 0) return fail(LSQ_ERR_INVALID_ARG, "window < 0");
  if (err_trace && !o->x_ref) return fail(LSQ_ERR_INVALID_ARG, "err_trace needs x_ref");
  const int ring = std::max(1, std::min(o->window, o->iters));
  if (ring > FCG_MAX_WINDOW) return fail(LSQ_ERR_UNSUPPORTED, "min(window, iters) > 1024");
  const int64_t d = p->d, m = s->m;
  const hipStream_t st = c->st;
  const int a_f32 = p->a_dtype == LSQ_F32;
  double *SA, *R, *W, *WT, *diff, *P, *HP, *php;
  CHK(wsT(c, "SA", (size_t)m * d, &SA));
  CHK(wsT(c, "f_R", (size_t)d * d, &R));
  CHK(wsT(c, "f_W", (size_t)d * d, &W));
  CHK(wsT(c, "f_WT", (size_t)d * d, &WT));
  CHK(wsT(c, "ihs_diff", d, &diff));
  CHK(wsT(c, "fcg_P", (size_t)ring * d, &P));
  CHK(wsT(c, "fcg_HP", (size_t)ring * d, &HP));
  CHK(wsT(c, "fcg_php", ring, &php));
  SolveBufs b;
  CHK(solve_bufs(c, p->n, d, &b));
  double ax2 = 0.0;
  auto error_at = [&](int t) -> lsq_status {
    // err_trace[t] = ||A (x - x_ref)|| / ||A x_ref||
    vec_copy(st, diff, x, d);
    vec_axpy(st, diff, o->x_ref, -1.0, d);
    const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 0, diff, nullptr, b.part, b.nwg, nullptr);
    reduce_partials(st, b.part, b.part2, ng_, d, b.red, nullptr);
    error_from_resid(st, b.red + d, ax2, err_trace + t);
    HIPCHK(hipGetLastError());
    return LSQ_OK;
  };
  if (err_trace) {
    const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 0, o->x_ref, nullptr, b.part, b.nwg, nullptr);
    reduce_partials(st, b.part, b.part2, ng_, d, b.red, nullptr);
    HIPCHK(hipMemcpyAsync(c->hflags, b.red + d, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    memcpy(&ax2, c->hflags, sizeof(double));
    CHK(error_at(0));
  }
  double t_sketch = 0.0, t_factor = 0.0, t_iter = 0.0;
  HIPCHK(hipEventRecord(c->ev[4], st));
  {
    // r_0 = A^T (y - A x_0)
    const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 1, x, p->y, b.part, b.nwg, nullptr);
    reduce_partials(st, b.part, b.part2, ng_, d, b.red, nullptr);
    vec_copy(st, b.r, b.red, d);
  }
  for (int t = 0; t < o->iters; ++t) {
    if (t == 0 || o->refresh) {
      float ms;
      HIPCHK(hipEventRecord(c->ev[0], st));
      CHK(do_sketch(c, p, s, s->t + (o->refresh ? (uint64_t)t : 0), SA, d));
      HIPCHK(hipEventRecord(c->ev[1], st));
      CHK(do_factor(c, SA, m, d, d, R, W, WT));
      HIPCHK(hipEventRecord(c->ev[2], st));
      HIPCHK(hipEventSynchronize(c->ev[2]));
      hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
      t_sketch += ms;
      hipEventElapsedTime(&ms, c->ev[1], c->ev[2]);
      t_factor += ms;
    }
    HIPCHK(hipEventRecord(c->ev[0], st));
    int ndot;
    precond_apply_any(st, W, WT, d, b.r, b.u, b.rhat, b.dotpart, &ndot, nullptr, c->w_dense);  // v_t
    const int kt = std::min(o->window, t);
    const int slot = t % ring;
    double* pt = P + (size_t)slot * d;
    fcg_orth(st, b.rhat, P, HP, php, d, t, kt, ring);
    const int ng_ = fused_pass(st, p->A, a_f32, 0, p->n, d, p->lda, 0, pt, nullptr, b.part, b.nwg, nullptr);
    reduce_partials(st, b.part, b.part2, ng_, d, b.red, nullptr);
    fcg_step(st, pt, b.red, d, x, b.r, HP + (size_t)slot * d, php + slot);
    HIPCHK(hipEventRecord(c->ev[1], st));
    HIPCHK(hipEventSynchronize(c->ev[1]));
    float ms;
    hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
    t_iter += ms;
    if (err_trace) CHK(error_at(t + 1));
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(c->ev[5], st));
  HIPCHK(hipStreamSynchronize(st));
  if (info) {
    float ms;
    info->iters = o->iters;
    info->refinements = 0;
    info->est_rel_err = 0.0;
    if (err_trace) {
      double e;
      hipMemcpy(&e, err_trace + o->iters, sizeof(double), hipMemcpyDeviceToHost);
      info->est_rel_err = e;
    }
    info->t_sketch_ms = t_sketch;
    info->t_factor_ms = t_factor;
    info->t_iter_ms = t_iter;
    hipEventElapsedTime(&ms, c->ev[4], c->ev[5]);
    info->t_total_ms = ms;
    info->bytes_streamed = (double)(o->iters + 1) * p->n * d * (a_f32 ? 4.0 : 8.0);
    info->mu = 0.0;
    info->status = LSQ_OK;
    info->pad_ = 0;
    info->t_start_ms = 0.0;
  }
  return LSQ_OK;
}

lsq_status lsq_draw_srht(lsq_ctx* c, uint64_t seed, uint64_t t, int64_t N, int64_t m, int8_t* signs,
                         int64_t* rows) {
  if (!c) return fail(LSQ_ERR_INVALID_ARG, "null context");
  if (N < 1 || (N & (N - 1))) return fail(LSQ_ERR_INVALID_ARG, "N must be a power of two");
  if (m < 1 || m > N) return fail(LSQ_ERR_INVALID_ARG, "need 1 <= m <= N");
  uint64_t* keys;
  int *hist, *bcount;
  void* state;
  CHK(wsT(c, "srht_keys", N, &keys));
  CHK(wsT(c, "sel_hist", 65536, &hist));
  CHK(wsT(c, "sel_bcount", srht_select_bcount_len(N), &bcount));
  CHK(ws(c, "sel_state", 64, &state));
  launch_srht_draw(c->st, seed, t, N, signs, keys);
  if (rows) srht_select(c->st, keys, N, m, rows, SelectScratch{hist, bcount, state});
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return LSQ_OK;
}

lsq_status lsq_draw_sjlt(lsq_ctx* c, uint64_t seed, uint64_t t, int64_t n, int64_t m, int32_t s,
                         int32_t* targets, int8_t* signs) {
  if (!c || !targets || !signs) return fail(LSQ_ERR_INVALID_ARG, "null argument");
  if (n < 1 || m < 1 || s < 1 || s > m || s > MAX_SJLT_S)
    return fail(LSQ_ERR_INVALID_ARG, "need n, m >= 1 and 1 <= s <= min(m, 32)");
  HIPCHK(hipMemsetAsync(c->dflags + 1, 0, sizeof(int), c->st));
  launch_sjlt_draw(c->st, seed, t, n, m, s, targets, signs, c->dflags + 1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->hflags + 1, c->dflags + 1, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (c->hflags[1]) return fail(LSQ_ERR_INVALID_ARG, "SJLT draw limit exhausted");
  return LSQ_OK;
}

lsq_status lsq_draw_gaussian(lsq_ctx* c, uint64_t seed, uint64_t t, int64_t m, int64_t j0,
                             int64_t ncols, double* G) {
  if (!c || !G) return fail(LSQ_ERR_INVALID_ARG, "null argument");
  if (m < 1 || ncols < 1 || j0 < 0) return fail(LSQ_ERR_INVALID_ARG, "bad sizes");
  launch_gauss_draw(c->st, seed, t, m, j0, ncols, G);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->st));
  return LSQ_OK;
}

lsq_status lsq_tune(const char* key, int64_t value) {
  if (!key) return fail(LSQ_ERR_INVALID_ARG, "null key");
  const std::string k(key);
  if (k == "fused_groups_per_cu") {
    if (value < 1 || value > 64) return fail(LSQ_ERR_INVALID_ARG, "fused_groups_per_cu in [1, 64]");
    g_fused_groups_per_cu = (int)value;
    return LSQ_OK;
  }
  if (k == "batched_slots") {
    if (value < 0 || value > 65536) return fail(LSQ_ERR_INVALID_ARG, "batched_slots in [0, 65536]");
    g_batched_slots = (int)value;
    return LSQ_OK;
  }
  if (k == "batched_gang_unit") {
    if (value < 0 || (value > 0 && value < 65536))
      return fail(LSQ_ERR_INVALID_ARG, "batched_gang_unit: 0 (no gangs) or at least 65536 elements");
    g_batched_gang_unit = value;
    return LSQ_OK;
  }
  struct Knob {
    const char* key;
    int* var;
    int64_t lo, hi;
  };
  const Knob knobs[] = {{"srht_fold8_rows_f32", &g_srht_fold8_rows_f32, 1, 1 << 20},
                        {"srht_fold8_rows_f64", &g_srht_fold8_rows_f64, 1, 1 << 20},
                        {"srht_stream_rows_f32", &g_srht_stream_rows_f32, 1, 1 << 20},
                        {"srht_stream_rows_f64", &g_srht_stream_rows_f64, 1, 1 << 20},
                        {"srht_passa_wgs", &g_srht_passa_wgs, 0, 1 << 22},
                        {"srht_passb_wgs", &g_srht_passb_wgs, 256, 1 << 20},
                        {"gauss_wgs", &g_gauss_wgs, 64, 1 << 16},
                        {"gauss_planes_min_d", &g_gauss_planes_min_d, 1, 1 << 30},
                        {"gauss_planes_wgs", &g_gauss_planes_wgs, 8, 1 << 16},
                        {"gauss_chunk_rows", &g_gauss_chunk_rows, 0, 1 << 30},
                        {"gram_wgs", &g_gram_wgs, 64, 1 << 16}};
  for (const Knob& kn : knobs)
    if (k == kn.key) {
      if (value < kn.lo || value > kn.hi)
        return fail(LSQ_ERR_INVALID_ARG, k + " in [" + std::to_string(kn.lo) + ", " + std::to_string(kn.hi) + "]");
      *kn.var = (int)value;
      return LSQ_OK;
    }
  return fail(LSQ_ERR_INVALID_ARG, "unknown tuning key: " + k);
}

lsq_status lsq_set_option(lsq_ctx* c, const char* key, int64_t value) {
  if (!c || !key) return fail(LSQ_ERR_INVALID_ARG, "null context or key");
  const std::string k(key);
  if (k == "factor") {
    if (value < 0 || value > 5)
      return fail(LSQ_ERR_INVALID_ARG,
                  "factor: 0 (CholeskyQR, second pass when needed), 1 (Householder), 2 (SVD), 3 (column-pivoted "
                  "QR), 4 (CholeskyQR2) or 5 (one-pass CholeskyQR)");
    c->factor_mode = (int)value;
    return LSQ_OK;
  }
  if (k == "srht_passb") {
    if (value < 0 || value > 6)
      return fail(LSQ_ERR_INVALID_ARG,
                  "srht_passb: 0 (form and fold width by bucket size, the default), 1 (register-direct), 2 "
                  "(register-staged, 8 wavefronts), 3 (16 wavefronts, 4-point fold), 4 (16 wavefronts, 8-point "
                  "fold), 5 (streamed into LDS, 8-point fold) or 6 (streamed, 16-point fold)");
    c->srht_passb = (int)value;
    return LSQ_OK;
  }
  if (k == "sketch_upgrade") {
    if (value < 0 || value > 1) return fail(LSQ_ERR_INVALID_ARG, "sketch_upgrade: 0 or 1");
    c->sketch_upgrade = (int)value;
    return LSQ_OK;
  }
  return fail(LSQ_ERR_INVALID_ARG, "unknown option: " + k);
}

lsq_status lsq_pcg_solve_batched(lsq_ctx* c, int32_t count, const lsq_problem* probs,
                                 const lsq_sketch_desc* descs, const lsq_pcg_opts* o,
                                 double* const* xs, double* const* Rs, lsq_info* infos) {
  if (!c || !probs || !descs || !o || !xs)
    return fail(LSQ_ERR_INVALID_ARG, "null context, problems, descriptors, options or xs");
  if (count < 1) return fail(LSQ_ERR_INVALID_ARG, "count < 1");
  if (o->max_iter < 1) return fail(LSQ_ERR_INVALID_ARG, "max_iter < 1");
  if (!(o->tol > 0.0)) return fail(LSQ_ERR_INVALID_ARG, "tol must be > 0");
  if (o->mixed && o->max_refine < 1) return fail(LSQ_ERR_INVALID_ARG, "max_refine < 1");
  if (o->stop_rule != 0 || o->inner_f32 || o->x_ref)
    return fail(LSQ_ERR_UNSUPPORTED, "batched form: stop_rule 0 only, no inner_f32, no x_ref");
  // validation and the queue order (largest n d first)
  std::vector<int> order(count);
  int64_t kmax = 1, mpmax = 16, dpmax = 16;
  for (int i = 0; i < count; ++i) {
    const lsq_problem& p = probs[i];
    const lsq_sketch_desc& s = descs[i];
    const std::string at = "problem " + std::to_string(i) + ": ";
    lsq_status st = check_problem(c, &p);
    if (st != LSQ_OK) return fail(st, at + g_err);
    if (!xs[i]) return fail(LSQ_ERR_INVALID_ARG, at + "null x");
    if (s.kind != LSQ_SJLT) return fail(LSQ_ERR_UNSUPPORTED, at + "the batched form uses the SJLT");
    if (p.d > 256) return fail(LSQ_ERR_UNSUPPORTED, at + "batched form limited to d <= 256");
    if (p.n < p.d || p.n > (int64_t(1) << 22))
      return fail(LSQ_ERR_UNSUPPORTED, at + "batched form needs d <= n <= 2^22");
    if (s.m < p.d || s.m > 1024) return fail(LSQ_ERR_UNSUPPORTED, at + "batched form needs d <= m <= 1024");
    if (s.s < 1 || s.s > 32 || s.s > s.m) return fail(LSQ_ERR_INVALID_ARG, at + "need 1 <= s <= min(m, 32)");
    order[i] = i;
    kmax = std::max(kmax, (int64_t)s.s * p.n);
    mpmax = std::max(mpmax, (s.m + 15) / 16 * 16);
    dpmax = std::max(dpmax, (p.d + 15) / 16 * 16);
  }
  int cus = 0;
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->dev));
  // gang size of each problem: one workgroup per g_batched_gang_unit elements of n d (rounded), at most
  // BATCH_GANG_KMAX; a function of the problem alone, so that the result does not depend on the number
  // of workgroups (as long as there are at least BATCH_GANG_KMAX of them)
  auto gang_size = [&](int i) -> int {
    if (g_batched_gang_unit <= 0) return 1;
    const double nd = (double)probs[i].n * (double)probs[i].d;
    const int k = (int)std::llround(nd / (double)g_batched_gang_unit);
    return std::max(1, std::min(BATCH_GANG_KMAX, k));
  };
  std::vector<int> gsize(count);
  int64_t ntasks = 0;
  for (int i = 0; i < count; ++i) {
    gsize[i] = gang_size(i);
    ntasks += gsize[i];
  }
  // queue order: largest work per member first (longest processing time first)
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return probs[a].n * probs[a].d / gsize[a] > probs[b].n * probs[b].d / gsize[b];
  });
  const int slots = (int)std::min<int64_t>(ntasks, g_batched_slots > 0 ? g_batched_slots : std::max(cus, 1));
  for (int i = 0; i < count; ++i)
    if (gsize[i] > slots) return fail(LSQ_ERR_UNSUPPORTED, "batched form: fewer workgroups than a gang needs");
  // workspace (per slot) and the problem table
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  a.count = count;
  a.mixed = o->mixed ? 1 : 0;
  a.max_iter = o->max_iter;
  a.max_refine = o->mixed ? o->max_refine : 1;
  a.tol = o->tol;
  a.keys_stride = kmax;
  a.sa_stride = mpmax * dpmax;
  a.v_stride = mpmax * 16;
  a.r_stride = dpmax * dpmax;
  a.last_stride = 256;
  BatchDesc* dtab;
  CHK(wsT(c, "b_desc", (size_t)count, &dtab));
  BatchTask* ttab;
  CHK(wsT(c, "b_tasks", (size_t)ntasks, &ttab));
  a.ntasks = (int)ntasks;
  std::vector<BatchTask> tasks;
  tasks.reserve(ntasks);
  int ngangs = 0;
  for (int q = 0; q < count; ++q) {
    const int K = gsize[order[q]];
    const int gid = K > 1 ? ngangs++ : -1;
    for (int r = 0; r < K; ++r) tasks.push_back(BatchTask{q, r, K, gid});
  }
  a.ngangs = ngangs;
  a.gpart_stride = dpmax + 1;
  CHK(wsT(c, "b_gstate", (size_t)std::max(ngangs, 1) * 4, &a.gstate));
  CHK(wsT(c, "b_gpart", (size_t)std::max(ngangs, 1) * 2 * BATCH_GANG_KMAX * a.gpart_stride, &a.gpart));
  a.tasks = ttab;
  CHK(wsT(c, "b_out", (size_t)count, &a.out));
  CHK(wsT(c, "b_queue", 1, &a.queue));
  CHK(wsT(c, "b_keys", (size_t)slots * kmax, &a.keys));
  CHK(wsT(c, "b_sorted", (size_t)slots * kmax, &a.sorted));
  CHK(wsT(c, "b_SA", (size_t)slots * a.sa_stride, &a.SA));
  CHK(wsT(c, "b_V", (size_t)slots * a.v_stride, &a.V));
  CHK(wsT(c, "b_R", (size_t)slots * a.r_stride, &a.R));
  CHK(wsT(c, "b_W", (size_t)slots * a.r_stride, &a.W));
  CHK(wsT(c, "b_WT", (size_t)slots * a.r_stride, &a.WT));
  CHK(wsT(c, "b_last", (size_t)slots * a.last_stride, &a.last));
  a.descs = dtab;
  std::vector<BatchDesc> table(count);
  for (int q = 0; q < count; ++q) {
    const int i = order[q];
    const lsq_problem& p = probs[i];
    const lsq_sketch_desc& s = descs[i];
    BatchDesc& t = table[q];
    memset(&t, 0, sizeof(t));
    t.A = p.A;
    t.y = (const double*)p.y;
    t.x = xs[i];
    t.R = Rs ? Rs[i] : nullptr;
    t.n = p.n;
    t.lda = p.lda;
    t.d = (int32_t)p.d;
    t.m = (int32_t)s.m;
    t.s = s.s;
    t.a_f32 = p.a_dtype == LSQ_F32;
    t.seed = s.seed;
    t.t = s.t;
    t.idx = i;
  }
  if (!c->bst) {
    HIPCHK(hipStreamCreateWithFlags(&c->bst, hipStreamNonBlocking));
    for (int i = 0; i < 3; ++i) HIPCHK(hipEventCreate(&c->bev[i]));
  }
  const size_t out_bytes = sizeof(BatchOut) * (size_t)count;
  if (c->bhost_bytes < out_bytes) {
    if (c->bhost) HIPCHK(hipHostFree(c->bhost));
    c->bhost = nullptr;
    c->bhost_bytes = 0;
    HIPCHK(hipHostMalloc(&c->bhost, out_bytes, hipHostMallocDefault));
    c->bhost_bytes = out_bytes;
  }
  // the graph depends only on the launch arguments: capture again when they change
  std::vector<unsigned char> key(sizeof(a) + sizeof(int));
  memcpy(key.data(), &a, sizeof(a));
  memcpy(key.data() + sizeof(a), &slots, sizeof(int));
  if (!c->bexec || key != c->bkey) {
    if (c->bexec) HIPCHK(hipGraphExecDestroy(c->bexec));
    if (c->bgraph) HIPCHK(hipGraphDestroy(c->bgraph));
    c->bexec = nullptr;
    c->bgraph = nullptr;
    HIPCHK(hipStreamBeginCapture(c->bst, hipStreamCaptureModeThreadLocal));
    batched_launch(c->bst, a, slots);
    const hipError_t le = hipGetLastError();
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(c->bst, &g);
    if (le != hipSuccess || ce != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(LSQ_ERR_HIP, std::string("graph capture failed: ") +
                                   hipGetErrorString(le != hipSuccess ? le : ce));
    }
    c->bgraph = g;
    HIPCHK(hipGraphInstantiate(&c->bexec, g, nullptr, nullptr, 0));
    c->bkey = key;
  }
  // order after the caller's stream, upload the table, run, copy the results back
  HIPCHK(hipEventRecord(c->bev[0], c->st));
  HIPCHK(hipStreamWaitEvent(c->bst, c->bev[0], 0));
  HIPCHK(hipMemcpyAsync(dtab, table.data(), sizeof(BatchDesc) * count, hipMemcpyHostToDevice, c->bst));
  HIPCHK(hipMemcpyAsync(ttab, tasks.data(), sizeof(BatchTask) * tasks.size(), hipMemcpyHostToDevice, c->bst));
  HIPCHK(hipEventRecord(c->bev[1], c->bst));
  HIPCHK(hipGraphLaunch(c->bexec, c->bst));
  HIPCHK(hipEventRecord(c->bev[2], c->bst));
  HIPCHK(hipMemcpyAsync(c->bhost, a.out, out_bytes, hipMemcpyDeviceToHost, c->bst));
  HIPCHK(hipStreamSynchronize(c->bst));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, c->bev[1], c->bev[2]));
  int clk_khz = 0;
  HIPCHK(hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, c->dev));
  const double tick_ms = clk_khz > 0 ? 1.0 / clk_khz : 0.0;
  const BatchOut* res = (const BatchOut*)c->bhost;
  uint64_t t0_min = ~0ull;
  for (int i = 0; i < count; ++i) t0_min = std::min(t0_min, res[i].t_start);
  lsq_status ret = LSQ_OK;
  int first_bad = -1;
  for (int i = 0; i < count; ++i) {
    const int st = res[i].status;
    if (infos) {
      lsq_info& f = infos[i];
      memset(&f, 0, sizeof(f));
      f.iters = res[i].iters;
      f.refinements = res[i].refinements;
      f.est_rel_err = res[i].est;
      f.t_sketch_ms = (double)(res[i].t_sketch - res[i].t_start) * tick_ms;
      f.t_factor_ms = (double)(res[i].t_factor - res[i].t_sketch) * tick_ms;
      f.t_iter_ms = (double)(res[i].t_end - res[i].t_factor) * tick_ms;
      f.t_total_ms = ms;
      f.t_start_ms = (double)(res[i].t_start - t0_min) * tick_ms;
      f.bytes_streamed = (double)(res[i].iters + res[i].refinements + 1) * (double)probs[i].n *
                         (double)probs[i].d * (probs[i].a_dtype == LSQ_F32 ? 4.0 : 8.0);
      f.status = st < 0 ? LSQ_ERR_HIP : st;
    }
    if (st != LSQ_OK && first_bad < 0) {
      first_bad = i;
      ret = st < 0 ? LSQ_ERR_HIP : (lsq_status)st;
    }
  }
  if (ret != LSQ_OK)
    return fail(ret, "problem " + std::to_string(first_bad) + ": " + lsq_status_string(ret));
  return LSQ_OK;
}

}  // extern "C"
