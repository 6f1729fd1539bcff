/*
 * liblsq — sketch-preconditioned least squares for tall matrices on AMD Instinct MI355X (gfx950).
 *
 * Method: Lacotte & Pilanci, "Faster Least Squares Optimization" (arXiv 1911.02675).
 *   Problem (Section 1):  x* = argmin_x 1/2 <x, H x> - <b, x>,  H = A^T A, A in R^{n x d}, n >= d.
 *   For least squares the caller passes y in R^n and b = A^T y, i.e. x* = argmin ||A x - y||_2.
 *   Embeddings (Section 2): Gaussian (entries N(0, 1/m)), SRHT (S = R H E with zero padding to a power
 *   of two), SJLT (s nonzeros +-1/sqrt(s) per column), Haar (orthonormal rows, S S^T = I_m, spanning a
 *   uniformly distributed subspace: S = Q^T for the positive-diagonal QR g^T = Q R of the Gaussian
 *   embedding's unscaled draws g, formed as R^{-T} (g A) without Q).
 *   Preconditioner (Section 1.2): H_S = (S A)^T (S A) = R^T R, R from a QR of S A.
 *   Solvers: PCG with a fixed sketch (Section 1.2), IHS and Polyak-IHS (Section 1.1) with a fixed or a
 *   refreshed sketch (Sections 3 and 4).
 *
 * Conventions for every entry point:
 *   - Matrices are ROW-MAJOR.  A has n rows of d entries at stride lda >= d (elements).
 *   - Pointers are DEVICE pointers unless marked (host).  The caller owns every buffer; the library
 *     never frees caller memory.  Internal workspace lives in the context, is allocated on first need
 *     (hipMalloc) and reused; it grows when a larger problem arrives.
 *   - Calls are synchronous with respect to the host: they return after the work queued on the
 *     context's stream has completed.  Calls on one context must not overlap.
 *   - No exception crosses the ABI.  On a non-OK status lsq_last_error() returns a thread-local message.
 *   - Argument errors leave every output untouched.  LSQ_ERR_NOT_CONVERGED returns the last iterate.
 *   - Random draws are pure functions of (seed, t, index) through Philox4x64-10 (Salmon et al., SC'11)
 *     with key (seed, 0).  The draw specification (bit-exact for signs, row subsets and SJLT targets):
 *       SRHT : row j of the zero-padded A (j < N = 2^ceil(log2 n)) uses block (j, 1, t, 0) -> w0..w3;
 *              sign e_j = -1 iff bit 63 of w0; R keeps the m rows with the smallest (w1, j), in
 *              increasing j.  S = m^{-1/2} R H_N E with the +-1 Sylvester Hadamard H_N.
 *       SJLT : row j of A reads words w0..w3 of blocks (j, 2, t, 0), (j, 2, t, 1), ...; each word w
 *              proposes h = ((w >> 32) * m) >> 32, rejected when ((w >> 32) * m) mod 2^32 < 2^32 mod m
 *              (exact uniformity) or when h is already taken; the sign is -1 iff bit 0 of w.  s distinct
 *              targets per row; entries +-1/sqrt(s).
 *       GAUSS: S_ij (i < m, j < n) = g / sqrt(m), g from block (j >> 3, 3, t, i), word p = (j & 7) >> 1,
 *              a = low 32 bits, b = high 32 bits, u1 = (a + 1) 2^-32, u2 = b 2^-32,
 *              g = sqrt(-2 ln u1) cos(2 pi u2) for even j, sin(...) for odd j (Box-Muller; the GPU
 *              evaluates it in FP64 with 2 pi u2 rounded once, as the oracle does, for the FP64 sketch,
 *              and in single precision with the hardware transcendentals for the BF16 form, whose
 *              entries are rounded to BF16).
 */
#ifndef LSQ_H
#define LSQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LSQ_OK = 0,
  LSQ_ERR_INVALID_ARG = 1,   /* bad size, null pointer, unsupported combination of arguments        */
  LSQ_ERR_RANK = 2,          /* zero pivot in R (S A rank deficient) or breakdown p^T H p <= 0       */
  LSQ_ERR_NOT_CONVERGED = 3, /* iteration budget spent before the stop rule held; x = last iterate  */
  LSQ_ERR_NONFINITE = 4,     /* NaN or Inf met in a reduction                                       */
  LSQ_ERR_HIP = 5,           /* a HIP runtime call failed                                           */
  LSQ_ERR_NOMEM = 6,         /* workspace allocation failed                                         */
  LSQ_ERR_UNSUPPORTED = 7    /* valid request outside the implemented range (e.g. d > 1024)         */
} lsq_status;

typedef enum { LSQ_F64 = 0, LSQ_F32 = 1, LSQ_BF16 = 2 } lsq_dtype;
typedef enum { LSQ_GAUSSIAN = 0, LSQ_SRHT = 1, LSQ_SJLT = 2, LSQ_HAAR = 3 } lsq_sketch_kind;

typedef struct lsq_ctx lsq_ctx; /* opaque: stream, workspace, device state, tuning table */

/* A context bound to the current HIP device and to `stream` (a hipStream_t; NULL = default stream).
 * ctx (host) receives the handle. */
lsq_status lsq_create(lsq_ctx** ctx, void* stream);
void lsq_destroy(lsq_ctx* ctx);

/* The least-squares problem min ||A x - y||.  a_dtype is LSQ_F64 or LSQ_F32 (A stored in FP32 and
 * promoted exactly; this is the "precision form" storage).  y is FP64, length n. */
typedef struct {
  int64_t n, d, lda;
  int32_t a_dtype;
  int32_t pad_;
  const void* A;
  const double* y;
} lsq_problem;

/* The embedding S (m x n).  s: nonzeros per column for the SJLT (1 <= s <= min(m, 32)).
 * compute: arithmetic of the sketch: LSQ_F64, LSQ_F32 (SRHT transform in single precision), or
 * LSQ_BF16 (Gaussian only: bf16 S times a three-term bf16 split of A on matrix cores, FP32
 * accumulation).  t: refresh counter (independent draws for every t). */
typedef struct {
  int32_t kind;
  int32_t s;
  int64_t m;
  int32_t compute;
  int32_t pad_;
  uint64_t seed;
  uint64_t t;
} lsq_sketch_desc;

/* PCG options.
 *   tol:        target relative A-norm error ||A (x - x*)|| / ||A x*||.  The stop rule uses
 *               rho_t = r_t^T H_S^{-1} r_t = Delta_t^T C_S^{-1} Delta_t: it stops when
 *               4 sqrt(rho_t / rho_0) <= tol, which implies the target whenever the eigenvalues of
 *               C_S = U^T S^T S U span a ratio of at most 16 (the subspace-embedding event of Section 3).
 *               With stop_rule = 0 the result is verified: PCG runs until its recursively updated
 *               residual meets the rule, then the residual A^T (y - A x) is measured in double-double
 *               arithmetic (rounded once) and the rule is applied to the measured value.  When the
 *               measured residual falls short (the recursive one drifts from the true one by about
 *               u kappa(A) relative to its start, which matters near the FP64 conditioning floor), PCG
 *               solves for the correction from the measured residual and x += dx (residual
 *               replacement), up to max_refine correction solves in all; LSQ_ERR_NOT_CONVERGED when the
 *               budget ends, or when a measured residual is not half the previous one.  After a
 *               correction solved from a measured residual the new estimate is the measured one times
 *               that solve's own relative reduction (the rounding in that solve is relative to the
 *               correction), so the call ends without a further residual once that meets tol (not with
 *               x_ref).  From x = 0 the first residual is A^T y in FP64 arithmetic (no cancellation).
 *   max_iter:   PCG iteration budget of each correction solve.
 *   stop_rule:  0 = the rule above; 1 = exactly max_iter iterations (plain form: one solve, no
 *               measurement; mixed form: one correction solve after the first residual).
 *   mixed:      0 = plain form: A as given (FP64 or FP32 storage), FP64 arithmetic; the first correction
 *                   accumulates into x itself;
 *               1 = precision form: as above with every correction solved in a separate vector (x += dx
 *                   in FP64) and, with inner_f32, FP32-arithmetic inner products.
 *   max_refine: budget of correction solves (both forms; the plain form takes values below 1 as 1).
 *   inner_f32:  mixed = 1 only: 1 = inner matrix-vector products in FP32 arithmetic (p rounded to
 *               FP32); 0 = FP32 storage read into FP64 registers.
 *   x_ref:      optional device pointer to the exact minimiser; when given, err_trace holds the exact
 *               relative A-norm error per iteration of the first correction solve (computed as
 *               sqrt(-(x_t - x*)^T r_t / x*^T b)), otherwise the stop-rule estimate 4 sqrt(rho_t / rho_0),
 *               and info->est_rel_err is the exact error at the last measured residual. */
typedef struct {
  double tol;
  int32_t max_iter;
  int32_t stop_rule;
  int32_t mixed;
  int32_t max_refine;
  int32_t inner_f32;
  int32_t check_every; /* iterations queued between host checks of the device stop flag (0 = 8) */
  const double* x_ref;
} lsq_pcg_opts;

/* IHS / Polyak-IHS options (x_{t+1} = x_t - mu H_{S_t}^{-1} grad f(x_t) + beta (x_t - x_{t-1}),
 * x_{-1} = x_0).
 *   refresh: 1 = S_t drawn with refresh counter desc.t + t (Section 4); 0 = S_t = S fixed (Section 3).
 *   mu_rule: 0 = mu = theta_1 / theta_2 from the inverse moments (Theorem 4.1): the Gaussian closed
 *            form for LSQ_GAUSSIAN (needs m >= d + 4), the Haar/SRHT trace approximation for LSQ_SRHT
 *            rescaled to S S^T = (N/m) I, i.e. mu = (N/m) theta_1/theta_2; for LSQ_HAAR the same trace
 *            approximation with n, unscaled (S S^T = I); LSQ_SJLT has no closed form and needs
 *            mu_rule = 1.  1 = use `mu` as given.  2 and 3 are the fixed-sketch parameters of
 *            Theorem 3.2 with rho = d/m (meant for refresh = 0; need m > d): 2 = IHS step
 *            mu = (1 - rho)^2 / (1 + rho) (the optimal step of Theorem 3.4) with `beta` as given;
 *            3 = Polyak-IHS mu = (1 - rho)^2, beta = rho (the given `beta` is ignored).
 *   x_ref:   optional; when given err_trace[t] = ||A (x_t - x_ref)|| / ||A x_ref|| for t = 0..iters
 *            (one extra pass over A per iteration; use it for studies, not for timing). */
typedef struct {
  double mu;
  double beta;
  int32_t iters;
  int32_t refresh;
  int32_t mu_rule;
  int32_t pad_;
  const double* x_ref;
} lsq_ihs_opts;

/* Flexible conjugate gradient options (Section 1.2, analysed with refreshed sketches in Section 4):
 * with r_t = A^T (y - A x_t) and H_{S_t} = R_t^T R_t,
 *   v_t = H_{S_t}^{-1} r_t,   p_t = v_t - sum_{j=t-k_t}^{t-1} (<v_t, H p_j> / <p_j, H p_j>) p_j,
 *   x_{t+1} = x_t + (<p_t, r_t> / <p_t, H p_t>) p_t       (exact line search along p_t)
 * with k_t = min(window, t).
 *   window:  conjugation window k >= 0: 0 = IHS direction with an exact line search, 1 = IPCG,
 *            >= iters = GCC (every earlier direction).  min(window, iters) <= 1024.
 *   refresh: 1 = S_t drawn with refresh counter desc.t + t; 0 = S_t = S fixed (then every window
 *            k >= 1 reproduces PCG).
 *   x_ref:   optional; when given err_trace[t] = ||A (x_t - x_ref)|| / ||A x_ref|| for t = 0..iters. */
typedef struct {
  int32_t iters;
  int32_t window;
  int32_t refresh;
  int32_t pad_;
  const double* x_ref;
} lsq_fcg_opts;

/* Per-call report (host).  Times are HIP-event times on the context stream. */
typedef struct {
  int32_t iters;       /* PCG iterations (summed over correction solves), IHS or FCG iterations */
  int32_t refinements; /* correction solves (lsq_pcg_solve, stop_rule 0 or mixed)          */
  double est_rel_err;  /* final stop-rule estimate (or exact error when x_ref was given) */
  double t_sketch_ms, t_factor_ms, t_iter_ms, t_total_ms;
  double bytes_streamed; /* algorithmic bytes of A read by the iteration passes           */
  double mu;             /* step used by lsq_ihs_solve                                     */
  int32_t status;        /* this problem's lsq_status (lsq_pcg_solve_batched; else LSQ_OK) */
  int32_t pad_;
  double t_start_ms;     /* lsq_pcg_solve_batched: start of this problem within the launch   */
} lsq_info;

/* S A (m x d) into SA (device, row-major, leading dimension ldsa >= d).  sa_dtype must be LSQ_F64.
 * A NaN or an infinity in A propagates into S A (every embedding here mixes each row of A into at
 * least one row of S A); lsq_factor and the solvers report it as LSQ_ERR_NONFINITE.
 * Section 2.  Errors: INVALID_ARG for m < 1, m > N (SRHT), m > n (Haar), s outside [1, min(m, 32)]
 * (SJLT), a compute other than LSQ_F64 for Haar, lda < d, null pointers; UNSUPPORTED for d > 1024 or,
 * for Haar, m > min(1024, n/4) (the m x m Gram of the draws is factored once on the device, which keeps
 * the rows orthonormal to rounding while the n x m draws are well conditioned; the workspace holds the
 * n x m draws in FP64); RANK if that Gram is not positive definite. */
lsq_status lsq_sketch(lsq_ctx* ctx, const lsq_problem* prob, const lsq_sketch_desc* desc, void* SA,
                      int64_t ldsa, int32_t sa_dtype);

/* Upper-triangular R (d x d, row-major, positive diagonal) with R^T R = (SA)^T (SA) of SA (m x d,
 * row-major, ld lds, m >= d), and W = R^{-1} (d x d, row-major).  Section 1.2 (the paper names QR of S A
 * or a Cholesky factor of H_S = (SA)^T (SA)).  Default: CholeskyQR2, R = chol(Q1^T Q1) chol(X^T X) with
 * X = SA and Q1 = X chol(X^T X)^{-1}, backward stable like QR (lsq_pcg_solve and lsq_choose_sketch_size
 * instead stop at R = chol(X^T X), the Cholesky factor of H_S itself, when the spread max|R_jj| / min|R_jj|
 * of that factor is at most 2e5: its error, about eps kappa(SA)^2 relative, perturbs the preconditioned
 * operator by a factor 1 + O(eps kappa^2), which leaves the PCG iteration count unchanged there and never
 * the verified answer); when the first Cholesky breaks down or its spread exceeds 1e7 (kappa(SA) beyond
 * about 1e7), Householder QR for m <= 8192 and shifted CholeskyQR3 above.  Option "factor" 4 forces
 * CholeskyQR2 and 5 the one-pass factor, everywhere (both with the same fallbacks).  Option "factor" 1
 * selects Householder QR alone; 2
 * selects the SVD (LSRN) form: R by Householder QR (m <= 8192, rank deficiency allowed) or CholeskyQR2,
 * then one-sided Jacobi on R gives S A = U Sigma V^T; R is returned as Sigma V^T and W = V Sigma^+
 * (both dense; singular values at or below 1e-12 sigma_max dropped, their rows of R and columns of W
 * zero), and every solver then applies H_S^+ = W W^T, so that PCG from x_0 = 0 converges to the
 * minimum-norm solution of a rank-deficient problem.  Option "factor" 3 selects column-pivoted
 * Householder QR: R11 the leading block with |R_kk| > 1e-12 |R_00|, W = P [R11^{-1}; 0] (dense), R returned
 * as R_pivoted P^T; PCG then returns the basic solution on the kept columns (the others exactly zero).
 * R or W may be NULL.  NONFINITE when SA holds a NaN or an infinity (checked before factoring).  RANK
 * when some |R_kk| <= 8 d eps max |R_jj|.  UNSUPPORTED for d > 1024 or m > 65536 (m > 8192 with
 * Householder).  The form is this context's option "factor" (lsq_set_option). */
lsq_status lsq_factor(lsq_ctx* ctx, const double* SA, int64_t m, int64_t d, int64_t lds, double* R,
                      double* W);

/* One fused pass over A (Section 1.2: each PCG step multiplies by A and A^T):
 *   mode 0: w = A^T (A v), scal = ||A v||^2            (v = p,  H p and p^T H p)
 *   mode 1: w = A^T (y - A v), scal = ||y - A v||^2    (v = x,  b - H x and the residual norm)
 *   mode 2: as mode 1 with a_j . v, y_j - a_j . v and the sum over rows in double-double arithmetic,
 *           rounded to FP64 once (the refinement residual of the mixed form; not the paper's, which
 *           does not discuss precision); f32_math must be 0
 * with FP64 arithmetic (FP32 A promoted exactly), or FP32 arithmetic when f32_math = 1 (FP32 A only).
 * w (device, d), scal (device, 1). */
lsq_status lsq_fused_pass(lsq_ctx* ctx, const lsq_problem* prob, int32_t mode, int32_t f32_math,
                          const double* v, double* w, double* scal);

/* lsq_fused_pass (modes 0 and 1) for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It calls no allocating routine and does
 * not touch the context's workspace: the per-workgroup partials and both reduction stages live in a static
 * device array of 8 MiB per device (NOALLOC: 2^20 doubles), loaded with the library and held until the
 * process ends; the workgroup count is capped so that nwg (d + 1) + 33 (d + 1) doubles fit, so results can
 * differ from lsq_fused_pass in the last bits when its grid is larger.  Asynchronous: the work is queued on
 * the context's stream and the call returns without waiting (errors of the launches surface at the
 * caller's next synchronisation).  Every call on one GPU shares that GPU's array (it keeps the last call's
 * contents; every value read is written first by the same call): calls that overlap on one GPU, from any
 * context or stream, race.  INVALID_ARG as lsq_fused_pass; UNSUPPORTED for mode 2. */
lsq_status lsq_fused_pass_noalloc(lsq_ctx* ctx, const lsq_problem* prob, int32_t mode, int32_t f32_math,
                                  const double* v, double* w, double* scal);

/* One row of the sketch-size chooser's table (lsq_choose_sketch_size). */
typedef struct {
  int64_t m;           /* candidate sketch size                                              */
  int32_t iters;       /* T(m) = ceil(log(4 / tol^2) / log(m / d)), Section 6 with rho = d/m  */
  int32_t pad_;
  double t_sketch_ms;  /* measured: fastest of reps sketches on this problem                  */
  double t_factor_ms;  /* measured: fastest of reps factorizations of that sketch             */
  double predicted_ms; /* t_sketch + t_factor + (T(m) + extra_passes) t_pass                  */
  double r_spread;     /* max |R_ii| / min |R_ii| of the factor (about kappa(A) / 25)        */
} lsq_msize_entry;

/* Sketch size m for PCG by Section 6's cost model C(m) = C_sketch(m) + C_factor(m) + T(m) C_pass with
 * T(m) = ceil(log(4 / eps) / log(m / d)), eps = tol^2 (rho = d/m; Theorems 6.1 and 6.2 minimise the same
 * model in flop counts, and Section 6 leaves a hardware-specific version as future work): here the sketch,
 * the factorization and one fused pass are timed on this GPU on the caller's problem (desc's kind, s,
 * compute, seed and t; desc->m is ignored), for m in {1.5, 2, 3, 4, 5, 6, 8, 10, 12, 16, 24, 32, 40, 48, 64}
 * times d (multiples of 64 when d >= 64), above d and within the embedding's limits.  extra_passes: passes
 * over A beyond T(m) that the caller's solve makes (e.g. a verification residual).  reps >= 1 timed rounds
 * after one warm-up round per candidate.  table (host, optional, capacity >= the candidate count, at most
 * 15) receives every candidate; *count (host, optional) their number, *m_best (host) the argmin of the
 * predicted times (ties: the smaller m), *t_pass_ms (host, optional) the pass time.  Synchronous; the sketches
 * use the context's workspace.  Errors as lsq_sketch and lsq_factor; INVALID_ARG for tol outside (0, 1),
 * reps < 1, extra_passes < 0 or a table smaller than the candidate list. */
lsq_status lsq_choose_sketch_size(lsq_ctx* ctx, const lsq_problem* prob, const lsq_sketch_desc* desc, double tol,
                                  double extra_passes, int32_t reps, lsq_msize_entry* table, int32_t capacity,
                                  int32_t* count, int64_t* m_best, double* t_pass_ms);

/* PCG with a fixed sketch (Section 1.2): x (device, d) holds x_0 on entry (zeros are a valid start)
 * and the solution on exit.  The stop rule measures the error relative to that of x_0 (for x_0 = 0,
 * relative to ||A x*||): a warm start already near x* asks for a correspondingly smaller error and
 * can end in LSQ_ERR_NOT_CONVERGED at the rounding floor.  err_trace (device, optional) receives max_iter+1 values per inner solve
 * (see lsq_pcg_opts.x_ref); info (host, optional).  From x_0 = 0 with an SRHT sketch whose first pass
 * streams A in vector form (d and lda multiples of 16 bytes' worth of elements, A aligned, the
 * transform no narrower than A), that pass also forms the first residual A^T y, so the solve reads A
 * once less; x_0 is copied to the host once to decide this. */
lsq_status lsq_pcg_solve(lsq_ctx* ctx, const lsq_problem* prob, const lsq_sketch_desc* desc,
                         const lsq_pcg_opts* opts, double* x, double* err_trace, lsq_info* info);

/* IHS / Polyak-IHS (Section 1.1) for opts->iters iterations from x (device, in: x_0, out: x_iters).
 * err_trace (device, optional, iters+1 values) needs opts->x_ref. */
lsq_status lsq_ihs_solve(lsq_ctx* ctx, const lsq_problem* prob, const lsq_sketch_desc* desc,
                         const lsq_ihs_opts* opts, double* x, double* err_trace, lsq_info* info);

/* FCG / GCC / IPCG (lsq_fcg_opts) for opts->iters iterations from x (device, in: x_0, out: x_iters).
 * One pass over A per iteration (H p_t; the residual is updated as r_{t+1} = r_t - alpha_t H p_t) plus
 * one for r_0, a sketch and a factorization per iteration when refresh = 1.  err_trace (device,
 * optional, iters+1 values) needs opts->x_ref.  The workspace holds min(window, iters) directions and
 * their images H p_j (2 d doubles each).  Errors: INVALID_ARG for iters < 0, window < 0, err_trace
 * without x_ref; UNSUPPORTED for min(window, iters) > 1024; RANK from the factorization. */
lsq_status lsq_fcg_solve(lsq_ctx* ctx, const lsq_problem* prob, const lsq_sketch_desc* desc,
                         const lsq_fcg_opts* opts, double* x, double* err_trace, lsq_info* info);

/* `count` independent problems solved together (Section 1.2 with the sparse embedding of
 * Section 2, the SJLT): the sketch S_i A_i, the Householder QR S_i A_i = Q_i R_i, W_i = R_i^{-1}
 * and PCG (inside FP64 iterative refinement when opts->mixed) of every problem run inside one
 * persistent kernel, problems taken from a work queue ordered by decreasing work per workgroup.  A
 * problem is solved by K_i = round(n_i d_i / "batched_gang_unit") workgroups (1 <= K_i <= 4; lsq_tune,
 * default 8 Mi elements, 0 = one workgroup for every problem): the first factors S_i A_i, then each of
 * the K_i streams its block of rows in every pass, and the partial sums are added in the same order on
 * all of them after a barrier in device memory (bounded: a barrier that runs out of time reports
 * LSQ_ERR_HIP for that problem).  K_i depends on the problem alone, so the results do not depend on
 * the number of workgroups as long as there are at least 4 (UNSUPPORTED when some K_i exceeds it).  The
 * launch is captured in a HIP graph that is replayed while the batch shape (count, workspace sizes,
 * options) stays the same.
 *   probs, descs, xs: host arrays of length count.  xs[i]: device pointer to x_i (d_i entries;
 *     in: x_0, zeros are a valid start; out: the solution).
 *   Rs (optional host array, entries may be NULL): device d_i x d_i row-major buffers that
 *     receive R_i (diag > 0).
 *   infos (optional host array of length count): per-problem iterations, refinements, estimate,
 *     status and phase times (sketch, factor including W, iterations; from the device clock);
 *     t_total_ms is the wall time of the whole batch and t_start_ms the problem's start within it.
 * Limits: descs[i].kind == LSQ_SJLT, 1 <= d_i <= 256, d_i <= m_i <= 1024, 1 <= s_i <= min(m_i, 32),
 * d_i <= n_i <= 2^22; opts->stop_rule 0 only, no inner_f32, no x_ref (UNSUPPORTED otherwise).
 * The call is synchronous.  It returns LSQ_OK when every problem met the stop rule, otherwise the
 * status of the lowest-index problem that did not (every x_i is still written, and infos tell
 * which problems failed). */
lsq_status lsq_pcg_solve_batched(lsq_ctx* ctx, int32_t count, const lsq_problem* probs,
                                 const lsq_sketch_desc* descs, const lsq_pcg_opts* opts,
                                 double* const* xs, double* const* Rs, lsq_info* infos);

/* Draw-level entry points (the specification above), for bit-exact checks.
 *   lsq_draw_srht: signs (device int8, N entries, may be NULL) and rows (device int64, m entries,
 *                  increasing).  N must be a power of two.
 *   lsq_draw_sjlt: targets (device int32, n*s, row-major by row of A, in draw order) and signs
 *                  (device int8, n*s).
 *   lsq_draw_gaussian: g(i, j0 + c) for i < m, c < ncols into G (device FP64, m x ncols row-major),
 *                  unscaled standard normals as the FP64 sketch uses them. */
lsq_status lsq_draw_srht(lsq_ctx* ctx, uint64_t seed, uint64_t t, int64_t N, int64_t m, int8_t* signs,
                         int64_t* rows);
lsq_status lsq_draw_sjlt(lsq_ctx* ctx, uint64_t seed, uint64_t t, int64_t n, int64_t m, int32_t s,
                         int32_t* targets, int8_t* signs);
lsq_status lsq_draw_gaussian(lsq_ctx* ctx, uint64_t seed, uint64_t t, int64_t m, int64_t j0,
                             int64_t ncols, double* G);

/* Wall time (ms, HIP events on the context stream) of the last fused pass launched by the library,
 * and the average over all fused-pass launches since the last reset (for roofline reporting). */
lsq_status lsq_fused_pass_timing(lsq_ctx* ctx, int32_t reset, double* last_ms, double* avg_ms,
                                 int64_t* launches);

/* Measured read ceiling of the device memory, the reference the streaming kernels' achieved bandwidth is
 * compared with beside the datasheet peak: the whole 16-byte vectors of buf (device, 16-byte aligned,
 * `bytes` long) are read `reps` times by a bare streaming-read kernel (the fused pass's 16-byte
 * non-temporal loads, no arithmetic beyond a running sum) at 4, 8 and 16 workgroups per compute unit;
 * *gbs (host) receives the best rate in GB/s (1e9 bytes per second), timed with HIP events on the
 * context's stream.  Synchronous.  INVALID_ARG for null pointers, bytes < 16, reps < 1 or a misaligned
 * buffer. */
lsq_status lsq_read_bandwidth(lsq_ctx* ctx, const void* buf, int64_t bytes, int32_t reps, double* gbs);

/* Measured read + write ceiling, the reference for kernels that stream one buffer in and another out
 * (the SRHT's first pass): the whole 16-byte vectors of src (device, `bytes` long) are copied to dst
 * (device, same length, not overlapping src; both 16-byte aligned) `reps` times by a bare streaming-copy
 * kernel (16-byte non-temporal loads and stores) at 4, 8 and 16 workgroups per compute unit; *gbs (host)
 * receives the best rate in GB/s counting both directions (2 bytes moved per byte copied).  Synchronous.
 * INVALID_ARG for null pointers, bytes < 16, reps < 1, misaligned or overlapping buffers. */
lsq_status lsq_copy_bandwidth(lsq_ctx* ctx, const void* src, void* dst, int64_t bytes, int32_t reps,
                              double* gbs);

/* Process-wide launch parameters, set by the autotuner (paper_1911_02675_amd/autotune.py) from its
 * measured table; they change launch shapes (and with them the fixed order of some reductions), not the
 * method.  Keys: "fused_groups_per_cu" (workgroups per CU of the fused pass, 1..64, default 8);
 * "batched_slots" (workgroups of the batched persistent kernel, 0 = one per compute unit, else
 * 1..65536); "batched_gang_unit" (elements of n d per workgroup of a batched problem's gang, 0 or at
 * least 65536; default 8 Mi); "srht_fold8_rows_f32" / "srht_fold8_rows_f64" (the SRHT's staged second pass folds by
 * the 8-point transform, rather than the 4-point one, from this many selected rows per 256-row bucket on
 * average, FP32 / FP64 intermediate; defaults 64 / 128); "srht_stream_rows_f32" / "srht_stream_rows_f64"
 * (from this many rows per bucket the streamed form with the 16-point fold; default 192 for both);
 * "srht_passa_wgs" (workgroups the SRHT's first
 * pass aims at, 0 = 2^17 for an FP32 transform and 2^15 for FP64, the default); "srht_passb_wgs"
 * (workgroups the LDS-staged second pass aims at when splitting its sums over j_hi, default 8192);
 * "gauss_wgs" (workgroups the Gaussian sketch aims at when splitting the rows of A, default 1024);
 * "gauss_planes_min_d" (the BF16 Gaussian sketch forms the three BF16 terms of A once per chunk of rows
 * and multiplies them in 64 x 512 tiles from this d on, default 384; 1..2^30); "gauss_planes_wgs"
 * (workgroups that form aims at per launch, 8..65536, default 512); "gauss_chunk_rows" (rows of A per
 * chunk of that form, 0 = terms of about 1 GiB, the default; rounded down to a multiple of 32; the
 * terms of one chunk live in the context's workspace);
 * "gram_wgs" (workgroups the CholeskyQR Gram kernel aims at when splitting the rows of S A, default 2048).
 * INVALID_ARG for an unknown key or an out-of-range value. */
lsq_status lsq_tune(const char* key, int64_t value);

/* Numerics options of one context (each context starts with the defaults; calls on other contexts are
 * unaffected).  Keys:
 *   "factor" (Section 1.2 names QR of S A or a Cholesky factor of H_S; Section 6 the same; pivoted QR and
 *     the SVD are the alternatives it cites): 0 = CholeskyQR2 with its fallbacks, the default (PCG takes
 *     one pass or two by the spread of the first factor's diagonal); 1 = Householder QR only; 2 = the SVD
 *     form; 3 = column-pivoted QR; 4 = CholeskyQR2 everywhere; 5 = one-pass CholeskyQR everywhere (see
 *     lsq_factor).  The batched form keeps its own Householder QR.
 *   "srht_passb" (Section 2, SRHT; which kernel evaluates the high-bit sum for buckets of more than 24
 *     selected rows on average): 0 = by the average bucket size, the default: staged through registers
 *     into LDS, sixteen wavefronts of one row tile each (up to 16 tiles of a bucket share one pass over
 *     its block of the intermediate), folding by the 8-point transform from "srht_fold8_rows_f32" /
 *     "_f64" rows per bucket (lsq_tune; 64 / 128) and by the 4-point one below; from
 *     "srht_stream_rows_f32" / "_f64" rows (192) the intermediate streamed into LDS by the memory system
 *     (no staging registers) and folded there in place by the 16-point transform, eight wavefronts of up
 *     to four tiles each (up to 32 tiles per pass); 1 = operands loaded straight into registers (FP32
 *     intermediate; the FP64 one takes its general form); 2 = staged, eight wavefronts, 4-point fold;
 *     3 = staged, sixteen wavefronts, 4-point fold; 4 = the same with the 8-point fold; 5 and 6 =
 *     streamed with the 8- and the 16-point fold.  Every form computes the same sums (exactly, for
 *     integer-valued A).
 *   "sketch_upgrade" (the precision form, mixed = 1, with an SRHT in FP32): 1 = after the factorization
 *     the spread max |R_ii| / min |R_ii| (about kappa(A) / 25 for tall A) is checked, and above 1e6 the
 *     sketch and factor are taken again with an FP64 transform of the same FP32 A, because the FP32
 *     transform's rounding then weakens the preconditioner (measured at n = 2^22, d = 1024, m = 40960:
 *     37 PCG iterations at kappa = 1e8 with the FP32 transform, 17 with the FP64 one; 16 either way at
 *     kappa = 1e7), the default; 0 = never.
 * INVALID_ARG for a null context, an unknown key or an out-of-range value. */
lsq_status lsq_set_option(lsq_ctx* ctx, const char* key, int64_t value);

const char* lsq_status_string(lsq_status s);
const char* lsq_last_error(void);
const char* lsq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LSQ_H */
