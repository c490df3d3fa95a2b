/*
 * kron_regress.h -- C ABI of the MI355X (gfx950) library for subquadratic
 * Kronecker regression (Fahrbach, Fu, Ghadiri, NeurIPS 2022).
 *
 * The library solves, to a (1+eps) approximation,
 *     min_x ||K x - b||_2^2 + lambda ||x||_2^2,   K = A(1) kron A(2) kron ... kron A(N)
 * by Algorithm 2 (FastKroneckerRegression): factor leverage scores, i.i.d. row
 * sampling from their product distribution (Lemma kronecker_cross_leverage_scores),
 * and preconditioned Richardson iteration on the sketched problem (Lemma
 * richardson_iteration) with M^+ = (kron V) D (kron V)^T applied by KronMatMul
 * mode products (Lemma kron_mat_mul) and the sampled products K~ x, K~^T r computed
 * level by level over the distinct sampled rows (Theorem kron_mat_mul_sqrt_decomp).
 *
 * Conventions (all entry points)
 *   - Row-major, last index fastest.  Row (i_1..i_N) of K is the linear index
 *     sum_n i_n prod_{k>n} I_k; column (r_1..r_N) likewise; x is the row-major vec
 *     of an R_1 x .. x R_N tensor; b has prod(I_n) rows.  With nrhs > 1, b is
 *     prod(I) x nrhs and x is prod(R) x nrhs, both row-major.
 *   - Pointers named d_* (and the A[], b, x members) are DEVICE pointers owned by
 *     the caller; the library never frees them.  Host pointers are named h_*.
 *   - Every call runs on the handle's HIP stream.  Calls that return kr_info or a
 *     host value synchronise that stream before returning; others are
 *     asynchronous.  Workspace belongs to the handle; a handle must not be used
 *     from two host threads at once.
 *   - Errors are returned as kr_status; kr_last_error() gives a message.  On an
 *     error no output is guaranteed.  No C++ exception crosses this ABI.
 *   - Sampling randomness: Philox4x64-10 (Salmon et al., SC'11) with key
 *     (seed, stream) and counter (t, n/4, row, 0) for sample t, mode n, sketch
 *     row (0 here); mode n uses output word n%4 and its top 32 bits u pick the
 *     index i with C_{i-1} <= u < C_i on the inclusive CDF of integer weights
 *     Q_i = max(1, round(2^32 l_i / sum l)) (largest weight absorbs the rounding
 *     deficit so sum Q = 2^32).  The sketch weight of a sample is
 *     omega = 1/(m prod_n Q_{i_n} 2^-32).
 */
#ifndef KRON_REGRESS_H
#define KRON_REGRESS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KR_MAX_MODES 8

typedef enum {
  KR_OK = 0,
  KR_WMAXITER = 1,       /* iteration limit reached; x holds the last iterate          */
  KR_EINVAL = -1,        /* invalid argument (shape, range, NaN/Inf input)             */
  KR_ENOMEM = -2,        /* device allocation failed                                   */
  KR_EHIP = -3,          /* HIP runtime error                                          */
  KR_ESINGULAR = -4,     /* lambda = 0 and a factor Gram matrix is singular            */
  KR_EDIVERGED = -5,     /* Richardson produced a non-finite or exploding update       */
  KR_EUNSUPPORTED = -6   /* shape outside the implemented limits                       */
} kr_status;

typedef enum { KR_F64 = 0, KR_F32 = 1 } kr_dtype;

typedef struct kr_handle_s* kr_handle;

/* An implicit response b = K X_true + sigma E, for problems whose dense b would
 * not fit in memory (prod(I) x nrhs entries).  Only the sampled rows of b are
 * ever formed: K X_true at a sampled row by the sample tree's Kronecker-row
 * products (the same contraction as K~x in the iteration), plus sigma E[i][q].
 * E[i][q] is a standard normal drawn by the Box-Muller transform from the first
 * two words (w0, w1) of Philox4x64-10 with key (seed, stream) and counter
 * (i, q, 0, 0), where i is K's row index:
 *   u1 = ((w0 >> 11) + 1) 2^-53 in (0, 1],  u2 = (w1 >> 11) 2^-53 in [0, 1),
 *   E  = sqrt(-2 ln u1) cos(2 pi u2).
 * X_true is a device pointer to prod(R) x nrhs float64 (row-major); the struct
 * itself is read during the call only.  kron_loss and kron_exact accept a
 * generator (they stream every row's noise once: s = K^T E and ||E||^2, see
 * there); tucker_factor_update needs a dense b. */
typedef struct {
  const double* X_true;
  double sigma;
  uint64_t seed;
  uint64_t stream;
} kr_response_gen;

/* One Kronecker regression problem.  A[n] points to an I[n] x R[n] row-major
 * matrix of dtype a_dtype; b to prod(I) x nrhs entries of dtype b_dtype, or b is
 * NULL and gen describes an implicit response. */
typedef struct {
  int32_t N;                       /* number of factors, 1..KR_MAX_MODES            */
  int32_t nrhs;                    /* right-hand sides sharing the sketch (>= 1)    */
  int64_t I[KR_MAX_MODES];         /* rows of each factor (I_n >= R_n)              */
  int64_t R[KR_MAX_MODES];         /* columns of each factor                        */
  const void* A[KR_MAX_MODES];     /* device pointers                                */
  int32_t a_dtype;                 /* kr_dtype                                       */
  int32_t b_dtype;                 /* kr_dtype                                       */
  const void* b;                   /* device pointer, or NULL with gen               */
  const kr_response_gen* gen;      /* host pointer or NULL                           */
} kr_problem;

typedef struct {
  int64_t m;          /* number of row samples; 0 selects Algorithm 2's
                         ceil(1680 R ln(40R) ln(1/delta)/eps)                         */
  int32_t max_iter;   /* Richardson iteration limit (default 200 when <= 0)           */
  int32_t check_every;/* iterations before the first convergence check (when <= 0:
                         the iterations the handle's last solve of the same shape
                         and parameters took, else 8); later checks come after the
                         number the observed contraction rate predicts             */
  double tol;         /* stop when (1-sqrt(eps)) ||d|| <= tol ||x||, per RHS
                         (default when <= 0: 1e-12 for KR_PREC_F64, 1e-9 for the
                         refined precisions)                                          */
  uint64_t seed;      /* Philox key word 0                                            */
  uint64_t stream;    /* Philox key word 1                                            */
  int32_t flags;      /* KR_OPT_* bits                                                */
  int32_t workgroups; /* unused; must be 0                                           */
  int32_t precision;  /* kr_precision of the Richardson iteration (0 = KR_PREC_F64)   */
  int32_t reserved;   /* must be 0                                                    */
  int32_t lev_rows;   /* KR_OPT_APPROX_LEVERAGE: rows k_n of each spectral
                         approximation (0 = 64 R_n ceil(log2(2 R_n)))                 */
  int32_t lev_proj;   /* KR_OPT_APPROX_LEVERAGE: rows r of the Johnson-Lindenstrauss
                         projection, 1..64 (0 = 32)                                   */
} kr_opts;

/* kr_opts.precision.  The fixed point of the Richardson iteration of Algorithm 2
 * is set by the gradient alone; the preconditioner only sets the rate.  The
 * refined precisions therefore keep the residual K~x - b~, the update of x and
 * the norms of the stopping rule in float64, accumulate the adjoint
 * K~^T Omega u in float32 and apply the preconditioner's mode products in
 * KR_PREC_F32: float32; KR_PREC_BF16: bf16 MFMA; KR_PREC_FP8: e4m3 MFMA with
 * per-operand scaling; all with float32 accumulation.  The result is still
 * float64.  Refined precisions are not available in tucker_factor_update or
 * kron_ridge_batched (KR_EUNSUPPORTED). */
typedef enum { KR_PREC_F64 = 0, KR_PREC_F32 = 1, KR_PREC_BF16 = 2, KR_PREC_FP8 = 3 } kr_precision;

/* kr_opts.flags bit 0 (value 1) is reserved and rejected (KR_EINVAL). */
/* kr_opts.flags: with opts.m == 0, take m = ceil(R ln R / eps) samples (R = prod R_n,
 * natural log) instead of Algorithm 2's theory count. */
#define KR_OPT_M_RLNR 2
/* kron_ridge_batched only.  KR_OPT_GRAPH: the enqueued work of the call is
 * captured into a HIP graph the first time and replayed by later calls whose
 * problems, buffers, parameters and handle workspace are all unchanged (the
 * handle keeps one graph; problems on the multi-kernel path run outside it).
 * KR_OPT_AUTOTUNE: the first call for a batch shape (count, orders, sizes) times
 * each candidate launch configuration -- the size above which a problem joins
 * the team of workgroups rather than the one-workgroup queue, and the team's
 * workgroups per compute unit -- by solving the batch with it, keeps the
 * fastest for the handle, and returns the results of a final solve with it. */
#define KR_OPT_GRAPH 4
#define KR_OPT_AUTOTUNE 8
/* kr_opts.flags: approximate leverage scores for large factors, as Algorithm 2's
 * first loop states it, instead of exact ones.  Per factor: a spectral
 * approximation A~ of k_n = opts.lev_rows rows drawn i.i.d. from the even mixture
 * q_i = (||a_i||^2 / ||A||_F^2 + 1/I_n) / 2 of the squared row norms and the
 * uniform distribution (quantised on the 2^32 grid like the sampling weights; row
 * t = a_i / sqrt(k_n q'_i), so E[A~^T A~] = A^T A; Lemma
 * block_sketch_is_spectral_approx, the mixture being a beta-overestimate with
 * beta >= max(1/kappa(A)^2, R_n / (I_n max l)) / 2); the eigen-decomposition of
 * A~^T A~, which also gives the
 * preconditioner's V and Sigma; then the scores of Lemma fast-ls-comp,
 * ||G A~ M a_i||^2 / ((1 + eps/4)(1 - eps/20)) with M = (1 + eps/4)(A~^T A~)^+ and
 * a Gaussian projection G / sqrt(r) of r = opts.lev_proj rows (Lemma
 * random-projection).  Random bits: Philox4x64-10 with key (seed, stream); row t
 * of A~ for mode n from word 0 of counter (t, n, 0, 1) (top 32 bits against the
 * inclusive CDF of those weights); G[c][t] of mode n by the Box-Muller
 * transform above on words 0 and 1 of counter (t, c, n, 2).  The row sampling of
 * K then draws from these scores exactly as from exact ones (any distribution
 * gives an unbiased sketch; its quality is the beta of the scores).  Exact
 * leverage stays the default. */
#define KR_OPT_APPROX_LEVERAGE 16
/* kr_opts.flags (kron_regress, kron_ridge): fill kr_info.loss with the float64
 * loss of the returned x (one kron_loss pass over b, or over the implicit
 * response's noise, after the solve). */
#define KR_OPT_LOSS 32
/* kr_opts.flags (kron_regress, kron_ridge): for three-factor problems, run the
 * sampled products level by level (forward level, rows, adjoint level: three
 * launches per iteration) even where the fused pass applies.  The fused pass
 * (three factors, R_3 <= 16, R_2 R_3 nrhs <= 4096, R_3 nrhs <= 256) forms the
 * first forward level, the rows and the last adjoint level in one launch, one
 * workgroup per run of at most max(1, 8 / nrhs) level-2 prefixes of one level-1
 * prefix; the root adjoint then sums those runs.  Both compute the same sums; the
 * grouping of the last adjoint level's terms differs, so results agree to
 * rounding.  The fused pass is skipped, as if this flag were set, when the runs
 * outnumber 2 S_1 + 4096 (S_1 level-1 prefixes). */
#define KR_OPT_LEVEL_PASSES 64

typedef struct {
  int32_t iters;          /* Richardson iterations performed (max over RHS)          */
  int32_t status;         /* kr_status of the solve                                   */
  int64_t m;              /* samples drawn                                            */
  int64_t distinct_rows;  /* distinct sampled rows of K                               */
  double rel_update;      /* final (1-sqrt(eps))||d|| / ||x|| (max over RHS)          */
  double loss;            /* with KR_OPT_LOSS: f(x) = ||K x - b||^2 + lambda ||x||^2
                             in float64 (max over RHS; kron_loss after the solve),
                             else NaN                                                 */
  double ms;              /* host wall-clock milliseconds of the call                 */
} kr_info;

/* Handle lifetime.  `hip_stream` is a hipStream_t (NULL = default stream). */
kr_status kr_create(kr_handle* h, void* hip_stream);
kr_status kr_destroy(kr_handle h);
kr_status kr_set_stream(kr_handle h, void* hip_stream);
const char* kr_last_error(kr_handle h);
const char* kr_version(void);

/* Algorithm 2, FastKroneckerRegression, with lambda = 0 (Theorem
 * fast_kronecker_regression).  Writes d_x (prod(R) x nrhs, float64).
 * eps in (0, 1/4]; delta in (0, 1) (used only when opts->m == 0).
 * Returns KR_ESINGULAR if a factor Gram matrix is numerically singular. */
kr_status kron_regress(kr_handle h, const kr_problem* p, double eps, double delta,
                       const kr_opts* opts, void* d_x, kr_info* h_info);

/* Algorithm 2 with L2 regularisation lambda >= 0 (Corollary
 * approximate_ridge_regression); sampling uses the statistical leverage scores of
 * K, the preconditioner is (K^T K + lambda I)^+.  Writes d_x (float64). */
kr_status kron_ridge(kr_handle h, const kr_problem* p, double lambda, double eps,
                     double delta, const kr_opts* opts, void* d_x, kr_info* h_info);

/* f(x) = ||K x - b||^2 + lambda ||x||^2 in float64 (the quantity of the
 * guarantee of Theorem fast_kronecker_regression), streaming b once.  x is
 * float64 prod(R) x nrhs; h_loss receives nrhs values.  With an implicit response
 * (p->gen, b = K X_true + sigma E) every noise entry is generated once for
 * s = K^T E and e2 = ||E||^2, and with v = x - X_true
 *   f(x) = v^T (kron A_n^T A_n) v - 2 sigma v^T s + sigma^2 e2 + lambda ||x||^2. */
kr_status kron_loss(kr_handle h, const kr_problem* p, double lambda, const void* d_x,
                    double* h_loss);

/* The loss gate of an implicit-response problem in one pass over its noise: the
 * loss f(x) of kron_loss and OPT = f(x*) at the exact minimiser of kron_exact,
 * nrhs values each (h_loss, h_opt).  p must carry a generator (KR_EINVAL
 * otherwise; with a dense b call kron_exact and kron_loss). */
kr_status kron_loss_opt(kr_handle h, const kr_problem* p, double lambda, const void* d_x, double* h_loss,
                        double* h_opt);

/* kron_ridge without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as kron_ridge; the workspace
 * is a fixed device array of kr_noalloc_capacity() bytes (64 MiB) in the library,
 * one per device, held until the process ends, instead of the handle's
 * growable workspace.  Problems whose workspace exceeds it return
 * KR_EUNSUPPORTED (the message gives both sizes) before anything is enqueued.
 * Every call on a device shares that device's array and overwrites it (the
 * kernels clear what must start at zero); calls that overlap on one device,
 * from any handle or thread, race.  kr_export_sketch after such a call reads
 * the array, so it is valid until the next allocation-free call. */
kr_status kron_ridge_noalloc(kr_handle h, const kr_problem* p, double lambda, double eps,
                             double delta, const kr_opts* opts, void* d_x, kr_info* h_info);
/* Bytes of device scratch behind kron_ridge_noalloc. */
int64_t kr_noalloc_capacity(void);

/* Many independent ridge problems (Algorithm 2 each; uneven N, I_n, R_n and
 * right-hand sides) in one call: count problems probs[i] with regularisation
 * lambda[i] (host array) and outputs d_x[i] (host array of device pointers, each
 * prod(R) x nrhs float64).  Each problem's setup and sketch is enqueued with the
 * single-problem kernels; the Richardson iterations then run in two persistent
 * launches: small problems on a queue (one workgroup per problem, largest
 * first, workgroup barriers only), and the rest iterated together by a team of
 * workgroups in lockstep stages separated by a bounded team barrier (at most
 * 1024 such problems; a large single-factor problem takes the single-problem
 * path).  opts applies to every problem (seed and stream shared; problem i
 * draws with Philox stream opts->stream + i); flags KR_OPT_M_RLNR, KR_OPT_GRAPH
 * and KR_OPT_AUTOTUNE apply; float64 only; every R_n <= 16 and prod(R) x nrhs
 * below 2^31 (else KR_EUNSUPPORTED).  KR_EHIP if the team barrier times out.
 * h_info (host array of count entries, may be NULL) receives each problem's
 * result; the return value is KR_OK when every problem converged, else the first
 * failing problem's status (its message in kr_last_error). */
kr_status kron_ridge_batched(kr_handle h, int32_t count, const kr_problem* probs, const double* lambda,
                             double eps, double delta, const kr_opts* opts, void* const* d_x,
                             kr_info* h_info);

/* The launch configuration the handle's autotuner chose last (or the default
 * when it has tuned nothing): the team threshold in sampled rows x right-hand
 * sides, and the team's workgroups per compute unit (0 = as many as fit).
 * Host pointers; either may be NULL. */
kr_status kr_batched_config(kr_handle h, double* big_rows, int32_t* team_per_cu);

/* The exact minimiser via the factor thin SVDs and KronMatMul (the paper's
 * exact baseline): x* = (kron V) diag(kron s / (kron s^2 + lambda)) (kron U)^T b.
 * Writes d_x (float64, prod(R) x nrhs).  With an implicit response, K^T b =
 * (kron A_n^T A_n) X_true + sigma K^T E (one pass generating the noise) and
 * x* = (kron V) diag(1 / (kron s^2 + lambda)) (kron V)^T K^T b. */
kr_status kron_exact(kr_handle h, const kr_problem* p, double lambda, void* d_x);

/* Algorithm 3 (FastFactorMatrixUpdate): the ALS update of factor `mode` of a
 * Tucker decomposition (Theorem fast_factor_matrix_update).  p->A[0..N-1] are the
 * current factors (A[mode] supplies only its shape), p->b is the tensor X
 * (row-major I_1..I_N, dtype p->b_dtype), p->nrhs must be 1; d_core is the core
 * G (float64, row-major R_1..R_N).  Every row i of the new factor is the
 * (1+eps)-approximate solution of min_y ||K G_(n)^T y - X_(n)[i]||^2 + lambda ||y||^2
 * (K = Kronecker product of the other factors) from its own leverage sketch of K
 * with opts->m samples (0 selects ceil(1680 R' ln(40 R') ln(I_n/delta)/eps),
 * R' = prod_{m != n} R_m), drawn with Philox counter word 2 = row.  Writes
 * d_A_out (I_mode x R_mode float64; may alias p->A[mode]).  h_info: iters = max
 * over rows, distinct_rows = sum over rows.  KR_ESINGULAR when G_(n) G_(n)^T is
 * singular.  eps in (0, 1/3) for the guarantee.  Limits: prod_{m != n} R_m <= 2048. */
kr_status tucker_factor_update(kr_handle h, const kr_problem* p, const void* d_core, int32_t mode,
                               double lambda, double eps, double delta, const kr_opts* opts,
                               void* d_A_out, kr_info* h_info);

/* The exact factor update of Algorithm 1 (TuckerALS), the ALS baseline of the
 * paper's Tucker experiments: every row i of factor `mode` is
 * argmin_y ||K G_(n)^T y - X_(n)[i]^T||^2 + lambda ||y||^2 (K the Kronecker product of
 * the other factors in mode order), solved through its normal equations
 * (G_(n) K^T K G_(n)^T + lambda I) y = G_(n) K^T X_(n)[i]^T with K^T K the Kronecker
 * product of the other Gram matrices and K^T X_(n)^T the tensor-times-matrix chain
 * X x_{m != n} A_m^T.  Arguments as tucker_factor_update (p->b the tensor, FP64 or
 * FP32; d_core float64 R_1..R_N; d_A_out I_mode x R_mode float64, may alias
 * p->A[mode]).  KR_ESINGULAR when the R_mode x R_mode matrix is not positive
 * definite. */
kr_status tucker_factor_exact(kr_handle h, const kr_problem* p, const void* d_core, int32_t mode,
                              double lambda, void* d_A_out);

/* Algorithm 1 (TuckerALS) with the sketched updates, as one call: for each of
 * `sweeps` sweeps, the factor updates of modes 0..N-1 by Algorithm 3
 * (tucker_factor_update with *factor_opts, Philox stream (sweep << 8) | mode),
 * then the core update by Algorithm 2 with b = vec(X) (kron_ridge with
 * *core_opts, stream (sweep << 8) | N), then the relative reconstruction error
 * ||K vec(G) - vec(X)||^2 / ||X||^2 (kron_loss with lambda = 0).  p->b is the
 * tensor X (FP64 or FP32, row-major I_1..I_N, nrhs = 1); p->A[n] are float64
 * device factors, overwritten in place by their updates (a_dtype must be F64);
 * d_core (float64, row-major R_1..R_N) is read by the factor updates and
 * overwritten by each core update.  The streams in the options are ignored.
 * Host outputs (each may be NULL): h_rre[sweeps]; h_iters[sweeps (N + 1)], the
 * iterations of each update in order; *h_failed_step, the index (sweep (N + 1) +
 * step) of an update that did not end in KR_OK, else -1.  The call stops at such
 * an update and returns its status (a positive status such as KR_WMAXITER
 * included: the factors and core then hold that update's result). */
kr_status kr_tucker_als(kr_handle h, const kr_problem* p, void* d_core, double lambda, double eps,
                        double delta, int32_t sweeps, const kr_opts* factor_opts, const kr_opts* core_opts,
                        double* h_rre, int32_t* h_iters, int32_t* h_failed_step);

/* Test support: copy the last solve's sketch to host memory.  Any pointer may be
 * NULL.  h_Q: sum_n I_n uint64 integer weights (mode-major); h_rows: distinct
 * rows as per-mode indices, D x N int32 (sorted by linear row index); h_Omega: D
 * float64 merged weights; h_counts: D int32 multiplicities.  cap is the capacity
 * in distinct rows; *h_D receives D.  After tucker_factor_update the first
 * index of every distinct row is the factor row it belongs to and h_Q holds the
 * weights of the other modes (entries of the row pseudo-mode are zero). */
kr_status kr_export_sketch(kr_handle h, uint64_t* h_Q, int32_t* h_rows, double* h_Omega,
                           int32_t* h_counts, int64_t cap, int64_t* h_D);

/* Test support: the sketch of problem `problem` (0-based) of the last
 * kron_ridge_batched call, in the same form as kr_export_sketch and in the
 * caller's mode order: h_Q holds the weights of the problem's modes in the order
 * it passed them, and h_rows its distinct rows as per-mode indices in that
 * order, sorted by the caller's linear row index (Omega and counts follow the
 * rows).  KR_EINVAL for a problem outside the last call, or for a problem that
 * took the single-problem path (its sketch is not kept).  Valid until the
 * handle's next call. */
/* Test support: the samples t = first .. first + count - 1 of the last single
 * solve (kron_regress, kron_ridge, kron_ridge_noalloc), drawn again from its kept
 * sampling tables with its seed and stream, before any merging: h_idx receives
 * count x N int32 per-mode indices in sample order (row t - first holds
 * (i_1(t), .., i_N(t))), the draws of Algorithm 2's sampling step.  KR_EINVAL
 * when the last call was not a single solve or the range is outside [0, m). */
kr_status kr_export_samples(kr_handle h, int64_t first, int64_t count, int32_t* h_idx);

kr_status kr_export_batched_sketch(kr_handle h, int32_t problem, uint64_t* h_Q, int32_t* h_rows,
                                   double* h_Omega, int32_t* h_counts, int64_t cap, int64_t* h_D);

/* Test support: the float64 leverage scores l_i = a_i^T (A^T A)^+ a_i of every
 * factor (the statistical leverage of the paper's definition in its
 * preliminaries, from which the sampling weights are quantised), sum_n I_n
 * values, mode-major in the caller's mode order, into h_lev (capacity cap
 * values).  problem < 0: the last single solve; else problem `problem` of the
 * last batched call.  A mode without leverage scores (the row pseudo-mode of a
 * Tucker factor update) reads as zeros. */
kr_status kr_export_leverage(kr_handle h, int32_t problem, double* h_lev, int64_t cap);

/* Measurement support: when enabled, every kernel launch of the handle whose
 * name contains `filter`, or one of its '|'-separated alternatives (NULL or "" =
 * every kernel), is bracketed by a pair of
 * HIP events on the handle's stream (adds a little launch overhead per bracketed
 * launch).  kr_profile_enable clears earlier records.
 * kr_profile_query synchronises on the recorded events and returns the number
 * of launches of the named kernel (e.g. "k_stream_loss<16>") and their summed
 * device time in milliseconds (0 launches when the name is unknown). */
kr_status kr_profile_enable(kr_handle h, int32_t enable, const char* filter);
kr_status kr_profile_query(kr_handle h, const char* kernel, int64_t* h_launches, double* h_total_ms);
/* Newline-separated names of the kernels recorded since kr_profile_enable,
 * NUL-terminated in h_buf (KR_EINVAL when cap is too small; the list is cut). */
kr_status kr_profile_list(kr_handle h, char* h_buf, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* KRON_REGRESS_H */
