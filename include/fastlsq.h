/*
 * fastlsq.h -- C ABI of the MI355X (gfx950) FastLSQ hot path.
 *
 * The method (arXiv 2602.10541):
 *   u_N(x) = (1/sqrt(N)) sum_j beta_j sin(W_j . x + b_j)                     Eq. (1)
 *   D^alpha phi_j(x) = (prod_k W_jk^alpha_k) Phi_{|alpha| mod 4}(W_j . x + b_j) Eq. (2)
 *   with Phi_0..3 = sin, cos, -sin, -cos
 *   A = [A_pde; lambda A_bc], rhs = [f; lambda g]                              Eq. (3)
 *   beta = argmin ||A beta - rhs||^2 + mu ||beta||^2                          Sections 2.3-2.5
 *   Newton: J delta = -R, beta += alpha delta, each step a Tikhonov LSQ        Eq. (4)-(5)
 *
 * Conventions for every call:
 *   - Arrays named "device" are caller-owned device pointers on the context's
 *     device; "host" arrays are caller-owned host memory.  The library only
 *     allocates its own workspace (owned by the context) and opaque factor
 *     objects (owned by the caller, released with flsq_factor_free).
 *   - Matrices are row-major float64 unless stated otherwise.
 *   - Every call is ordered on the context's HIP stream.  Calls whose control
 *     flow needs device results (refinement, Newton, factorisation status)
 *     synchronise that stream before returning; all outputs are valid on return.
 *   - A non-zero status means the outputs are unspecified; flsq_last_error()
 *     returns a text description.  Invalid arguments are rejected before any
 *     kernel is launched.
 *   - Calls on one context must not overlap (one host thread per context).
 */
#ifndef FASTLSQ_H
#define FASTLSQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FLSQ_OK = 0,
    FLSQ_EINVAL = 1,       /* bad argument (sizes, null pointer, multi-index beyond d) */
    FLSQ_ENOTSPD = 2,      /* Cholesky met a non-positive pivot after all shift retries */
    FLSQ_ENOCONV = 3,      /* refinement / Newton hit its iteration limit (outputs hold the last iterate) */
    FLSQ_EHIP = 4,         /* a HIP runtime call failed */
    FLSQ_ENOMEM = 5,       /* workspace allocation failed */
    FLSQ_ENONFINITE = 6    /* a NaN or Inf was found in an input or in the result */
} flsq_status;

/* Arithmetic of the bulk Gram product G = A^T A (Section 2.3, normal equations). */
typedef enum {
    FLSQ_PREC_FP64 = 0,          /* FP64 assembly, FP64 MFMA Gram, FP64 Cholesky + refinement */
    FLSQ_PREC_FP32_REFINE = 1,   /* FP32 assembly + FP32 MFMA Gram -> FP64 Cholesky preconditioner, FP64 refinement */
    FLSQ_PREC_BF16X3_REFINE = 2, /* FP32 entries split into bf16 hi + lo, three bf16 MFMA products, FP32 accumulate */
    FLSQ_PREC_INT8_CRT = 3       /* FP64 entries rounded to ~42-bit integers (per-feature scale), Gram of their
                                    residues modulo 13 coprime odd moduli on the int8 matrix cores (exact
                                    int32 sums), Chinese-remainder reconstruction to FP64; then the FP64
                                    Cholesky + refinement of FLSQ_PREC_FP64.  Needs P <= 133 000 rows. */
} flsq_precision;

#define FLSQ_MAX_DIM 8

/* One term coef * D^alpha of a linear operator (Eq. (2)); alpha[k] = 0 for k >= d. */
typedef struct {
    double coef;
    uint8_t alpha[FLSQ_MAX_DIM];
} flsq_term;

/* A linear operator sum_t terms[t].coef * D^{terms[t].alpha}; terms is host memory. */
typedef struct {
    const flsq_term* terms;
    int32_t n_terms;
} flsq_op;

/* Frozen features (Eq. (1)): W device n_feat x d, b device n_feat; normalize = 1 applies 1/sqrt(N). */
typedef struct {
    int32_t d;
    int32_t n_feat;
    const double* W;
    const double* b;
    int32_t normalize;
} flsq_basis;

/* One row block of Eq. (3): rows A_ij = weight * op[phi_j](x_i), data weight * rhs_i.
 * x: device n_rows x d; rhs: device n_rows (unweighted f or g), may be NULL for calls
 * that take no data. */
typedef struct {
    int64_t n_rows;
    const double* x;
    flsq_op op;
    double weight;
    const double* rhs;
} flsq_rows;

typedef struct {
    double mu;            /* Tikhonov weight on ||beta||^2 (absolute) */
    int32_t prec;         /* flsq_precision */
    int32_t max_refine;   /* CGLS refinement iterations after the Cholesky solve (>= 0) */
    double refine_tol;    /* a column stops when the change of its solution at the collocation rows of
                             even-order blocks (else of its fitted values A beta), relative to their
                             size, is below refine_tol -- or is predicted to be at the next step, once
                             the changes fall at least 10x per iteration; also when FP64 no longer
                             resolves progress (see flsq_solve_info.refine_iters) */
    double shift_rel;     /* initial Cholesky diagonal shift, relative to the unit diagonal of the
                             equilibrated Gram D G D (D = diag(G)^{-1/2}), for the
                             FP32 / BF16x3 preconditioner (0 = automatic) */
    int32_t report_grad;  /* nonzero: fill flsq_solve_info.grad_norm at the returned beta (two extra
                             matrix-free passes); otherwise grad_norm repeats grad_norm0 */
    int32_t second_pass;  /* re-factor through the preconditioned matrix [A; sqrt(mu) I] X (A formed in
                             HBM), so that the refinement converges in a few steps on nearly singular
                             Grams.  0 = automatic (FP64 and INT8_CRT Grams): at factorisation when the
                             first Cholesky needed a diagonal shift and 2 P N^2 <= 2e11, and in the
                             one-call solvers also after 8 refinement steps that did not converge when
                             2 P N^2 <= 4e10; Newton steps take it when asked for, and when a step
                             forms the factor that later steps reuse (flsq_newton_opts.refactor_iters).
                             1 = always (same precisions); -1 = never */
    double pivot_boost;   /* modified Cholesky (Gill and Murray): > 0 raises pivots of the unit-diagonal
                             equilibrated Gram below this value to it during the factorisation, so a
                             Gram that rounding left indefinite factors without a restart unless the
                             raised pivots make entries overflow; 0 = off: a non-positive pivot
                             restarts the factorisation with a diagonal shift (see shift_rel);
                             must be in [0, 1) */
    int32_t store_matrix; /* flsq_factorize only: 1 keeps A and A^T (2 P N doubles) in HBM with the
                             factor, and its products with more than 16 columns (solves, refinement,
                             flsq_apply_A / _At, the inverse-problem calls) stream them through the
                             FP64 matrix cores instead of recomputing the entries; 0 = matrix-free */
} flsq_solve_opts;

typedef struct {
    int32_t refine_iters;   /* refinement iterations performed */
    int32_t chol_retries;   /* Cholesky restarts with a larger shift */
    double shift;           /* diagonal shift added to the unit-diagonal (equilibrated) Gram in the factor
                               (0 for FP64 unless a pivot failed) */
    double grad_norm0;      /* ||A^T (rhs - A beta) - mu beta|| after the Cholesky solve */
    double grad_norm;       /* same, at the returned beta (when opts.report_grad is set) */
    double last_step_rel;   /* relative size of the last refinement step, in the measure refine_tol uses */
    double t_gram_ms, t_chol_ms, t_refine_ms, t_total_ms; /* phases: the Gram phase's device time (HIP
                                events around its kernels), the factorisation from the Gram's end to the
                                inverse factor (host clock), the refinement and the whole call */
    double t_gram_kernel_ms; /* the matrix-core Gram kernel alone (HIP events on the stream): the fused
                                assembly + Gram kernel for FP64 / FP32, the int8 tile kernel for INT8_CRT */
    int32_t second_pass;     /* 1 if the factor was refined by the second pass (opts.second_pass) */
    double t_second_pass_ms; /* its time (included in t_chol_ms) */
    int32_t boosted_pivots;  /* pivots raised by opts.pivot_boost in the factor that was kept */
    int32_t shift_recalled;  /* 1 if the factorisation started at the shift this context kept from an
                                earlier factorisation of a Gram with the same size, settings and 64-bit
                                fingerprint (its upper triangle), skipping the attempts that failed then;
                                chol_retries then counts only retries beyond that shift.  The factor is
                                the one the retries would reach (the kernels are deterministic).  A context
                                keeps up to four such shifts; nothing is fingerprinted for a size whose last
                                factorisation needed no retry. */
} flsq_solve_info;

typedef struct flsq_ctx flsq_ctx;
typedef struct flsq_factor flsq_factor;

/* Context bound to HIP device `device` and stream `hip_stream` (a hipStream_t; NULL = the
 * default stream).  Returns FLSQ_EHIP if the device cannot be selected. */
flsq_status flsq_create(flsq_ctx** ctx, int device, void* hip_stream);
void flsq_destroy(flsq_ctx* ctx);
const char* flsq_last_error(const flsq_ctx* ctx);
/* Library version and the offload architecture it was built for (static strings). */
const char* flsq_build_info(void);

/* Assembly to HBM (Eq. (2)-(3)): A_out is device P x n_feat row-major, P = sum of block rows,
 * float64 if fp32 == 0, float32 otherwise; rhs_out (nullable) device P float64 = weight * rhs.
 * A debugging / checking path: the solvers never write A to memory. */
flsq_status flsq_assemble(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks,
                          int32_t fp32, void* A_out, double* rhs_out);

/* Gram product of the stacked blocks without forming A (fused assembly + MFMA):
 * G_out device n_feat x n_feat float64 (full symmetric) = A^T A computed in precision `prec`
 * (mu is NOT added).  c_out (nullable) device n_feat = A^T rhs_w computed in FP64. */
flsq_status flsq_gram(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks,
                      int32_t prec, double* G_out, double* c_out);

/* Linear solve (Algorithm 1 with the Tikhonov weight of Section 2.4): beta_out device n_feat.
 * Normal equations (A^T A + mu I) beta = A^T rhs_w: Gram in opts->prec, FP64 Cholesky, then
 * CGLS refinement with FP64 matrix-free products A v and A^T y, preconditioned by the factor.
 * info may be NULL.  Returns FLSQ_ENOCONV if refinement did not reach refine_tol within
 * max_refine iterations (beta_out then holds the last iterate). */
flsq_status flsq_solve_linear(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks,
                              const flsq_solve_opts* opts, double* beta_out, flsq_solve_info* info);

/* Factor object (Section 2.5): one factorisation reused for every right-hand side and every
 * adjoint solve of the same system, as in the inverse application.
 * Copies the basis and block geometry to the device; the caller's arrays may be freed after. */
flsq_status flsq_factorize(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks,
                           const flsq_solve_opts* opts, flsq_factor** F, flsq_solve_info* info);
void flsq_factor_free(flsq_factor* F);
/* Number of rows P and features N of a factor (host outputs). */
flsq_status flsq_factor_shape(const flsq_factor* F, int64_t* n_rows, int32_t* n_feat);

/* Multi-RHS least squares with the cached factor: rhs_rows device P x K (already weighted,
 * i.e. rows of the stacked right-hand side), beta_out device n_feat x K. */
flsq_status flsq_factor_solve(flsq_ctx* ctx, const flsq_factor* F, const double* rhs_rows, int32_t K,
                              double* beta_out, flsq_solve_info* info);
/* out = (A^T A + mu I)^{-1} V, V and out device n_feat x K, refined with FP64 matrix-free products. */
flsq_status flsq_factor_solve_normal(flsq_ctx* ctx, const flsq_factor* F, const double* V, int32_t K,
                                     double* out);
/* out = A V (device P x K) and out = A^T Y (device n_feat x K), FP64, matrix-free. */
flsq_status flsq_apply_A(flsq_ctx* ctx, const flsq_factor* F, const double* V, int32_t K, double* out);
flsq_status flsq_apply_At(flsq_ctx* ctx, const flsq_factor* F, const double* Y, int32_t K, double* out);

/* Evaluation of D^alpha u_N at query points (Eq. (1)-(2)).
 * beta: device n_feat float64.  xq: device n_q x d, float32 if xq_is_fp32 else float64.
 * alphas: host n_alpha x d uint8 multi-indices.  out: device n_q x n_alpha, same dtype as xq. */
flsq_status flsq_evaluate(flsq_ctx* ctx, const flsq_basis* basis, const double* beta, int64_t n_q,
                          const void* xq, int32_t xq_is_fp32, const uint8_t* alphas, int32_t n_alpha,
                          void* out);

/* ---- Allocation-free evaluation, for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc) ----
 * Same arguments, kernels and results as flsq_evaluate, but the per-call staging (transposed W,
 * folded coefficients, FP32 copies, the multi-index list: 12 d N + 12 n_alpha N + 4 N + d n_alpha
 * bytes, each piece rounded up to 256) lives in a static device array of FLSQ_EVAL_SCRATCH_BYTES,
 * one copy per GPU, held until the process ends; the call allocates nothing.  N <= 16384 fits for
 * every d <= 8 and n_alpha <= 8.  Larger staging is rejected with FLSQ_EINVAL before any work.
 * All calls on one GPU share that GPU's array, from any context: calls that overlap in time on
 * one GPU (other host threads, other streams) race and must be serialised by the caller.  Every
 * staged value is written before it is read, so the array's previous contents do not matter. */
#define FLSQ_EVAL_SCRATCH_BYTES (4 << 20)
flsq_status flsq_evaluate_noalloc(flsq_ctx* ctx, const flsq_basis* basis, const double* beta, int64_t n_q,
                                  const void* xq, int32_t xq_is_fp32, const uint8_t* alphas, int32_t n_alpha,
                                  void* out);

/* Pointwise nonlinearity N(u) = sum_k poly[k] u^k (host array) applied on one row block. */
typedef struct {
    int32_t n_poly;
    const double* poly;
} flsq_nonlin;

typedef struct {
    flsq_solve_opts lin;    /* per-step linear solve */
    double tol_dbeta;       /* stop when ||alpha delta||_2 < tol_dbeta */
    int32_t max_iter;       /* Newton steps after the warm start */
    double armijo_c;        /* sufficient decrease ||R(beta + a d)|| <= (1 - c a) ||R(beta)|| */
    int32_t max_halvings;   /* backtracking halvings before the smallest step is taken */
    int32_t warm_start;     /* 1: beta_inout is overwritten by the linear solve with N dropped */
    int32_t refactor_iters; /* > 0: a step's solve is preconditioned by the factor of the last system
                               factored (the warm start's, or an earlier step's) for at most this many
                               CG steps, and forms its own Jacobian Gram and factor (with the second
                               pass) only if they do not converge; the Newton step is solved to the
                               same tolerance either way.  0: every step forms its own Gram and
                               factor. */
} flsq_newton_opts;

typedef struct {
    int32_t iters;                   /* Newton steps taken */
    int32_t converged;               /* ||alpha delta|| < tol_dbeta reached */
    double res_norm[64];             /* ||R|| at the start of each step */
    double alpha[64];
    double step_norm[64];            /* ||alpha delta|| */
    double du_rel[64];               /* ||Delta u|| / ||u|| at collocation rows */
    int32_t halvings[64];
    double t_total_ms;
    int32_t refine_iters[64];        /* CGLS iterations of each step's linear solve */
    double shift[64];                /* Cholesky diagonal shift of each step's factor */
    double t_solve_ms[64];           /* Gram + factor + refinement time of each step */
    int32_t factored[64];            /* 1 if the step formed its own Gram and factor */
} flsq_newton_trace;

/* Newton-Raphson for L[u] + N(u) = f (Section 2.4).  The nonlinearity acts on block
 * `nonlin_block`, whose operator must contain only even-order terms (the Jacobian
 * row coefficient N'(u_i) multiplies phi_j = sin, Eq. (2) with |alpha| = 0).
 * beta_inout: device n_feat.  trace may be NULL.  max_iter <= 64. */
flsq_status flsq_solve_newton(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks,
                              int32_t nonlin_block, const flsq_nonlin* nonlin, const flsq_newton_opts* opts,
                              double* beta_inout, flsq_newton_trace* trace);

/* ---- Inverse heat-source support (Section 2.5 and the inverse heat-source application) ----
 * Source s(x; theta) = a exp(-((x0 - cx)^2 + (x1 - cy)^2) / (2 w^2)), theta = (a, cx, cy, w).
 * The factor F is built for the full system; the source acts on its first `n_src_rows` rows
 * (the interior block, row weight `src_weight`), the remaining rows carry zero data. */

/* Misfit and gradients for K hypotheses in one call:
 *   B = (A^T A + mu I)^{-1} A^T rhs(theta_h)   (refined with the cached factor)
 *   U = H B, H_kj = phi_j(x_obs,k) (with 1/sqrt(N)), L_h = mean_k (U_kh - data_k)^2
 *   Lam = (A^T A + mu I)^{-1} H^T (2/n_obs)(U - data)
 *   dL_h/dtheta_h = (A Lam_h)^T d rhs_h / d theta_h
 *   dL_h/dkappa   = (A_k Lam_h)^T (rhs_h - A B_h) - (A Lam_h)^T (A_k B_h)
 * where A_k = dA/dkappa: the interior operator is d/dt - kappa Laplace_x, so A_k is the
 * row-block assembly of +(sum_k D^{2 e_k}) over `n_lap_dims` leading coordinates, negated.
 * thetas: device K x 4; x_obs: device n_obs x d; data: device n_obs.
 * loss_out: device K; grad_theta_out: device K x 4; grad_kappa_out: device K (nullable). */
flsq_status flsq_inverse_loss_grad(flsq_ctx* ctx, const flsq_factor* F, int64_t n_src_rows, double src_weight,
                                   int32_t n_lap_dims, const double* thetas, int32_t K, int64_t n_obs,
                                   const double* x_obs, const double* data, double* loss_out,
                                   double* grad_theta_out, double* grad_kappa_out);

/* Observation operator of the factored system (the cached-solve idea of the paper's
 * matrix-caching appendix applied to Section 2.5): with Z = (A^T A + mu I)^{-1} H^T (n_obs solves
 * with the factor, refined like every other solve), keeps
 *   R = H (A^T A + mu I)^{-1} A_src^T   (n_obs x n_src_rows, A_src = the first n_src_rows rows)
 * on the factor, in FP64.  Since rhs(theta) vanishes outside those rows, U = H B = R rhs_src, and
 * since Lam = Z g_u, (A Lam)_src = R^T g_u: afterwards flsq_inverse_loss_grad calls that ask for no
 * kappa gradient (grad_kappa_out NULL) with the same n_src_rows and x_obs pointer (and n_obs)
 * take two products with R instead of the two refined solves and the passes over A, with the
 * same results up to rounding.  Cost: ceil(n_obs / 64) multi-column solves and passes, once;
 * memory about 2 n_obs n_src_rows doubles.  Re-factoring F drops it.
 * x_obs: device n_obs x d (the pointer is the cache key); n_obs >= 1. */
flsq_status flsq_inverse_prepare(flsq_ctx* ctx, flsq_factor* F, int64_t n_src_rows, int64_t n_obs,
                                 const double* x_obs);

/* ---- Learnable bandwidth (the reparameterisation appendix, Eq. for W_j = L What_j) ----
 * base: the frozen draws, base->W = What (device n_feat x d row-major) and base->b; the
 *   weights actually used are W_j = L What_j.  The scalar bandwidth is L = sigma I.
 * L: host d x d row-major, lower triangular (entries above the diagonal must be 0).
 * blocks: the stacked operator rows with their data (rhs required), as for flsq_solve_linear.
 * opts: the inner solve (Tikhonov weight mu, Gram precision, refinement), as for flsq_factorize.
 * Outputs: beta_out device n_feat, the inner solution beta* = (A^T A + mu I)^{-1} A^T rhs_w;
 *   loss_out host scalar, the outer loss ||A beta* - rhs_w||^2 (rows weighted, mu term excluded);
 *   grad_out host d(d+1)/2, dLoss/dL_pq for q <= p packed row by row ((0,0), (1,0), (1,1), ...),
 *   the exact derivative of that loss through the regularised inner solve:
 *     dLoss/dL_pq = -2 [ r^T A' beta* + mu ( r^T A' lam - (A lam)^T A' beta* ) ],
 *   r = rhs_w - A beta*, lam = (A^T A + mu I)^{-1} beta*, A' = dA/dL_pq (Eq. (2) differentiated
 *   in W: a quarter-period phase shift, so every A' product is a matrix-free FP64 pass).
 * Errors: FLSQ_EINVAL for NULL arguments, a non-lower-triangular L or invalid blocks;
 *   FLSQ_ENONFINITE for a non-finite L; solver errors as for flsq_factorize / flsq_factor_solve. */
flsq_status flsq_bandwidth_loss_grad(flsq_ctx* ctx, const flsq_basis* base, const double* L, const flsq_rows* blocks,
                                     int32_t n_blocks, const flsq_solve_opts* opts, double* beta_out,
                                     double* loss_out, double* grad_out);

/* ---- Row-dependent coefficients (the coil operator nu Laplace A + grad nu . grad A of the
 * applications section) and nonlinearities with first derivatives (steady Burgers u u' - nu u''
 * of the Newton experiments, Section 2.4) ----
 * A row block whose operator is sum_t a_t(x) L_t with constant-coefficient operators L_t
 * (Eq. (2) per channel) and per-row coefficients a_t:
 *   A_ij = weight * sum_t a_t(x_i) L_t[phi_j](x_i),   data weight * rhs_i.
 * These operators are assembled explicitly to HBM (row-major and transposed, 16 P N bytes) and
 * solved through the Gram of the stored matrix on the FP64 matrix cores, the FP64 Cholesky of
 * flsq_solve_linear and CGLS refinement with the stored matrix; only FLSQ_PREC_FP64 is accepted. */
#define FLSQ_MAX_CHANNELS 8

typedef struct {
    flsq_op op;              /* L_t (host terms) */
    const double* coef;      /* device n_rows: a_t(x_i) for the block's rows; NULL means a_t = 1 */
} flsq_channel;

typedef struct {
    int64_t n_rows;
    const double* x;         /* device n_rows x d */
    double weight;
    const double* rhs;       /* device n_rows (unweighted data); required by the solvers */
    int32_t n_channels;      /* 1 .. FLSQ_MAX_CHANNELS */
    const flsq_channel* channels;   /* host array of n_channels */
} flsq_vrows;

/* A_out device P x n_feat (row-major, P = sum of block rows) = the stacked weighted operator
 * rows; rhs_out (nullable) device P = weight * rhs. */
flsq_status flsq_assemble_var(flsq_ctx* ctx, const flsq_basis* basis, const flsq_vrows* blocks, int32_t n_blocks,
                              double* A_out, double* rhs_out);

/* beta_out device n_feat = argmin ||A beta - rhs_w||^2 + mu ||beta||^2 for the stacked blocks
 * (opts->prec must be FLSQ_PREC_FP64).  info may be NULL; FLSQ_ENOCONV as for flsq_solve_linear. */
flsq_status flsq_solve_linear_var(flsq_ctx* ctx, const flsq_basis* basis, const flsq_vrows* blocks,
                                  int32_t n_blocks, const flsq_solve_opts* opts, double* beta_out,
                                  flsq_solve_info* info);

/* N(u, grad u) = sum_k poly[k] u^k + exp_coef e^u + sum_t adv_coef[t] u^{adv_pow[t]} d_{adv_axis[t]} u
 * (host arrays; n_poly <= 8, n_adv <= 8, adv_pow in [0, 16], 0 <= adv_axis < d).  Steady Burgers:
 * n_poly = 0, one advection term (1, 1, 0); Bratu -Laplace u - lambda e^u: exp_coef = -lambda. */
typedef struct {
    int32_t n_poly;
    const double* poly;
    int32_t n_adv;
    const double* adv_coef;
    const int32_t* adv_pow;
    const int32_t* adv_axis;
    double exp_coef;
} flsq_nonlin_grad;

/* Newton-Raphson (Section 2.4) for sum_t a_t L_t[u] + N(u, grad u) = f, N acting on block
 * `nonlin_block`: residual R_i = w (L[u_N](x_i) + N(u_N, grad u_N)(x_i) - data_i), Jacobian rows
 * L[phi_j] + dN/du phi_j + sum_k dN/d(d_k u) d_k phi_j in closed form, each step the Tikhonov
 * least squares of Eq. (5) with Armijo backtracking (opts->armijo_c, opts->max_halvings).
 * Warm start (opts->warm_start = 1): beta_inout is overwritten by the linear solve with N dropped;
 * otherwise beta_inout is the starting point (continuation in a parameter passes each stage's
 * solution to the next).  Stops when ||Delta u|| / ||u|| at every collocation row < tol_du, or
 * ||alpha delta|| < opts->tol_dbeta; FLSQ_ENOCONV if neither within opts->max_iter (<= 64) steps.
 * opts->lin.prec must be FLSQ_PREC_FP64.  trace may be NULL. */
flsq_status flsq_solve_newton_var(flsq_ctx* ctx, const flsq_basis* basis, const flsq_vrows* blocks,
                                  int32_t n_blocks, int32_t nonlin_block, const flsq_nonlin_grad* nonlin,
                                  const flsq_newton_opts* opts, double tol_du, double* beta_inout,
                                  flsq_newton_trace* trace);

/* Batched Adam step on K x P parameters (all device arrays, updated in place; Kingma and Ba, with
 * Loshchilov and Hutter's decoupled weight decay):
 * p *= 1 - lr weight_decay; m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
 * p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
 * then p[:, clamp_col] = max(p[:, clamp_col], clamp_min) when clamp_col >= 0.  t >= 1. */
flsq_status flsq_adam_step(flsq_ctx* ctx, double* params, const double* grads, double* m, double* v, int32_t K,
                           int32_t P, int32_t t, double lr, double b1, double b2, double eps, int32_t clamp_col,
                           double clamp_min, double weight_decay);

#ifdef __cplusplus
}
#endif

#endif /* FASTLSQ_H */
