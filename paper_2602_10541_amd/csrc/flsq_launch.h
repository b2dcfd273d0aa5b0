// Host-side launchers of the gfx950 kernels (internal to libfastlsq).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flsq_device.h"

namespace flsq {

// ---- coefficient preparation, layout transforms, assembly to HBM, evaluation
struct OpTerms {
  int n_terms;
  double coef[32];
  uint8_t alpha[32][kMaxDim];
};
hipError_t launch_prep_block(const OpTerms& op, double weight, double norm, int d, int n, const double* W,
                             const double* b, double* amp, double* ph, float* amp32, float* ph32,
                             hipStream_t s);
// Rows of up to kRowStageMax blocks (block0 + b is the global index of group member b):
// Xt / Xt32 (d x P), Xrm (P x d), row_block and rhs_w = weight * rhs (0 for a NULL rhs).
constexpr int kRowStageMax = 16;
struct RowStage {
  const double* x[kRowStageMax];     // n_rows x d row-major
  const double* rhs[kRowStageMax];   // nullable
  double weight[kRowStageMax];
  int64_t row0[kRowStageMax];
  int64_t rows[kRowStageMax];
  int block0;
  int count;
};
hipError_t launch_stage_rows(const RowStage& rs, int d, int64_t P, double* Xt, float* Xt32, double* Xrm,
                             int32_t* row_block, double* rhs_w, hipStream_t s);
hipError_t launch_transpose(const double* X, int64_t rows, int d, double* Xt, float* Xt32, int64_t ld_out,
                            hipStream_t s);
hipError_t launch_pack_features(const double* Wrm, const double* amp, const double* ph, int n_blocks, int n, int d,
                                double* rec, hipStream_t s);
// Learnable bandwidth: W[j] = L What[j] (L lower triangular, row-major kMaxDim x kMaxDim by
// value), ph += delta over count entries, V = [beta_j What_jc | lam_j What_jc] (n x 2d).
struct LowerMat {
  double v[kMaxDim * kMaxDim];
};
hipError_t launch_apply_lower(const double* What, int n, int d, const LowerMat& Lm, double* W, hipStream_t s);
hipError_t launch_add_phase(double* ph, int64_t count, double delta, hipStream_t s);
hipError_t launch_scaled_cols(const double* beta, const double* lam, const double* What, int n, int d, double* V,
                              hipStream_t s);
// Row-dependent-coefficient operators stored explicitly (A_ij = sum_t a_t(x_i)(S sin z + C cos z)).
struct VarTerm {
  double coef;
  int32_t alpha[kMaxDim];
};
struct VarGeo {
  int d, n, T;               // dimension, features, channels per block
  int64_t P;                 // rows
  const double* W;           // n x d
  const double* b;           // n
  const double* X;           // P x d
  const int32_t* row_block;  // P
  const double* S;           // (n_blocks * T) x n
  const double* C;
  const double* acoef;       // T x P
  double* A;                 // P x n (row-major)
  double* At;                // n x P (nullable)
};
hipError_t launch_fold_var(const double* W, int n, int d, const VarTerm* terms, const int32_t* off,
                           const double* scale, int n_slots, double* S, double* C, hipStream_t s);
hipError_t launch_assemble_var(const VarGeo& g, hipStream_t s);
hipError_t launch_rowdot(const double* M, int64_t R, int64_t len, int64_t ld, const double* v, const double* Y,
                         double alpha, double beta_y, double* out, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
// A (P x n, an explicit assembly of the linear rows) += rho_i sin(z_ij + ph_gj) where rho_i != 0
hipError_t launch_add_rho(const Geo& g, const double* rho, double* A, hipStream_t s);
// At (cols x rows, row-major) = A^T for A rows x cols row-major
hipError_t launch_transpose_f64(const double* A, int64_t rows, int cols, double* At, hipStream_t s);
constexpr int kMaxNlTerms = 8;
struct NlSpec {
  int n_poly;
  double poly[kMaxNlTerms];
  int n_adv;
  double c[kMaxNlTerms];
  int m[kMaxNlTerms];
  int slot[kMaxNlTerms];     // derivative slot of each advection term
  int n_slots;
  double exp_coef;           // + exp_coef e^u
};
hipError_t launch_nl_var(const NlSpec& nl, const double* U, int64_t P, int64_t row0, int64_t rows, double w,
                         double* R, double* rho, double* kap, int64_t kap_ld, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_scale_copy(const double* src, double* dst, int64_t n, double scale, hipStream_t s);
hipError_t launch_assemble(const Geo& g, int fp32, void* A, hipStream_t s);
hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s);

struct EvalArgs {
  int d, n, n_alpha;
  int64_t n_q;
  const double* Wt;        // d x n
  const double* b;
  const double* beta;
  const uint8_t* alphas;   // device n_alpha x d
  const void* xq;          // n_q x d
  void* out;               // n_q x n_alpha
  int fp32;
  double norm;
  double* coef;            // workspace n_alpha x n (double)
  float* coef32;           // workspace n_alpha x n
  float* Wt32;             // workspace d x n
  float* b32;              // workspace n
  uint32_t cos_mask;       // bit a set when |alpha_a| is odd
};
hipError_t launch_evaluate(const EvalArgs& a, hipStream_t s);

// ---- fused Gram
struct GramLaunch {
  Geo g;
  int prec;                 // 0 fp64, 1 fp32, 2 bf16x3
  const double* rho;
  const float* rho32;
  const Chunk* chunks;
  int n_chunks;
  int nt;
  int64_t total_units;
  int64_t units_per_wg;
  int max_seg;
  int n_wg;
  void* partial;
};
int gram_tile();
int gram_chunk_rows();
int gram_occupancy(int prec);
hipError_t launch_gram(const GramLaunch& L, hipStream_t s);
hipError_t launch_gram_reduce(int prec, const void* partial, const int32_t* slot_ptr, const int32_t* slots,
                              int nt, int n, double* G, int mirror, double diag_add, hipStream_t s);

// ---- Gram from exact integer products on the int8 matrix cores (k_gram_i8.hip)
constexpr int kI8MaxMod = 16;
struct I8Moduli {
  int n_mod;
  int ip[kI8MaxMod];                 // odd, pairwise coprime, <= 255
  double p[kI8MaxMod];
  double inv_p[kI8MaxMod];
  float pf[kI8MaxMod];
  float inv_pf[kI8MaxMod];
  int cinv[kI8MaxMod][kI8MaxMod];    // cinv[m][k] = p_m^{-1} mod p_k for m < k
  float cinvf[kI8MaxMod][kI8MaxMod]; // the same as floats (exact)
};
struct I8GemmJob {
  const int8_t* R;     // residues [n_mod][KB][n_pad][64]
  int n_pad;           // features padded to whole tiles
  int KB;              // 64-row K blocks (even)
  int nt, n_tiles;     // tiles per side, upper-triangle tiles
  int n_mod;
  const int2* order;   // n_tiles (ti, tj) pairs: the order in which tiles are taken
  int32_t* out;        // [n_mod][n_tiles][256 * 256], tile slot = row-major upper-triangle index
};
// 4 x 4 super-tile order of the upper-triangle tiles of an nt x nt tile grid.
void i8_tile_order(int nt, int2* out);
struct I8CrtJob {
  I8Moduli M;
  const int32_t* Gt;   // k_gram_i8 output
  const double* scale; // c_j 2^-B per feature
  int n, nt, n_tiles;
  double* G;           // n x n row-major, upper triangle (both with mirror)
  int mirror;
  double diag_add;
};
int i8_tile();
int i8_kblock();
size_t i8_gemm_lds_bytes();
// c_j = max_g |amp_gj| + max_i |rho_i| (rho nullable; rho_max: device scalar workspace)
hipError_t launch_i8_scale(const double* amp, int n_blocks, int n, const double* rho, int64_t P, double* rho_max,
                           int B, double* inv_scale, double* scale, hipStream_t s);
// With Y (P doubles), cpart (KB * n_pad doubles of workspace) and c (n doubles) all given, the
// same pass also writes c = A^T Y, summed in a fixed order; all three null otherwise.
hipError_t launch_i8_residues(const Geo& g, const double* rho, const double* inv_scale, const I8Moduli& M, int n_pad,
                              int KB, int8_t* R, const double* Y, double* cpart, double* c, hipStream_t s);
hipError_t launch_gram_i8(const I8GemmJob& J, hipStream_t s);
hipError_t launch_i8_crt(const I8CrtJob& J, hipStream_t s);

// ---- matrix-free FP64 products over the stacked rows (A recomputed per entry)
struct PassGeo {
  Geo g;
  const Chunk* runs;   // block-aligned runs of at most pass_rows() rows
  int n_runs;
  const Chunk* wide;   // block-aligned runs of at most wide_rows() rows (row pass, K <= 16)
  int n_wide;
  uint64_t even_mask;  // bit g set when block g's operator has only even-order terms (phase = b)
  double norm;         // 1/sqrt(N) or 1
};
int pass_rows();
int wide_rows();
size_t pass_work_elems(int n, int n_runs, int K);
// out[i][c] = beta_y * Y[i][c] + alpha * sum_j A_ij V[j][c]   (Y nullable).  With u_out
// (K <= 16) also u_out[i][c] = norm sum_j V[j][c] phi_j(x_i) on even blocks, 0 elsewhere.
// work: rowpass_work_elems(pg, K) doubles (feature-group partials; many-column partials).
hipError_t launch_rowpass_runs(const PassGeo& pg, const double* rho, const double* V, int K, const double* Y,
                               double alpha, double beta_y, double* out, hipStream_t s, double* u_out = nullptr,
                               double* work = nullptr);
size_t rowpass_work_elems(const PassGeo& pg, int K);
// out[j][c] = beta_v * V[j][c] + alpha * sum_i A_ij Y[i][c]   (V nullable)
hipError_t launch_colpass_runs(const PassGeo& pg, const double* rho, const double* Y, int K, const double* V,
                               double alpha, double beta_v, double* out, double* work, hipStream_t s);
// Newton residual R_i = (A beta)_i + w N(u_i) - data_i; rho_i = w N'(u_i) norm; u_i on the nonlinear block.
// work: rowpass_work_elems(pg, 1) doubles.
hipError_t launch_newton_residual_runs(const PassGeo& pg, const double* beta, const double* data_w,
                                       int nonlin_block, const double* poly, int n_poly, double w_nl, double norm,
                                       double* R, double* rho_out, double* u_out, double* work, hipStream_t s);

// ---- dense FP64 linear algebra on the upper Cholesky factor (row-major, G = U^T U)
constexpr int kNb = 64;
// Blocked Cholesky steps (k_chol.hip): factor the diagonal block at k0 in place; block-row
// solve U_kj = U_kk^{-T} G_kj for columns >= k0 + kNb together with block row k of the
// inverse W = U^{-T} (lower triangular); update by the kr (64 or 128) solved panel rows from k0
// of the trailing rows [k0 + kr, row_lim) and columns [k0 + kr, n) of G and of W's columns
// [0, k0 + kr), fused with the factorisation of the next diagonal block at k0 + kr (row_lim
// below n: the next block row only).  W starts zeroed and is complete after the solve of the
// last block row; launch_inv_transpose then writes X = D W^T (upper, zero below; d nullable).
// Pivots below boost (> 0) are raised to it and counted in *nboost; with boost = 0, *info
// receives the first non-positive pivot (1-based), after which the remaining steps return at
// once.
hipError_t launch_potrf(double* G, int n, int k0, int* info, double boost, int* nboost, hipStream_t s);
hipError_t launch_trsm_row(double* G, double* W, int n, int k0, const int* info, hipStream_t s);
hipError_t launch_syrk_potrf(double* G, double* W, int n, int k0, int kr, int row_lim, int* info, double boost,
                             int* nboost, hipStream_t s);
// (nothing is written when *info, the factorisation's device status, is nonzero)
hipError_t launch_inv_transpose(const double* W, const double* d, int n, const int* info, double* X, hipStream_t s);
// dst = D src D + (diag_add + mu D^2) on the diagonal (upper triangle), D = diag(src)^{-1/2} -> d.
hipError_t launch_equilibrate(const double* G, double* dst, int n, double* d, double mu, double diag_add,
                              hipStream_t s);
// C = alpha op(A) B + beta C per descriptor (op(A) = A^T when transA); descriptors in device memory.
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int M, N, K;
  int lda, ldb, ldc;
  int tri;             // launch_gemm_tri only: 1 B upper triangular, 2 A upper triangular, 0 dense
};
hipError_t launch_gemm_batched(const GemmDesc* d_descs, int n_batch, int maxM, int maxN, double alpha, double beta,
                               int transA, hipStream_t s);
// out[e] = sum_s part[s * len + e] (fixed summation order)
hipError_t launch_sum_partials(const double* part, int n_split, int64_t len, double* out, hipStream_t s);
// C = alpha A B with one upper-triangular operand (desc.tri), skipping its zero blocks.  K is
// split across workgroups when the batch has too few tiles to fill the chip; the partials
// use work (work_elems doubles; NULL: no split).
hipError_t launch_gemm_tri(const GemmDesc* d_descs, int n_batch, int maxM, int maxN, int maxK, double alpha,
                           double* work, size_t work_elems, hipStream_t s);
// out = X (X^T v) for upper-triangular X (n x n); tmp n, work precond_work_elems(n).
hipError_t launch_precond_apply(const double* X, int n, const double* v, double* tmp, double* work, double* out,
                                hipStream_t s);
size_t precond_work_elems(int n);
// Z = X (X^T Y) for 2 <= K <= 64 columns (Y, T, Z n x K row-major; T scratch n x K; part
// chol_multi_work_elems(n, K) doubles).  Z must not alias Y or T.
hipError_t launch_chol_solve_multi(const double* X, int n, const double* Y, int K, double* T, double* part, double* Z,
                                   hipStream_t s);
size_t chol_multi_work_elems(int n, int K);
// Kept matrices in FP64 MFMA operand order (16-row tiles x 4-deep k-groups, zero-padded):
// t16_elems(M, L) doubles for an M x L matrix; launch_to_t16 converts a row-major M x L matrix
// (trans = 0) or the transpose of a row-major L x M matrix (trans = 1).
size_t t16_elems(int64_t M, int64_t L);
hipError_t launch_to_t16(const double* src, int64_t M, int64_t L, int trans, double* dst, hipStream_t s);
// out (M x K) = alpha Mt B + beta_y Y for Mt in operand order, B row-major L x K, 1 <= K <= 64;
// part gemm_t16_work_elems(M, L, K) doubles (may be NULL when that is 0); out may alias Y.
hipError_t launch_gemm_t16(const double* Mt, int64_t M, int64_t L, const double* B, int K, const double* Y,
                           double alpha, double beta_y, double* out, double* part, hipStream_t s);
size_t gemm_t16_work_elems(int64_t M, int64_t L, int K);
hipError_t launch_copy_upper(const double* src, double* dst, int n, double diag_add, hipStream_t s);
hipError_t launch_diag_max(const double* G, int n, double* out, hipStream_t s);
// *out = a reproducible 64-bit fingerprint of the upper triangle of G (n x n); part: n words.
hipError_t launch_fingerprint_upper(const double* G, int n, unsigned long long* part, unsigned long long* out,
                                    hipStream_t s);

// ---- small vector kernels
// out[c] = sum_i x[i][c] * y[i][c] over n rows, K columns (deterministic two-stage).
// Up to kDotBatchMax column-dot products with a common column count K: out[p][c] = sum_i x_p[i][c] y_p[i][c].
// Small products run in one launch (a workgroup each); larger ones as launch_dot_cols in turn.
constexpr int kDotBatchMax = 4;
struct DotBatch {
  const double* x[kDotBatchMax];
  const double* y[kDotBatchMax];
  int64_t n[kDotBatchMax];
  double* out[kDotBatchMax];
  int count;
  int K;
};
hipError_t launch_dot_batch(const DotBatch& b, double* work, hipStream_t s);
// Up to kAxpyBatchMax updates y_q[i][c] += sign_q a[c] x_q[i][c] in one launch (launch_cg_step).
constexpr int kAxpyBatchMax = 3;
struct AxpyBatch {
  const double* x[kAxpyBatchMax];
  double* y[kAxpyBatchMax];
  int64_t n[kAxpyBatchMax];
  double sign[kAxpyBatchMax];
  int count;
  int K;
};
hipError_t launch_dot_cols(const double* x, const double* y, int64_t n, int K, double* out, double* work,
                           hipStream_t s);
// out[c] = sum_i u_i s_i Y[i][c] (Y n x K row-major), s_i = X[i * ldx + xcol] or 1 when X is NULL
// (deterministic two-stage reduction; work as for launch_dot_cols).
hipError_t launch_wsum_cols(const double* Y, int64_t n, int K, const double* u, const double* X, int ldx, int xcol,
                           double* out, double* work, hipStream_t s);
// Per-column scalars (K <= 64) passed by value in the kernel arguments, so the iterative
// solvers' step lengths reach the device without a copy or a stream synchronisation.
struct ColScalars {
  double v[64];
};
// y[i][c] += sign * a[c] * x[i][c]
hipError_t launch_axpy_cols(const ColScalars& a, const double* x, double* y, int64_t n, int K, double sign,
                            hipStream_t s);

// NaN / Inf scans of several arrays in one launch: flags[q * wgs + w] for item q and its
// workgroups w < wgs = finite_batch_wgs(fb) (each written, 0 or 1, so nothing needs clearing;
// an item is bad if any of its flags is).
constexpr int kFiniteBatchMax = 8;
constexpr int kFiniteBatchWgs = 64;
struct FiniteBatch {
  const double* p[kFiniteBatchMax];   // nullable: no entries
  int64_t n[kFiniteBatchMax];
  int count;
};
int finite_batch_wgs(const FiniteBatch& fb);
hipError_t launch_finite_batch(const FiniteBatch& fb, int* flags, hipStream_t s);
// dst[i][c] = src[i][c] for the columns c whose bit is set in mask
hipError_t launch_select_cols(const double* src, double* dst, int64_t n, int K, uint64_t mask, hipStream_t s);
// CG steps with device-resident scalars.  alpha_k = gam_k / (d1_k + mu d2_k) (columns set in
// active with both positive, else 0; d2 nullable), then y_q += sign_q alpha x_q for the batch, in
// one launch; alpha_out (K doubles) receives alpha.  keep (nullable): the columns of y_0 set in
// keep_mask are copied to keep before the update.  K <= 64.
hipError_t launch_cg_step(const double* gam, const double* d1, const double* d2, double mu, uint64_t active,
                          double* alpha_out, const AxpyBatch& b, double* keep, uint64_t keep_mask, hipStream_t s);
// A whole CG step of a small system in one workgroup (every vector at most 32768 entries, K <= 64):
// the dots pre[q] . pre[q] -> pre_out[q] (q < n_pre <= 4), alpha as launch_cg_step (to
// alpha_out), the batch's updates with the best-iterate copy into keep, then the dots
// post[q] . post[q] -> post_out[q] (q < n_post <= 2); each dot in k_dot_small's order.
struct CgStepSmall {
  const double* pre[4];
  int64_t pre_n[4];
  double* pre_out[4];
  int n_pre;
  const double* post[2];
  int64_t post_n[2];
  double* post_out[2];
  int n_post;
  const double *gam, *d1, *d2;
  double mu;
  uint64_t active;
  double* alpha_out;
  AxpyBatch step;
  double* keep;
  uint64_t keep_mask;
  int K;
};
bool cg_step_small_fits(const CgStepSmall& a);
hipError_t launch_cg_step_small(const CgStepSmall& a, hipStream_t s);
// gam_new = g . z per column (n x K row-major), p = z + (gam_new / gam_old) p (0 where
// gam_old <= 0), or p = z when gam_old is null; work as for launch_dot_cols.  gam_old is only
// read: the caller alternates the two buffers between iterations.  K <= 64.
hipError_t launch_cg_direction(const double* g, const double* z, double* p, int64_t n, int K, const double* gam_old,
                               double* gam_new, double* work, hipStream_t s);


// ---- inverse heat-source support
hipError_t launch_source(const double* Xt, int64_t P, int64_t n_src, double weight, const double* thetas, int K,
                         double* Rhs, hipStream_t s);
hipError_t launch_source_grad_dot(const double* Xt, int64_t P, int64_t n_src, double weight, const double* thetas,
                                  int K, const double* AL, double* grad, double* work, hipStream_t s);
hipError_t launch_combine_diff(const double* a, const double* b, double* out, int K, hipStream_t s);
hipError_t launch_misfit(const double* U, const double* data, int64_t n_obs, int K, double* loss, double* gu,
                         hipStream_t s);
hipError_t launch_adam(double* p, const double* g, double* m, double* v, int K, int P, int t, double lr, double b1,
                       double b2, double eps, int clamp_col, double clamp_min, double weight_decay, hipStream_t s);

}  // namespace flsq
