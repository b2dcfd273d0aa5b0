// Matrix-free FP64 products with the stacked matrix of Eq. (3): A is recomputed per entry
// from the closed form of Eq. (2) in double precision, never stored.  These carry the
// residual r = rhs - A beta and the gradient A^T r of the refinement in full FP64,
// whatever precision the Gram product used.
//
// Rows are processed in runs of kPassRows rows that never cross a block boundary
// (the host builds that run list), so the per-block amplitude/phase of a run is uniform.
#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

constexpr int kPassRows = 64;        // rows per run (row pass: one run per workgroup)
constexpr int kRowSlices = 4;        // feature slices per row-pass workgroup (one per wave)
constexpr int kRowFeat = 64;         // features staged per slice and round
constexpr int kColFeat = 256;        // features per column-pass workgroup (one per thread)


// ------------------------------------------------------------------ row pass
// out[i][c] = beta_y * Y[i][c] + alpha * sum_j A_ij V[j][c]
// MODE 1: also u_out[i][c] = norm * sum_j V[j][c] sin(W_j.x_i + b_j), the expansion itself at
//         the row, on blocks whose operator is even (their phase is b, so the sine is shared);
//         zero on other blocks.  This is the solution-level quantity the refinement stops on.
// MODE 2 (Newton, K = 1): u_i as above on the nonlinear block, then
//         R_i = (A beta)_i + w N(u_i) - data_i and rho_i = w N'(u_i) norm.
template <int D, int KMAX, int MODE>
__global__ __launch_bounds__(256) void k_rowpass(PassGeo pg, const double* __restrict__ rho,
                                                 const double* __restrict__ V, int K, const double* __restrict__ Y,
                                                 double alpha, double beta_y, double* __restrict__ out,
                                                 // Newton extras
                                                 int nonlin_block, const double* __restrict__ poly, int n_poly,
                                                 double norm, double w_nl, double* __restrict__ rho_out,
                                                 double* __restrict__ u_out) {
  constexpr bool NEWTON = (MODE == 2);
  constexpr int KU = (MODE == 1) ? KMAX : 1;
  constexpr int RF = (KMAX >= 16) ? 16 : kRowFeat;            // features staged per slice and round
  __shared__ double sW[kRowSlices][RF][D + 2];                // W, amp, ph
  __shared__ double sV[kRowSlices][RF][KMAX];
  __shared__ double red[kRowSlices][kPassRows][KMAX < 8 ? KMAX : 8];
  __shared__ double redu[kRowSlices][kPassRows];
  const Geo& g = pg.g;
  const Chunk run = pg.runs[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, slice = tid >> 6;
  const int n = g.n;
  const int64_t i = run.row0 + lane;
  const bool rvalid = lane < run.nrows;
  double x[D];
#pragma unroll
  for (int k = 0; k < D; ++k) x[k] = rvalid ? g.Xt[(int64_t)k * g.P + i] : 0.0;
  const double rh = (rho && rvalid) ? rho[i] : 0.0;
  double acc[KMAX];
#pragma unroll
  for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
  double uacc[KU];
#pragma unroll
  for (int c = 0; c < KU; ++c) uacc[c] = 0.0;
  const bool ev = (MODE == 1) && ((pg.even_mask >> run.block) & 1ull);
  const bool nl = NEWTON && (run.block == nonlin_block);
  const int per_slice = (n + kRowSlices - 1) / kRowSlices;
  const int j_begin = slice * per_slice;
  const int j_end = min(n, j_begin + per_slice);
  for (int r0 = 0; r0 < per_slice; r0 += RF) {
    __syncthreads();
    if (lane < RF) {  // each wave stages its own slice's next RF features
      const int j = j_begin + r0 + lane;
      const bool ok = j < j_end;
#pragma unroll
      for (int k = 0; k < D; ++k) sW[slice][lane][k] = ok ? g.Wt[(int64_t)k * n + j] : 0.0;
      sW[slice][lane][D] = ok ? g.amp[(int64_t)run.block * n + j] : 0.0;
      sW[slice][lane][D + 1] = ok ? g.ph[(int64_t)run.block * n + j] : 0.0;
      for (int c = 0; c < KMAX; ++c) sV[slice][lane][c] = (ok && c < K) ? V[(int64_t)j * K + c] : 0.0;
    }
    __syncthreads();
    const int cnt = min(RF, j_end - (j_begin + r0));
    for (int jj = 0; jj < cnt; ++jj) {
      double z = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) z = fma(sW[slice][jj][k], x[k], z);
      const double s = sin_f64(z + sW[slice][jj][D + 1]);
      const double a = (sW[slice][jj][D] + rh) * s;
#pragma unroll
      for (int c = 0; c < KMAX; ++c) acc[c] = fma(a, sV[slice][jj][c], acc[c]);
      if (MODE == 1 && ev) {
#pragma unroll
        for (int c = 0; c < KU; ++c) uacc[c] = fma(s, sV[slice][jj][c], uacc[c]);
      }
      if (NEWTON && nl) uacc[0] = fma(s, sV[slice][jj][0], uacc[0]);
    }
  }
  // reduce the slices: solution values first (MODE 1)
  if (MODE == 1) {
#pragma unroll
    for (int c0 = 0; c0 < KU; c0 += 8) {
      __syncthreads();
#pragma unroll
      for (int c = 0; c < (KU < 8 ? KU : 8); ++c) red[slice][lane][c] = uacc[c0 + c < KU ? c0 + c : 0];
      __syncthreads();
      if (slice == 0 && rvalid && u_out) {
#pragma unroll
        for (int c = 0; c < (KU < 8 ? KU : 8); ++c) {
          if (c0 + c >= K) break;
          const double s = red[0][lane][c] + red[1][lane][c] + red[2][lane][c] + red[3][lane][c];
          u_out[i * K + c0 + c] = ev ? norm * s : 0.0;
        }
      }
    }
  }
#pragma unroll
  for (int c0 = 0; c0 < KMAX; c0 += 8) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < (KMAX < 8 ? KMAX : 8); ++c) red[slice][lane][c] = acc[c0 + c < KMAX ? c0 + c : 0];
    if (NEWTON && c0 == 0) redu[slice][lane] = uacc[0];
    __syncthreads();
    if (slice == 0 && rvalid) {
#pragma unroll
      for (int c = 0; c < (KMAX < 8 ? KMAX : 8); ++c) {
        if (c0 + c >= K) break;
        const double s = red[0][lane][c] + red[1][lane][c] + red[2][lane][c] + red[3][lane][c];
        const double yv = Y ? Y[i * K + c0 + c] : 0.0;
        if (!NEWTON) {
          out[i * K + c0 + c] = fma(alpha, s, beta_y * yv);
        } else {
          // R_i = (A beta)_i + w N(u_i) - data_i  (K == 1)
          double R = s - yv;
          double rho_i = 0.0;
          if (nl) {
            const double u = norm * (redu[0][lane] + redu[1][lane] + redu[2][lane] + redu[3][lane]);
            double Nu = 0.0, dNu = 0.0, up = 1.0;
            for (int p = 0; p < n_poly; ++p) {
              Nu = fma(poly[p], up, Nu);
              if (p + 1 < n_poly) dNu = fma((double)(p + 1) * poly[p + 1], up, dNu);
              up *= u;
            }
            R += w_nl * Nu;
            rho_i = w_nl * dNu * norm;
            if (u_out) u_out[i] = u;
          }
          out[i] = R;
          if (rho_out) rho_out[i] = rho_i;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ column pass
// part[s][j][c] = sum over the runs of split s of sum_i A_ij Y[i][c]
template <int D, int KMAX>
__global__ __launch_bounds__(256) void k_colpass(PassGeo pg, const double* __restrict__ rho,
                                                 const double* __restrict__ Y, int K, int runs_per_split,
                                                 double* __restrict__ part) {
  __shared__ double sX[kPassRows][D + 1];       // x, rho
  __shared__ double sY[kPassRows][KMAX];
  const Geo& g = pg.g;
  const int n = g.n;
  const int j = blockIdx.x * kColFeat + threadIdx.x;
  const int split = blockIdx.y;
  const bool fvalid = j < n;
  double w[D];
#pragma unroll
  for (int k = 0; k < D; ++k) w[k] = fvalid ? g.Wt[(int64_t)k * n + j] : 0.0;
  double acc[KMAX];
#pragma unroll
  for (int c = 0; c < KMAX; ++c) acc[c] = 0.0;
  const int r_begin = split * runs_per_split;
  const int r_end = min(pg.n_runs, r_begin + runs_per_split);
  for (int ri = r_begin; ri < r_end; ++ri) {
    const Chunk run = pg.runs[ri];
    __syncthreads();
    for (int e = threadIdx.x; e < kPassRows * (D + 1); e += 256) {
      const int r = e / (D + 1), k = e % (D + 1);
      double v = 0.0;
      if (r < run.nrows) v = (k < D) ? g.Xt[(int64_t)k * g.P + run.row0 + r] : (rho ? rho[run.row0 + r] : 0.0);
      sX[r][k] = v;
    }
    for (int e = threadIdx.x; e < kPassRows * KMAX; e += 256) {
      const int r = e / KMAX, c = e % KMAX;
      sY[r][c] = (r < run.nrows && c < K) ? Y[(int64_t)(run.row0 + r) * K + c] : 0.0;
    }
    __syncthreads();
    const double amp = fvalid ? g.amp[(int64_t)run.block * n + j] : 0.0;
    const double ph = fvalid ? g.ph[(int64_t)run.block * n + j] : 0.0;
    for (int r = 0; r < run.nrows; ++r) {
      double z = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) z = fma(w[k], sX[r][k], z);
      const double a = (amp + sX[r][D]) * sin_f64(z + ph);
#pragma unroll
      for (int c = 0; c < KMAX; ++c) acc[c] = fma(a, sY[r][c], acc[c]);
    }
  }
  if (fvalid)
    for (int c = 0; c < K && c < KMAX; ++c) part[((int64_t)split * n + j) * K + c] = acc[c];
}

// out[e] = alpha * sum_sp part[sp][e] + beta_v * V[e].  Workgroup: 64 outputs x 4 groups of
// splits (group g sums splits g, g + 4, ...); the four group sums are added in a fixed
// order, so the result is deterministic.
__global__ __launch_bounds__(256) void k_colpass_reduce(const double* __restrict__ part, int n_split, int n, int K,
                                                        const double* __restrict__ V, double alpha, double beta_v,
                                                        double* __restrict__ out) {
  __shared__ double red[4][64];
  const int o = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + o;
  const int64_t nk = (int64_t)n * K;
  double s = 0.0;
  if (e < nk) {
#pragma unroll 8
    for (int sp = grp; sp < n_split; sp += 4) s += part[(int64_t)sp * nk + e];
  }
  red[grp][o] = s;
  __syncthreads();
  if (grp == 0 && e < nk) {
    const double t = (red[0][o] + red[1][o]) + (red[2][o] + red[3][o]);
    const double v = V ? V[e] : 0.0;
    out[e] = fma(alpha, t, beta_v * v);
  }
}

// ------------------------------------------------------------------ launchers
static int col_splits(const PassGeo& pg, int K) {
  // enough workgroups to fill the chip, partial buffer bounded by ~64 n K doubles
  const int ftiles = (pg.g.n + kColFeat - 1) / kColFeat;
  int want = (2048 + ftiles - 1) / ftiles;
  int cap = K <= 4 ? 256 : (K <= 16 ? 64 : 16);
  int s = want < cap ? want : cap;
  if (s > pg.n_runs) s = pg.n_runs;
  return s < 1 ? 1 : s;
}

size_t pass_work_elems(int n, int n_runs, int K) {
  PassGeo pg{};
  pg.g.n = n;
  pg.n_runs = n_runs;
  return (size_t)col_splits(pg, K) * n * K;
}

#define FLSQ_ROW_K(DIM, KM, MD)                                                                              \
  hipLaunchKernelGGL((k_rowpass<DIM, KM, MD>), dim3(pg.n_runs), dim3(256), 0, s, pg, rho, V, K, Y, alpha,     \
                     beta_y, out, -1, nullptr, 0, pg.norm, 0.0, nullptr, u_out)

#define FLSQ_ROW_CASE(DIM)                                                  \
  case DIM:                                                                 \
    if (u_out) {                                                            \
      if (K <= 1) FLSQ_ROW_K(DIM, 1, 1);                                    \
      else if (K <= 4) FLSQ_ROW_K(DIM, 4, 1);                               \
      else FLSQ_ROW_K(DIM, 16, 1);                                          \
    } else {                                                                \
      if (K <= 1) FLSQ_ROW_K(DIM, 1, 0);                                    \
      else if (K <= 4) FLSQ_ROW_K(DIM, 4, 0);                               \
      else if (K <= 16) FLSQ_ROW_K(DIM, 16, 0);                             \
      else FLSQ_ROW_K(DIM, 64, 0);                                          \
    }                                                                       \
    break;

hipError_t launch_rowpass_runs(const PassGeo& pg, const double* rho, const double* V, int K, const double* Y,
                               double alpha, double beta_y, double* out, hipStream_t s, double* u_out) {
  if (K > 64 || K < 1) return hipErrorInvalidValue;
  if (u_out && K > 16) return hipErrorInvalidValue;
  if (pg.n_runs == 0) return hipSuccess;
  switch (pg.g.d) {
    FLSQ_ROW_CASE(1) FLSQ_ROW_CASE(2) FLSQ_ROW_CASE(3) FLSQ_ROW_CASE(4)
    FLSQ_ROW_CASE(5) FLSQ_ROW_CASE(6) FLSQ_ROW_CASE(7) FLSQ_ROW_CASE(8)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define FLSQ_COL_K(DIM, KM)                                                                               \
  hipLaunchKernelGGL((k_colpass<DIM, KM>), dim3(ftiles, splits), dim3(256), 0, s, pg, rho, Y, K, per, work)

#define FLSQ_COL_CASE(DIM)          \
  case DIM:                         \
    if (K <= 1) FLSQ_COL_K(DIM, 1); \
    else if (K <= 4) FLSQ_COL_K(DIM, 4); \
    else if (K <= 16) FLSQ_COL_K(DIM, 16); \
    else FLSQ_COL_K(DIM, 64); \
    break;

hipError_t launch_colpass_runs(const PassGeo& pg, const double* rho, const double* Y, int K, const double* V,
                               double alpha, double beta_v, double* out, double* work, hipStream_t s) {
  if (K > 64 || K < 1) return hipErrorInvalidValue;
  const int n = pg.g.n;
  const int ftiles = (n + kColFeat - 1) / kColFeat;
  const int splits = col_splits(pg, K);
  const int per = (pg.n_runs + splits - 1) / splits;
  if (pg.n_runs > 0) {
    switch (pg.g.d) {
      FLSQ_COL_CASE(1) FLSQ_COL_CASE(2) FLSQ_COL_CASE(3) FLSQ_COL_CASE(4)
      FLSQ_COL_CASE(5) FLSQ_COL_CASE(6) FLSQ_COL_CASE(7) FLSQ_COL_CASE(8)
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t tot = (int64_t)n * K;
  hipLaunchKernelGGL(k_colpass_reduce, dim3((unsigned)((tot + 63) / 64)), dim3(256), 0, s, work,
                     pg.n_runs > 0 ? splits : 0, n, K, V, alpha, beta_v, out);
  return hipGetLastError();
}

#define FLSQ_NEWTON_CASE(DIM)                                                                              \
  case DIM:                                                                                                \
    hipLaunchKernelGGL((k_rowpass<DIM, 1, 2>), dim3(pg.n_runs), dim3(256), 0, s, pg, nullptr, beta, 1,     \
                       data_w, 1.0, 1.0, R, nonlin_block, poly, n_poly, norm, w_nl, rho_out, u_out);       \
    break;

hipError_t launch_newton_residual_runs(const PassGeo& pg, const double* beta, const double* data_w,
                                       int nonlin_block, const double* poly, int n_poly, double w_nl, double norm,
                                       double* R, double* rho_out, double* u_out, hipStream_t s) {
  if (pg.n_runs == 0) return hipSuccess;
  switch (pg.g.d) {
    FLSQ_NEWTON_CASE(1) FLSQ_NEWTON_CASE(2) FLSQ_NEWTON_CASE(3) FLSQ_NEWTON_CASE(4)
    FLSQ_NEWTON_CASE(5) FLSQ_NEWTON_CASE(6) FLSQ_NEWTON_CASE(7) FLSQ_NEWTON_CASE(8)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int pass_rows() { return kPassRows; }

}  // namespace flsq
