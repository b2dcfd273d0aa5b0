// Matrix-free FP64 products with the stacked matrix of Eq. (3): A is recomputed per entry
// from the closed form of Eq. (2) in double precision, never stored.  These carry the
// residual r = rhs - A beta and the gradient A^T r of the refinement in full FP64,
// whatever precision the Gram product used.
//
// Rows are processed in runs of kPassRows rows that never cross a block boundary
// (the host builds that run list), so the per-block amplitude/phase of a run is uniform.
//
// Every kernel here evaluates an entry the same way, bit for bit: z = sum_k W_jk x_ik as a
// chain of FMAs from zero in k order, then (amp_gj + rho_i) * sin(z + ph_gj).  The refinement
// and the adjoint solve apply A and A^T in separate kernels; if the two disagreed even in the
// last place, the operator they form would no longer be A^T A for one A, and on these
// systems (cond(A)^2 near 1/eps) that asymmetry can be amplified by 1/lambda_min into the
// solution.
#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

constexpr int kPassRows = 64;        // rows per run (column pass and the many-column row pass)
constexpr int kWideRows = 256;       // rows per wide run (row pass, K <= 16: one per workgroup)
constexpr int kColFeat = 256;        // features per workgroup in the split count of the many-column pass


// ------------------------------------------------------------------ row pass
// out[i][c] = beta_y * Y[i][c] + alpha * sum_j A_ij V[j][c]
// MODE 1: also u_out[i][c] = norm * sum_j V[j][c] sin(W_j.x_i + b_j), the expansion itself at
//         the row, on blocks whose operator is even (their phase is b, so the sine is shared);
//         zero on other blocks.  This is the solution-level quantity the refinement stops on.
// MODE 2 (Newton, K = 1): u_i as above on the nonlinear block, then
//         R_i = (A beta)_i + w N(u_i) - data_i and rho_i = w N'(u_i) norm.
//
// Workgroup: one wide run (<= kWideRows rows of one block) x one group of features.  A lane
// holds RPL rows of the run (x_i in registers) and every feature it visits is used for all
// of them, so the feature data (record {W_j, amp_gj, ph_gj} and V[j][:], read at
// wave-uniform addresses through the scalar cache) cost 1/RPL of a read per entry.  The
// waves of a workgroup split the run's rows into WR groups and the features into FS
// slices; the grid's y dimension adds feature groups to fill the chip.  With one feature
// group the epilogue runs here; otherwise per-group partial sums go to a workspace and
// k_rowpass_finish adds them in group order (deterministic).
template <int KMAX>
struct RowShape {
  static constexpr int RPL = KMAX == 1 ? 4 : (KMAX <= 4 ? 2 : 1);  // rows per lane
  static constexpr int WR = 4 / RPL;                              // row groups (waves along rows)
  static constexpr int FS = RPL;                                  // feature slices per workgroup
  static constexpr int UNROLL = KMAX <= 4 ? 2 : 1;                // features per step (scalar registers)
};

struct RowEpi {
  const double* Y;
  double alpha, beta_y;
  double* out;
  double* u_out;
  double* rho_out;
  const double* poly;
  int n_poly;
  int nonlin_block;
  double norm, w_nl;
};

// Final value of row i, column c from the full sums s = sum_j A_ij V[j][c] and
// su = sum_j phi_j(x_i) V[j][c] (MODE 1 / 2).
template <int MODE>
__device__ __forceinline__ void row_epilogue(const RowEpi& e, int64_t i, int K, int c, double s, double su, bool ev,
                                             bool nl) {
  const double yv = e.Y ? e.Y[i * K + c] : 0.0;
  if (MODE == 1 && e.u_out) e.u_out[i * K + c] = ev ? e.norm * su : 0.0;
  if (MODE != 2) {
    e.out[i * K + c] = fma(e.alpha, s, e.beta_y * yv);
    return;
  }
  // R_i = (A beta)_i + w N(u_i) - data_i  (K == 1)
  double R = s - yv;
  double rho_i = 0.0;
  if (nl) {
    const double u = e.norm * su;
    double Nu = 0.0, dNu = 0.0, up = 1.0;
    for (int p = 0; p < e.n_poly; ++p) {
      Nu = fma(e.poly[p], up, Nu);
      if (p + 1 < e.n_poly) dNu = fma((double)(p + 1) * e.poly[p + 1], up, dNu);
      up *= u;
    }
    R += e.w_nl * Nu;
    rho_i = e.w_nl * dNu * e.norm;
    if (e.u_out) e.u_out[i] = u;
  }
  e.out[i] = R;
  if (e.rho_out) e.rho_out[i] = rho_i;
}

template <int D, int KMAX, int MODE>
__global__ __launch_bounds__(256) void k_rowpass(PassGeo pg, const double* __restrict__ rho,
                                                 const double* __restrict__ V, int K, RowEpi epi,
                                                 double* __restrict__ part) {
  using S = RowShape<KMAX>;
  constexpr int RPL = S::RPL, WR = S::WR, FS = S::FS;
  constexpr bool USUM = (MODE != 0);
  constexpr int KU = (MODE == 1) ? KMAX : 1;
  constexpr int KC = KMAX < 8 ? KMAX : 8;                       // columns per reduction round
  __shared__ double red[FS > 1 ? FS : 1][kWideRows][KC];
  const Geo& g = pg.g;
  const Chunk run = pg.wide[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rg = wave % WR, fs = wave / WR;
  const int n = g.n;
  const int64_t P = g.P;
  // rows of this lane: run.row0 + rg * 64 RPL + 64 r + lane
  double x[RPL][D], rh[RPL];
  bool rv[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int lr = rg * 64 * RPL + 64 * r + lane;
    rv[r] = lr < run.nrows;
    const int64_t i = run.row0 + lr;
#pragma unroll
    for (int k = 0; k < D; ++k) x[r][k] = rv[r] ? g.Xt[(int64_t)k * P + i] : 0.0;
    rh[r] = (rho && rv[r]) ? rho[i] : 0.0;
  }
  double acc[RPL][KMAX], uacc[RPL][KU];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
#pragma unroll
    for (int c = 0; c < KMAX; ++c) acc[r][c] = 0.0;
#pragma unroll
    for (int c = 0; c < KU; ++c) uacc[r][c] = 0.0;
  }
  const bool ev = (MODE == 1) && ((pg.even_mask >> run.block) & 1ull);
  const bool nl = (MODE == 2) && (run.block == epi.nonlin_block);
  const int n_slices = gridDim.y * FS;
  const int per = (n + n_slices - 1) / n_slices;
  const int j_begin = min(n, (int)(blockIdx.y * FS + fs) * per);
  const int j_end = min(n, j_begin + per);
  constexpr int RS = frec_stride(D);
  const double* __restrict__ frb = g.frec + (int64_t)run.block * n * RS;
#pragma unroll S::UNROLL
  for (int j = j_begin; j < j_end; ++j) {
    const double* fr = frb + (int64_t)j * RS;
    double vj[KMAX];
#pragma unroll
    for (int c = 0; c < KMAX; ++c) vj[c] = (KMAX == 1 || c < K) ? V[(int64_t)j * K + c] : 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      double z = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) z = fma(fr[k], x[r][k], z);
      const double sn = sin_f64(z + fr[D + 1]);
      const double a = (fr[D] + rh[r]) * sn;
#pragma unroll
      for (int c = 0; c < KMAX; ++c) acc[r][c] = fma(a, vj[c], acc[r][c]);
      if (MODE == 1 && ev) {
#pragma unroll
        for (int c = 0; c < KU; ++c) uacc[r][c] = fma(sn, vj[c], uacc[r][c]);
      }
      if (MODE == 2 && nl) uacc[r][0] = fma(sn, vj[0], uacc[r][0]);
    }
  }
  // sum the workgroup's feature slices (slice order), then finish or store the partials
  const bool direct = gridDim.y == 1;
  for (int c0 = 0; c0 < KMAX; c0 += KC) {
    for (int pass = 0; pass < (USUM ? 2 : 1); ++pass) {
      if (pass == 1 && MODE == 2 && c0 > 0) break;
      double sum[RPL][KC];
#pragma unroll
      for (int r = 0; r < RPL; ++r)
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          const int cc = c0 + c < KMAX ? c0 + c : 0;
          sum[r][c] = pass == 0 ? acc[r][cc] : uacc[r][cc < KU ? cc : 0];
        }
      if (FS > 1) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPL; ++r)
#pragma unroll
          for (int c = 0; c < KC; ++c) red[fs][rg * 64 * RPL + 64 * r + lane][c] = sum[r][c];
        __syncthreads();
        if (fs == 0) {
#pragma unroll
          for (int r = 0; r < RPL; ++r)
#pragma unroll
            for (int c = 0; c < KC; ++c) {
              double t = red[0][rg * 64 * RPL + 64 * r + lane][c];
#pragma unroll
              for (int q = 1; q < FS; ++q) t += red[q][rg * 64 * RPL + 64 * r + lane][c];
              sum[r][c] = t;
            }
        }
      }
      if (fs != 0 || direct) {
        // keep the sums of the columns in registers for the direct epilogue below
#pragma unroll
        for (int r = 0; r < RPL; ++r)
#pragma unroll
          for (int c = 0; c < KC; ++c) {
            const int cc = c0 + c < KMAX ? c0 + c : 0;
            if (pass == 0) acc[r][cc] = sum[r][c];
            else if (cc < KU) uacc[r][cc] = sum[r][c];
          }
        continue;
      }
      // partials: part[y][i][c] (sums of A V), then part[gridDim.y + y][i][c] (sums of phi V)
      double* dst = part + ((int64_t)(pass * gridDim.y + blockIdx.y) * P) * K;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        if (!rv[r]) continue;
        const int64_t i = run.row0 + rg * 64 * RPL + 64 * r + lane;
#pragma unroll
        for (int c = 0; c < KC; ++c)
          if (c0 + c < K) dst[i * K + c0 + c] = sum[r][c];
      }
    }
  }
  if (!direct || fs != 0) return;
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    if (!rv[r]) continue;
    const int64_t i = run.row0 + rg * 64 * RPL + 64 * r + lane;
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < K) row_epilogue<MODE>(epi, i, K, c, acc[r][c], USUM ? uacc[r][c < KU ? c : 0] : 0.0, ev, nl);
  }
}

// Adds the per-group partial sums of k_rowpass in group order and applies the epilogue.
template <int MODE>
__global__ __launch_bounds__(256) void k_rowpass_finish(const double* __restrict__ part, int n_groups, int64_t P,
                                                        int K, const int32_t* __restrict__ row_block,
                                                        uint64_t even_mask, RowEpi epi) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= P * K) return;
  const int64_t i = e / K;
  const int c = (int)(e - i * K);
  const int64_t len = P * K;
  double s = 0.0, su = 0.0;
  for (int y = 0; y < n_groups; ++y) s += part[(int64_t)y * len + e];
  if (MODE != 0)
    for (int y = 0; y < n_groups; ++y) su += part[(int64_t)(n_groups + y) * len + e];
  const int b = row_block[i];
  row_epilogue<MODE>(epi, i, K, c, s, su, (MODE == 1) && ((even_mask >> b) & 1ull), (MODE == 2) && b == epi.nonlin_block);
}

// ------------------------------------------------------------------ column pass
// part[s][j][c] = sum over the runs of split s of sum_i A_ij Y[i][c]
// A thread owns FPT features (W_j in registers, amp/ph reloaded per run).  The rows of a run
// are staged once in LDS as records {x_i, rho_i, Y[i][:]} and read back as broadcasts, each
// used for all FPT features.
template <int KMAX>
struct ColShape {
  static constexpr int FPT = KMAX <= 4 ? 2 : 1;  // features per thread (4 measured slower: fewer waves)
};

template <int D, int KMAX>
__global__ __launch_bounds__(256) void k_colpass(PassGeo pg, const double* __restrict__ rho,
                                                 const double* __restrict__ Y, int K, int runs_per_split,
                                                 double* __restrict__ part) {
  constexpr int FPT = ColShape<KMAX>::FPT;
  constexpr int RR = (D + 1 + KMAX + 1) & ~1;              // row record: x, rho, Y (even length)
  __shared__ __align__(16) double sR[kPassRows][RR];
  const Geo& g = pg.g;
  const int n = g.n;
  const int j0 = blockIdx.x * 256 * FPT + threadIdx.x;   // features j0 + 256 f
  const int split = blockIdx.y;
  bool fv[FPT];
  double w[FPT][D];
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int j = j0 + 256 * f;
    fv[f] = j < n;
#pragma unroll
    for (int k = 0; k < D; ++k) w[f][k] = fv[f] ? g.Wt[(int64_t)k * n + j] : 0.0;
  }
  double acc[FPT][KMAX];
#pragma unroll
  for (int f = 0; f < FPT; ++f)
#pragma unroll
    for (int c = 0; c < KMAX; ++c) acc[f][c] = 0.0;
  const int r_begin = split * runs_per_split;
  const int r_end = min(pg.n_runs, r_begin + runs_per_split);
  for (int ri = r_begin; ri < r_end; ++ri) {
    const Chunk run = pg.runs[ri];
    __syncthreads();
    for (int e = threadIdx.x; e < kPassRows * RR; e += 256) {
      const int r = e / RR, q = e % RR;
      double v = 0.0;
      if (r < run.nrows) {
        const int64_t i = run.row0 + r;
        if (q < D) v = g.Xrm[i * D + q];
        else if (q == D) v = rho ? rho[i] : 0.0;
        else if (q - D - 1 < K && q - D - 1 < KMAX) v = Y[i * K + (q - D - 1)];
      }
      sR[r][q] = v;
    }
    double amp[FPT], ph[FPT];
#pragma unroll
    for (int f = 0; f < FPT; ++f) {
      const int64_t o = (int64_t)run.block * n + j0 + 256 * f;
      amp[f] = fv[f] ? g.amp[o] : 0.0;
      ph[f] = fv[f] ? g.ph[o] : 0.0;
    }
    __syncthreads();
#pragma unroll 2
    for (int r = 0; r < run.nrows; ++r) {
      double x[D], yv[KMAX];
#pragma unroll
      for (int k = 0; k < D; ++k) x[k] = sR[r][k];
      const double rh = sR[r][D];
#pragma unroll
      for (int c = 0; c < KMAX; ++c) yv[c] = sR[r][D + 1 + c];
#pragma unroll
      for (int f = 0; f < FPT; ++f) {
        double z = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) z = fma(w[f][k], x[k], z);
        const double a = (amp[f] + rh) * sin_f64(z + ph[f]);
#pragma unroll
        for (int c = 0; c < KMAX; ++c) acc[f][c] = fma(a, yv[c], acc[f][c]);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    if (!fv[f]) continue;
    const int64_t j = j0 + 256 * f;
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < K) part[((int64_t)split * n + j) * K + c] = acc[f][c];
  }
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

// ------------------------------------------------------------------ many right-hand sides on MFMA
// For K > 16 columns the passes are dense contractions, A V (rows x K) and A^T Y (features x
// K), and run on FP64 MFMA 16x16x4.  Each lane computes exactly the entry of A that its
// A-operand slot holds (one FP64 sine per lane per 4-deep k-step), so A never leaves
// registers; the other operand (V or Y, row-major with K contiguous) is staged in LDS per
// round with coalesced loads and read in the operand layout, 16 consecutive doubles per 16
// lanes.  Columns come in tiles of 64 (4 blocks of 16); a short last tile is masked.
constexpr int kMmCols = 64;

// Row pass: one run (<= 64 rows, one block) x 64 columns x one slice of the features per
// workgroup (the feature contraction is split into grid.z slices to fill the chip; slice
// results go to part and are summed by k_rowpass_reduce).  Wave w owns rows 16 w .. 16 w + 15
// of the run; k-steps of 4 features: A[m][k] = A_{i0 + 16 w + m, j0 + k} (lane l: m = l % 16,
// k = l / 16).  Features and the matching 64 x 64 slab of V are staged in LDS per round.
constexpr int kMmFeat = 64;      // features staged per LDS round

template <int D>
__global__ __launch_bounds__(256) void k_rowpass_mfma(PassGeo pg, const double* __restrict__ rho,
                                                      const double* __restrict__ V, int K, int feat_per_slice,
                                                      double* __restrict__ part) {
  __shared__ double sF[kMmFeat][D + 2];       // W, amp, ph
  __shared__ double sV[kMmFeat][kMmCols];     // V[j][c0 .. c0 + 63]
  const Geo& g = pg.g;
  const Chunk run = pg.runs[blockIdx.x];
  const int c0 = blockIdx.y * kMmCols;
  const int slice = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int n = g.n;
  const int m = lane & 15, kq = lane >> 4;
  const int r = 16 * wave + m;                 // row of the run this lane computes entries for
  const bool rvalid = r < run.nrows;
  const int64_t i = run.row0 + r;
  double x[D];
#pragma unroll
  for (int k = 0; k < D; ++k) x[k] = rvalid ? g.Xt[(int64_t)k * g.P + i] : 0.0;
  const double rh = (rho && rvalid) ? rho[i] : 0.0;
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int jb = slice * feat_per_slice, je = min(n, jb + feat_per_slice);
  for (int j0 = jb; j0 < je; j0 += kMmFeat) {
    const int jn = min(kMmFeat, je - j0);
    __syncthreads();
    for (int e = tid; e < kMmFeat; e += 256) {
      const int j = j0 + e;
      const bool ok = e < jn;
#pragma unroll
      for (int k = 0; k < D; ++k) sF[e][k] = ok ? g.Wt[(int64_t)k * n + j] : 0.0;
      sF[e][D] = ok ? g.amp[(int64_t)run.block * n + j] : 0.0;
      sF[e][D + 1] = ok ? g.ph[(int64_t)run.block * n + j] : 0.0;
    }
    for (int e = tid; e < kMmFeat * kMmCols; e += 256) {
      const int fj = e / kMmCols, c = e % kMmCols;
      sV[fj][c] = (fj < jn && c0 + c < K) ? V[(int64_t)(j0 + fj) * K + c0 + c] : 0.0;
    }
    __syncthreads();
    for (int jj = 0; jj < jn; jj += 4) {
      const int fl = jj + kq;                   // this lane's feature in the slab (zero past jn)
      double z = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) z = fma(sF[fl][k], x[k], z);
      const double a = rvalid ? (sF[fl][D] + rh) * sin_f64(z + sF[fl][D + 1]) : 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sV[fl][16 * b + m], acc[b], 0, 0, 0);
    }
  }
  // slot v: row 4 v + lane / 16 of the wave's 16 rows, column lane % 16 of block b
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rr = 16 * wave + 4 * v + kq;
      const int c = c0 + 16 * b + m;
      if (rr < run.nrows && c < K) part[((int64_t)slice * g.P + run.row0 + rr) * K + c] = acc[b][v];
    }
}

// out[i][c] = alpha sum_s part[s][i][c] + beta_y Y[i][c] over the P x K entries (fixed order).
__global__ __launch_bounds__(256) void k_rowpass_reduce(const double* __restrict__ part, int n_slice, int64_t len,
                                                        const double* __restrict__ Y, double alpha, double beta_y,
                                                        double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int sl = 0; sl < n_slice; ++sl) s += part[(int64_t)sl * len + e];
  out[e] = fma(alpha, s, Y ? beta_y * Y[e] : 0.0);
}

// Column pass: 64 features x 64 columns per workgroup, contraction over the rows of the
// runs of one split, partial result per split (summed by k_colpass_reduce).  Wave w owns
// features 16 w .. 16 w + 15 of the tile; A^T[m][k] = A_{i0 + k, j0 + 16 w + m}.
template <int D>
__global__ __launch_bounds__(256) void k_colpass_mfma(PassGeo pg, const double* __restrict__ rho,
                                                      const double* __restrict__ Y, int K, int runs_per_split,
                                                      double* __restrict__ part) {
  __shared__ double sX[kPassRows][D + 1];     // x, rho of the run's rows
  __shared__ double sY[kPassRows][kMmCols];   // Y[i][c0 .. c0 + 63] of the run's rows
  const Geo& g = pg.g;
  const int n = g.n;
  const int j0 = blockIdx.x * 64, c0 = blockIdx.y * kMmCols, split = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int j = j0 + 16 * wave + m;            // the feature this lane computes entries for
  const bool fvalid = j < n;
  double w[D];
#pragma unroll
  for (int k = 0; k < D; ++k) w[k] = fvalid ? g.Wt[(int64_t)k * n + j] : 0.0;
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int r_begin = split * runs_per_split;
  const int r_end = min(pg.n_runs, r_begin + runs_per_split);
  for (int ri = r_begin; ri < r_end; ++ri) {
    const Chunk run = pg.runs[ri];
    __syncthreads();
    for (int e = tid; e < kPassRows * (D + 1); e += 256) {
      const int r = e / (D + 1), k = e % (D + 1);
      double v = 0.0;
      if (r < run.nrows) v = (k < D) ? g.Xt[(int64_t)k * g.P + run.row0 + r] : (rho ? rho[run.row0 + r] : 0.0);
      sX[r][k] = v;
    }
    for (int e = tid; e < kPassRows * kMmCols; e += 256) {
      const int r = e / kMmCols, c = e % kMmCols;
      sY[r][c] = (r < run.nrows && c0 + c < K) ? Y[(int64_t)(run.row0 + r) * K + c0 + c] : 0.0;
    }
    __syncthreads();
    const double amp = fvalid ? g.amp[(int64_t)run.block * n + j] : 0.0;
    const double ph = fvalid ? g.ph[(int64_t)run.block * n + j] : 0.0;
    for (int r0 = 0; r0 < run.nrows; r0 += 4) {
      const int r = r0 + kq;                    // this lane's row of the k-step (zero past nrows)
      double z = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) z = fma(w[k], sX[r][k], z);
      const double a = (r < run.nrows && fvalid) ? (amp + sX[r][D]) * sin_f64(z + ph) : 0.0;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sY[r][16 * b + m], acc[b], 0, 0, 0);
    }
  }
  // slot v: feature 16 w + 4 v + lane / 16 of the tile, column lane % 16 of block b
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int jj = j0 + 16 * wave + 4 * v + kq;
      const int c = c0 + 16 * b + m;
      if (jj < n && c < K) part[((int64_t)split * n + jj) * K + c] = acc[b][v];
    }
}

// ------------------------------------------------------------------ launchers
static int col_splits(const PassGeo& pg, int K) {
  // about 1024 workgroups (one round of waves), partial buffer bounded by ~64 n K doubles
  const int feat_per_wg = K > 16 ? kColFeat : 256 * (K <= 1 ? ColShape<1>::FPT : K <= 4 ? ColShape<4>::FPT : 1);
  const int ftiles = (pg.g.n + feat_per_wg - 1) / feat_per_wg;
  int want = (1024 + ftiles - 1) / ftiles;
  int cap = K <= 4 ? 256 : (K <= 16 ? 64 : 16);
  int s = want < cap ? want : cap;
  if (s > pg.n_runs) s = pg.n_runs;
  return s < 1 ? 1 : s;
}

// feature slices of the many-column row pass: enough workgroups (runs x column tiles x
// slices) to fill the chip, slices of at least 256 features
static int row_slices(const PassGeo& pg, int K) {
  const int base = pg.n_runs * ((K + kMmCols - 1) / kMmCols);
  int s = base > 0 ? (768 + base - 1) / base : 1;
  const int smax = (pg.g.n + 255) / 256;
  if (s > smax) s = smax;
  return s < 1 ? 1 : s;
}

size_t pass_work_elems(int n, int n_runs, int K) {
  PassGeo pg{};
  pg.g.n = n;
  pg.n_runs = n_runs;
  return (size_t)col_splits(pg, K) * n * K;
}

// Feature slices per row-pass workgroup for K columns (RowShape<KMAX>::FS).
static int row_fs(int K) { return K <= 1 ? 4 : (K <= 4 ? 2 : 1); }

// Feature groups (grid.y) of the row pass: 6144 waves in all (2048 to 16384 measured within 5%),
// but at least 8 features per wave (small systems: a few hundred rows get enough workgroups).
static int row_groups(const PassGeo& pg, int K) {
  const int fs = row_fs(K);
  const int64_t waves = (int64_t)std::max(pg.n_wide, 1) * 4;
  const int64_t want = 6144 / waves;   // about 1.5 rounds of waves at 4 per SIMD
  const int64_t cap = std::max(1, pg.g.n / (8 * fs));
  return (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(want, cap), 64));
}

size_t rowpass_work_elems(const PassGeo& pg, int K) {
  if (K > 16) return (size_t)row_slices(pg, K) * (size_t)pg.g.P * K;
  const int fg = row_groups(pg, K);
  return fg > 1 ? (size_t)2 * fg * (size_t)pg.g.P * K : 0;
}

#define FLSQ_ROW_K(DIM, KM, MD)                                                                           \
  hipLaunchKernelGGL((k_rowpass<DIM, KM, MD>), dim3(pg.n_wide, fg), dim3(256), 0, s, pg, rho, V, K, epi, \
                     work)

#define FLSQ_ROW_CASE(DIM)                                                  \
  case DIM:                                                                 \
    if (u_out) {                                                            \
      if (K <= 1) FLSQ_ROW_K(DIM, 1, 1);                                    \
      else if (K <= 4) FLSQ_ROW_K(DIM, 4, 1);                               \
      else FLSQ_ROW_K(DIM, 16, 1);                                          \
    } else {                                                                \
      if (K <= 1) FLSQ_ROW_K(DIM, 1, 0);                                    \
      else if (K <= 4) FLSQ_ROW_K(DIM, 4, 0);                               \
      else FLSQ_ROW_K(DIM, 16, 0);                                          \
    }                                                                       \
    break;

#define FLSQ_ROW_MM(DIM)                                                                                \
  case DIM:                                                                                             \
    hipLaunchKernelGGL((k_rowpass_mfma<DIM>), dim3(pg.n_runs, ctiles, slices), dim3(256), 0, s, pg, rho, V, K, \
                       fps, work);                                                                      \
    break;

hipError_t launch_rowpass_runs(const PassGeo& pg, const double* rho, const double* V, int K, const double* Y,
                               double alpha, double beta_y, double* out, hipStream_t s, double* u_out, double* work) {
  if (K > 64 || K < 1) return hipErrorInvalidValue;
  if (u_out && K > 16) return hipErrorInvalidValue;
  if (pg.n_runs == 0) return hipSuccess;
  if (K > 16) {
    if (!work) return hipErrorInvalidValue;
    const int ctiles = (K + kMmCols - 1) / kMmCols;
    const int slices = row_slices(pg, K);
    const int fps = ((pg.g.n + slices - 1) / slices + kMmFeat - 1) / kMmFeat * kMmFeat;
    switch (pg.g.d) {
      FLSQ_ROW_MM(1) FLSQ_ROW_MM(2) FLSQ_ROW_MM(3) FLSQ_ROW_MM(4)
      FLSQ_ROW_MM(5) FLSQ_ROW_MM(6) FLSQ_ROW_MM(7) FLSQ_ROW_MM(8)
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t len = pg.g.P * K;
    hipLaunchKernelGGL(k_rowpass_reduce, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, work, slices, len, Y,
                       alpha, beta_y, out);
    return hipGetLastError();
  }
  if (pg.n_wide == 0) return hipSuccess;
  const int fg = row_groups(pg, K);
  if (fg > 1 && !work) return hipErrorInvalidValue;
  RowEpi epi{Y, alpha, beta_y, out, u_out, nullptr, nullptr, 0, -1, pg.norm, 0.0};
  switch (pg.g.d) {
    FLSQ_ROW_CASE(1) FLSQ_ROW_CASE(2) FLSQ_ROW_CASE(3) FLSQ_ROW_CASE(4)
    FLSQ_ROW_CASE(5) FLSQ_ROW_CASE(6) FLSQ_ROW_CASE(7) FLSQ_ROW_CASE(8)
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || fg == 1) return e;
  const int64_t len = pg.g.P * K;
  const dim3 grid((unsigned)((len + 255) / 256));
  if (u_out)
    hipLaunchKernelGGL(k_rowpass_finish<1>, grid, dim3(256), 0, s, work, fg, pg.g.P, K, pg.g.row_block,
                       pg.even_mask, epi);
  else
    hipLaunchKernelGGL(k_rowpass_finish<0>, grid, dim3(256), 0, s, work, fg, pg.g.P, K, pg.g.row_block,
                       pg.even_mask, epi);
  return hipGetLastError();
}

#define FLSQ_COL_K(DIM, KM)                                                                               \
  hipLaunchKernelGGL((k_colpass<DIM, KM>), dim3(ftiles, splits), dim3(256), 0, s, pg, rho, Y, K, per, work)

#define FLSQ_COL_CASE(DIM)          \
  case DIM:                         \
    if (K <= 1) FLSQ_COL_K(DIM, 1); \
    else if (K <= 4) FLSQ_COL_K(DIM, 4); \
    else if (K <= 16) FLSQ_COL_K(DIM, 16); \
    else hipLaunchKernelGGL((k_colpass_mfma<DIM>), dim3((n + 63) / 64, (K + kMmCols - 1) / kMmCols, splits), \
                            dim3(256), 0, s, pg, rho, Y, K, per, work); \
    break;

hipError_t launch_colpass_runs(const PassGeo& pg, const double* rho, const double* Y, int K, const double* V,
                               double alpha, double beta_v, double* out, double* work, hipStream_t s) {
  if (K > 64 || K < 1) return hipErrorInvalidValue;
  const int n = pg.g.n;
  const int fpt = K <= 1 ? ColShape<1>::FPT : (K <= 4 ? ColShape<4>::FPT : ColShape<16>::FPT);
  const int ftiles = (n + 256 * fpt - 1) / (256 * fpt);
  const int per = (pg.n_runs + col_splits(pg, K) - 1) / col_splits(pg, K);
  const int splits = per > 0 ? (pg.n_runs + per - 1) / per : 0;   // no empty splits
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
                     splits, n, K, V, alpha, beta_v, out);
  return hipGetLastError();
}

#define FLSQ_NEWTON_CASE(DIM)                                                                           \
  case DIM:                                                                                             \
    hipLaunchKernelGGL((k_rowpass<DIM, 1, 2>), dim3(pg.n_wide, fg), dim3(256), 0, s, pg, nullptr, beta, 1, \
                       epi, work);                                                                      \
    break;

hipError_t launch_newton_residual_runs(const PassGeo& pg, const double* beta, const double* data_w,
                                       int nonlin_block, const double* poly, int n_poly, double w_nl, double norm,
                                       double* R, double* rho_out, double* u_out, double* work, hipStream_t s) {
  if (pg.n_wide == 0) return hipSuccess;
  const int fg = row_groups(pg, 1);
  if (fg > 1 && !work) return hipErrorInvalidValue;
  RowEpi epi{data_w, 1.0, 1.0, R, u_out, rho_out, poly, n_poly, nonlin_block, norm, w_nl};
  switch (pg.g.d) {
    FLSQ_NEWTON_CASE(1) FLSQ_NEWTON_CASE(2) FLSQ_NEWTON_CASE(3) FLSQ_NEWTON_CASE(4)
    FLSQ_NEWTON_CASE(5) FLSQ_NEWTON_CASE(6) FLSQ_NEWTON_CASE(7) FLSQ_NEWTON_CASE(8)
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || fg == 1) return e;
  hipLaunchKernelGGL(k_rowpass_finish<2>, dim3((unsigned)((pg.g.P + 255) / 256)), dim3(256), 0, s, work, fg, pg.g.P,
                     1, pg.g.row_block, pg.even_mask, epi);
  return hipGetLastError();
}

int pass_rows() { return kPassRows; }
int wide_rows() { return kWideRows; }

}  // namespace flsq
