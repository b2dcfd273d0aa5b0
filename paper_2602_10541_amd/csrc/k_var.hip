// Operators with row-dependent coefficients, stored explicitly in HBM.
//
//   A_ij = sum_t a_t(x_i) * (S_gtj sin z_ij + C_gtj cos z_ij),   z_ij = W_j . x_i + b_j,
//
// for row i in block g.  Channel t of block g is a constant-coefficient operator folded per
// feature exactly as Eq. (2) folds one (S, C: the sine and cosine parts of
// w * norm * sum c W^alpha Phi_|alpha|), and a_t is its per-row coefficient.  The coil-type
// operator nu Laplace + grad nu . grad is three channels; a Newton Jacobian whose nonlinearity
// involves u and its first derivatives adds the channels (identity, dN/du) and
// (d_k, dN/d(d_k u)).  The matrix is written twice, row-major (A, P x n) and transposed
// (At, n x P), so that A v, A^T y and the Gram At A all stream rows in the layout they read.
#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

// S[s][j], C[s][j] for every slot s = (block, channel): terms [off[s], off[s + 1]) of the table,
// scaled by scale[s] (block weight times the feature normalisation).
__global__ void k_fold_var(const double* __restrict__ W, int n, int d, const VarTerm* __restrict__ terms,
                           const int32_t* __restrict__ off, const double* __restrict__ scale, double* __restrict__ S,
                           double* __restrict__ C) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= n) return;
  double Sv = 0.0, Cv = 0.0;
  for (int t = off[s]; t < off[s + 1]; ++t) {
    double mono = 1.0;
    int ord = 0;
    for (int k = 0; k < d; ++k) {
      const int a = terms[t].alpha[k];
      ord += a;
      const double wk = W[(int64_t)j * d + k];
      for (int p = 0; p < a; ++p) mono *= wk;
    }
    const double v = terms[t].coef * mono;
    switch (ord & 3) {
      case 0: Sv += v; break;
      case 1: Cv += v; break;
      case 2: Sv -= v; break;
      default: Cv -= v; break;
    }
  }
  S[(int64_t)s * n + j] = Sv * scale[s];
  C[(int64_t)s * n + j] = Cv * scale[s];
}

hipError_t launch_fold_var(const double* W, int n, int d, const VarTerm* terms, const int32_t* off,
                           const double* scale, int n_slots, double* S, double* C, hipStream_t s) {
  if (n <= 0 || n_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_var, dim3((n + 255) / 256, n_slots), dim3(256), 0, s, W, n, d, terms, off, scale, S, C);
  return hipGetLastError();
}

// 64 rows x 64 features per workgroup: lane f owns feature j0 + f, wave q rows i0 + 16q ... + 15,
// so x_i, the row's block and its channel coefficients are wave-uniform.  The tile passes
// through LDS to be written transposed with unit stride along the rows.
constexpr int kVT = 64;
constexpr int kVRowsPerWave = 16;

template <int D>
__global__ __launch_bounds__(256) void k_assemble_var(VarGeo g) {
  __shared__ double tile[kVT][kVT + 1];
  const int tid = threadIdx.x, f = tid & 63, q = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * kVT;
  const int j = blockIdx.y * kVT + f;
  const bool jv = j < g.n;
  double w[D];
#pragma unroll
  for (int k = 0; k < D; ++k) w[k] = jv ? g.W[(int64_t)j * D + k] : 0.0;
  const double bj = jv ? g.b[j] : 0.0;
  for (int r = 0; r < kVRowsPerWave; ++r) {
    const int rr = q * kVRowsPerWave + r;
    const int64_t i = i0 + rr;
    double v = 0.0;
    if (i < g.P) {
      double z = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) z = fma(w[k], g.X[i * D + k], z);
      double sn, cs;
      sincos_f64(z + bj, &sn, &cs);
      const int blk = g.row_block[i];
      if (jv)
        for (int t = 0; t < g.T; ++t) {
          const double a = g.acoef[(int64_t)t * g.P + i];
          const int64_t sl = ((int64_t)blk * g.T + t) * g.n + j;
          v = fma(a, fma(g.S[sl], sn, g.C[sl] * cs), v);
        }
      if (jv) g.A[i * g.n + j] = v;
    }
    tile[rr][f] = v;
  }
  if (!g.At) return;
  __syncthreads();
  for (int e = tid; e < kVT * kVT; e += 256) {
    const int fr = e / kVT, ic = e % kVT;
    const int jj = blockIdx.y * kVT + fr;
    const int64_t ii = i0 + ic;
    if (jj < g.n && ii < g.P) g.At[(int64_t)jj * g.P + ii] = tile[ic][fr];
  }
}

hipError_t launch_assemble_var(const VarGeo& g, hipStream_t s) {
  if (g.P <= 0 || g.n <= 0) return hipSuccess;
  dim3 grid((unsigned)((g.P + kVT - 1) / kVT), (g.n + kVT - 1) / kVT);
  switch (g.d) {
#define FLSQ_AV(DIM) \
  case DIM: hipLaunchKernelGGL(k_assemble_var<DIM>, grid, dim3(256), 0, s, g); break;
    FLSQ_AV(1) FLSQ_AV(2) FLSQ_AV(3) FLSQ_AV(4) FLSQ_AV(5) FLSQ_AV(6) FLSQ_AV(7) FLSQ_AV(8)
#undef FLSQ_AV
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// out[r] = beta_y * Y[r] + alpha * sum_c M[r][c] v[c] (Y nullable): one wave per row, lanes
// striding the row, a fixed butterfly order for the lane sums.
__global__ __launch_bounds__(256) void k_rowdot(const double* __restrict__ M, int64_t R, int64_t len, int64_t ld,
                                                const double* __restrict__ v, const double* __restrict__ Y,
                                                double alpha, double beta_y, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= R) return;
  const double* row = M + r * ld;
  double acc = 0.0;
  for (int64_t c = lane; c < len; c += 64) acc = fma(row[c], v[c], acc);
  for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if (lane == 0) out[r] = (Y ? beta_y * Y[r] : 0.0) + alpha * acc;
}

hipError_t launch_rowdot(const double* M, int64_t R, int64_t len, int64_t ld, const double* v, const double* Y,
                         double alpha, double beta_y, double* out, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rowdot, dim3((unsigned)((R + 3) / 4)), dim3(256), 0, s, M, R, len, ld, v, Y, alpha, beta_y,
                     out);
  return hipGetLastError();
}

// At (cols x rows) = A^T for a row-major rows x cols matrix: 32 x 32 tiles through LDS, both
// the reads and the writes with unit stride.
__global__ __launch_bounds__(256) void k_transpose_f64(const double* __restrict__ A, int64_t rows, int cols,
                                                       double* __restrict__ At) {
  __shared__ double t[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = r0 + k;
    const int c = c0 + tx;
    if (r < rows && c < cols) t[k][tx] = A[r * cols + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k;
    const int64_t r = r0 + tx;
    if (r < rows && c < cols) At[(int64_t)c * rows + r] = t[tx][k];
  }
}

hipError_t launch_transpose_f64(const double* A, int64_t rows, int cols, double* At, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_f64, dim3((unsigned)((rows + 31) / 32), (cols + 31) / 32), dim3(256), 0, s, A, rows,
                     cols, At);
  return hipGetLastError();
}

// A_ij += rho_i sin(z_ij + ph_gj) on the rows with rho_i != 0: the Newton row coefficient of
// the folded entry (amp_gj + rho_i) sin(z_ij + ph_gj) added to an explicit assembly of the
// linear rows (z as an FMA chain from zero in k order, as everywhere).  16 rows per workgroup
// row, 256 features per workgroup column.
__global__ __launch_bounds__(256) void k_add_rho(Geo g, const double* __restrict__ rho, double* __restrict__ A) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= g.n) return;
  for (int r = 0; r < 16; ++r) {
    const int64_t i = (int64_t)blockIdx.y * 16 + r;
    if (i >= g.P) return;
    const double rh = rho[i];
    if (rh == 0.0) continue;
    double z = 0.0;
    for (int k = 0; k < g.d; ++k) z = fma(g.Wt[(int64_t)k * g.n + j], g.Xrm[i * g.d + k], z);
    const int blk = g.row_block[i];
    A[i * g.n + j] = fma(rh, sin_f64(z + g.ph[(int64_t)blk * g.n + j]), A[i * g.n + j]);
  }
}

hipError_t launch_add_rho(const Geo& g, const double* rho, double* A, hipStream_t s) {
  if (g.P <= 0 || g.n <= 0) return hipSuccess;
  if ((g.P + 15) / 16 > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_add_rho, dim3((g.n + 255) / 256, (unsigned)((g.P + 15) / 16)), dim3(256), 0, s, g, rho, A);
  return hipGetLastError();
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Nonlinearity N(u, grad u) = sum_k poly_k u^k + e exp(u) + sum_t c_t u^{m_t} d_{axis_t} u on the rows
// [row0, row0 + rows) of the nonlinear block (weight w).  U holds u at every row of the system
// (first P entries) and then d_{slot axis} u on the block's rows, slot by slot.
//   R[row0 + i] += w N                (R nullable)
//   rho[i]       = dN/du              (rho nullable; row stride 1)
//   kap[s][i]    = dN/d(d_{axis_s} u) (kap nullable; slot stride kap_ld)
// The Jacobian channels that take rho and kap as row coefficients carry the block weight.
__global__ void k_nl_var(NlSpec nl, const double* __restrict__ U, int64_t P, int64_t row0, int64_t rows, double w,
                         double* R, double* rho, double* kap, int64_t kap_ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const double u = U[row0 + i];
  double val = 0.0, dval = 0.0, upow = 1.0;
  for (int k = 0; k < nl.n_poly; ++k) {
    val = fma(nl.poly[k], upow, val);
    if (k + 1 < nl.n_poly) dval = fma((double)(k + 1) * nl.poly[k + 1], upow, dval);
    upow *= u;
  }
  if (nl.exp_coef != 0.0) {
    const double eu = nl.exp_coef * exp(u);
    val += eu;
    dval += eu;
  }
  double dg[kMaxNlTerms];
  for (int s = 0; s < nl.n_slots; ++s) dg[s] = 0.0;
  for (int t = 0; t < nl.n_adv; ++t) {
    const int s = nl.slot[t];
    const double g = U[P + (int64_t)s * rows + i];
    double um = 1.0, um1 = 0.0;   // u^m and m u^(m-1)
    for (int p = 0; p < nl.m[t]; ++p) {
      um1 = fma(um1, u, um);
      um *= u;
    }
    val = fma(nl.c[t] * um, g, val);
    dval = fma(nl.c[t] * um1, g, dval);
    dg[s] = fma(nl.c[t], um, dg[s]);
  }
  if (R) R[row0 + i] = fma(w, val, R[row0 + i]);
  if (rho) rho[i] = dval;
  if (kap)
    for (int s = 0; s < nl.n_slots; ++s) kap[(int64_t)s * kap_ld + i] = dg[s];
}

hipError_t launch_nl_var(const NlSpec& nl, const double* U, int64_t P, int64_t row0, int64_t rows, double w,
                         double* R, double* rho, double* kap, int64_t kap_ld, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nl_var, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, nl, U, P, row0, rows, w, R,
                     rho, kap, kap_ld);
  return hipGetLastError();
}

}  // namespace flsq
