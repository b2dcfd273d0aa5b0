// Dense FP64 linear algebra for the regularised normal equations (A^T A + mu I) beta = A^T rhs.
//
// G is stored row-major and only its upper triangle is used.  The factor is upper
// triangular, G = U^T U, computed in place by a blocked right-looking Cholesky with
// block size kNb = 64:
//   1. factor the diagonal block              (one workgroup, in LDS)
//   2. block row: U_kj = U_kk^{-T} G_kj       (one thread per column; coalesced rows)
//   3. trailing update G_ij -= U_ki^T U_kj     (FP64 MFMA 16x16x4, 64 x 64 tiles, i <= j)
// Triangular solves run one block step per launch; every workgroup solves the small
// diagonal system redundantly in a wave (no inter-workgroup communication) and updates
// its share of the remaining right-hand side.
#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

// ------------------------------------------------------------------ Cholesky
__global__ __launch_bounds__(256) void k_potrf_diag(double* G, int n, int k0, int* info) {
  __shared__ double a[kNb][kNb + 1];
  const int nbk = min(kNb, n - k0);
  const int tid = threadIdx.x;
  for (int e = tid; e < nbk * nbk; e += 256) {
    const int i = e / nbk, j = e % nbk;
    a[i][j] = (j >= i) ? G[(int64_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  for (int l = 0; l < nbk; ++l) {
    double piv = a[l][l];
    if (!(piv > 0.0) || !isfinite(piv)) {   // not positive definite (or NaN): record, keep going
      if (tid == 0 && *info == 0) *info = k0 + l + 1;
      piv = 1.0;
    }
    const double dl = sqrt(piv);
    __syncthreads();
    if (tid == 0) a[l][l] = dl;
    for (int j = l + 1 + tid; j < nbk; j += 256) a[l][j] /= dl;
    __syncthreads();
    const int cnt = nbk - l - 1;
    for (int e = tid; e < cnt * cnt; e += 256) {
      const int i = l + 1 + e / cnt, j = l + 1 + e % cnt;
      if (j >= i) a[i][j] -= a[l][i] * a[l][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < nbk * nbk; e += 256) {
    const int i = e / nbk, j = e % nbk;
    if (j >= i) G[(int64_t)(k0 + i) * n + k0 + j] = a[i][j];
  }
}

hipError_t launch_potrf_diag(double* G, int n, int k0, int* info, double shift, hipStream_t s) {
  (void)shift;
  hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, G, n, k0, info);
  return hipGetLastError();
}

// Block row: for each column j >= k0 + kNb solve U_kk^T y = g (forward substitution).
__global__ __launch_bounds__(256) void k_trsm_row(double* G, int n, int k0) {
  __shared__ double u[kNb][kNb + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < kNb * kNb; e += 256) {
    const int i = e / kNb, j = e % kNb;
    u[i][j] = (j >= i) ? G[(int64_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  const int j = k0 + kNb + blockIdx.x * 256 + tid;
  if (j >= n) return;
  double y[kNb];
#pragma unroll
  for (int l = 0; l < kNb; ++l) y[l] = G[(int64_t)(k0 + l) * n + j];
#pragma unroll
  for (int l = 0; l < kNb; ++l) {
    y[l] /= u[l][l];
#pragma unroll
    for (int m = l + 1; m < kNb; ++m) y[m] = fma(-u[l][m], y[l], y[m]);
  }
#pragma unroll
  for (int l = 0; l < kNb; ++l) G[(int64_t)(k0 + l) * n + j] = y[l];
}

hipError_t launch_trsm_row(double* G, int n, int k0, hipStream_t s) {
  const int cols = n - k0 - kNb;
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm_row, dim3((cols + 255) / 256), dim3(256), 0, s, G, n, k0);
  return hipGetLastError();
}

__device__ __forceinline__ void tri_coords(int t, int nt, int* ti, int* tj) {
  int r = 0, rowlen = nt;
  while (t >= rowlen) {
    t -= rowlen;
    ++r;
    --rowlen;
  }
  *ti = r;
  *tj = r + t;
}

// Trailing update of the upper triangle: G[i][j] -= sum_l U[k0+l][i] U[k0+l][j], k1 <= i <= j.
__global__ __launch_bounds__(256) void k_syrk(double* G, int n, int k0) {
  __shared__ double pI[kNb][64 + 1];
  __shared__ double pJ[kNb][64 + 1];
  const int k1 = k0 + kNb;
  const int nt = (n - k1 + 63) / 64;
  int ti, tj;
  tri_coords(blockIdx.x, nt, &ti, &tj);
  const int i0 = k1 + ti * 64, j0 = k1 + tj * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < kNb * 64; e += 256) {
    const int l = e / 64, c = e % 64;
    const int64_t row = (int64_t)(k0 + l) * n;
    pI[l][c] = (i0 + c < n) ? G[row + i0 + c] : 0.0;
    pJ[l][c] = (j0 + c < n) ? G[row + j0 + c] : 0.0;
  }
  __syncthreads();
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // wave w owns output block-row w (16 rows), four 16-column blocks
#pragma unroll
  for (int kk = 0; kk < kNb / 4; ++kk) {
    const int l = kk * 4 + (lane >> 4);
    const double av = pI[l][wave * 16 + (lane & 15)];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double bv = pJ[l][b * 16 + (lane & 15)];
      acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + wave * 16 + 4 * v + (lane >> 4);
      const int j = j0 + b * 16 + (lane & 15);
      if (i < n && j < n && j >= i) G[(int64_t)i * n + j] -= acc[b][v];
    }
}

hipError_t launch_syrk(double* G, int n, int k0, hipStream_t s) {
  const int rem = n - k0 - kNb;
  if (rem <= 0) return hipSuccess;
  const int nt = (rem + 63) / 64;
  hipLaunchKernelGGL(k_syrk, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, G, n, k0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ triangular solves
// Diagonal-block solve inside one workgroup: each wave takes right-hand-side columns
// c = wave, wave + 4, ...; lane m holds entry m of the block.  Result into x[m][c] (LDS).
template <bool kForward>
__device__ __forceinline__ void diag_solve(const double (*u)[kNb + 1], int nbk, const double* Y, int n_ld, int k0,
                                           int K, double (*x)[65]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < K; c += 4) {
    double y = (lane < nbk) ? Y[(int64_t)(k0 + lane) * K + c] : 0.0;
    if (kForward) {
      for (int l = 0; l < nbk; ++l) {
        const double xl = __shfl(y, l) / u[l][l];
        if (lane == l) y = xl;
        if (lane > l) y = fma(-u[l][lane], xl, y);
      }
    } else {
      for (int l = nbk - 1; l >= 0; --l) {
        const double xl = __shfl(y, l) / u[l][l];
        if (lane == l) y = xl;
        if (lane < l) y = fma(-u[lane][l], xl, y);
      }
    }
    if (lane < nbk) x[lane][c] = y;
  }
  (void)n_ld;
}

// Forward step k (U^T X = Y): X[k] = U_kk^{-T} Y[k]; Y[j] -= U[k-rows][j]^T X[k] for j >= k1.
__global__ __launch_bounds__(256) void k_trsv_fwd(const double* U, int n, int k0, double* Y, double* X, int K) {
  __shared__ double u[kNb][kNb + 1];
  __shared__ double x[kNb][65];
  const int nbk = min(kNb, n - k0);
  const int tid = threadIdx.x;
  for (int e = tid; e < nbk * nbk; e += 256) {
    const int i = e / nbk, j = e % nbk;
    u[i][j] = (j >= i) ? U[(int64_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  diag_solve<true>(u, nbk, Y, n, k0, K, x);
  __syncthreads();
  if (blockIdx.x == 0)
    for (int e = tid; e < nbk * K; e += 256) X[(int64_t)(k0 + e / K) * K + e % K] = x[e / K][e % K];
  const int j = k0 + nbk + blockIdx.x * 256 + tid;
  if (j >= n) return;
  for (int c = 0; c < K; ++c) {
    double s = 0.0;
    for (int l = 0; l < nbk; ++l) s = fma(U[(int64_t)(k0 + l) * n + j], x[l][c], s);
    Y[(int64_t)j * K + c] -= s;
  }
}

// Backward step k (U X = Y): X[k] = U_kk^{-1} Y[k]; Y[i] -= U[i][k-cols] X[k] for i < k0.
__global__ __launch_bounds__(256) void k_trsv_bwd(const double* U, int n, int k0, double* Y, double* X, int K) {
  __shared__ double u[kNb][kNb + 1];
  __shared__ double x[kNb][65];
  __shared__ double r[64][kNb + 1];
  const int nbk = min(kNb, n - k0);
  const int tid = threadIdx.x;
  for (int e = tid; e < nbk * nbk; e += 256) {
    const int i = e / nbk, j = e % nbk;
    u[i][j] = (j >= i) ? U[(int64_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  diag_solve<false>(u, nbk, Y, n, k0, K, x);
  __syncthreads();
  if (blockIdx.x == 0)
    for (int e = tid; e < nbk * K; e += 256) X[(int64_t)(k0 + e / K) * K + e % K] = x[e / K][e % K];
  // rows i in [64 * (blockIdx.x - 0), ...) below k0: stage U[i][k0 .. k0 + nbk) through LDS
  const int i0 = blockIdx.x * 64;
  if (i0 >= k0) return;
  for (int e = tid; e < 64 * nbk; e += 256) {
    const int ii = e / nbk, l = e % nbk;
    r[ii][l] = (i0 + ii < k0) ? U[(int64_t)(i0 + ii) * n + k0 + l] : 0.0;
  }
  __syncthreads();
  const int ii = tid & 63, cg = tid >> 6;
  if (i0 + ii >= k0) return;
  for (int c = cg; c < K; c += 4) {
    double s = 0.0;
    for (int l = 0; l < nbk; ++l) s = fma(r[ii][l], x[l][c], s);
    Y[(int64_t)(i0 + ii) * K + c] -= s;
  }
}

// Full solves with the factor: Y (n x K) is consumed as scratch, the solution goes to X.
hipError_t launch_trsv_fwd(const double* U, int n, double* Y, double* X, int K, hipStream_t s) {
  for (int k0 = 0; k0 < n; k0 += kNb) {
    const int rem = n - k0 - kNb;
    const int grid = rem > 0 ? (rem + 255) / 256 : 1;
    hipLaunchKernelGGL(k_trsv_fwd, dim3(grid), dim3(256), 0, s, U, n, k0, Y, X, K);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_trsv_bwd(const double* U, int n, double* Y, double* X, int K, hipStream_t s) {
  const int last = ((n - 1) / kNb) * kNb;
  for (int k0 = last; k0 >= 0; k0 -= kNb) {
    const int grid = k0 > 0 ? (k0 + 63) / 64 : 1;
    hipLaunchKernelGGL(k_trsv_bwd, dim3(grid), dim3(256), 0, s, U, n, k0, Y, X, K);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ helpers
__global__ void k_copy_upper(const double* src, double* dst, int n, double diag_add) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n || j < i) return;
  const int64_t o = (int64_t)i * n + j;
  dst[o] = src[o] + ((i == j) ? diag_add : 0.0);
}

hipError_t launch_copy_upper(const double* src, double* dst, int n, double diag_add, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_upper, dim3((n + 255) / 256, n), dim3(256), 0, s, src, dst, n, diag_add);
  return hipGetLastError();
}

__global__ void k_diag_max(const double* G, int n, double* out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, G[(int64_t)i * n + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_diag_max(const double* G, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_max, dim3(1), dim3(256), 0, s, G, n, out);
  return hipGetLastError();
}

// Column dot products sum_i x[i][c] y[i][c]: stage 1 writes one partial per workgroup
// and column, stage 2 sums the partials in order (deterministic).
constexpr int kDotWg = 256;
constexpr int kDotBlocks = 512;

__global__ void k_dot_stage1(const double* x, const double* y, int64_t n, int K, double* work) {
  __shared__ double red[256];
  for (int c = 0; c < K; ++c) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kDotWg + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDotWg)
      s = fma(x[i * K + c], y[i * K + c], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) work[(int64_t)c * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ void k_dot_stage2(const double* work, int nblk, int K, double* out) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += work[(int64_t)c * nblk + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

hipError_t launch_dot_cols(const double* x, const double* y, int64_t n, int K, double* out, double* work,
                           hipStream_t s) {
  int64_t nb = (n + kDotWg - 1) / kDotWg;
  const int nblk = (int)(nb < kDotBlocks ? (nb > 0 ? nb : 1) : kDotBlocks);
  hipLaunchKernelGGL(k_dot_stage1, dim3(nblk), dim3(kDotWg), 0, s, x, y, n, K, work);
  hipLaunchKernelGGL(k_dot_stage2, dim3(K), dim3(256), 0, s, work, nblk, K, out);
  return hipGetLastError();
}

__global__ void k_axpy_cols(const double* a, const double* x, double* y, int64_t n, int K, double sign) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * K) return;
  y[e] = fma(sign * a[e % K], x[e], y[e]);
}

hipError_t launch_axpy_cols(const double* a, const double* x, double* y, int64_t n, int K, double sign,
                            hipStream_t s) {
  const int64_t tot = n * K;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a, x, y, n, K, sign);
  return hipGetLastError();
}

__global__ void k_xpby_cols(const double* z, const double* b, double* p, int64_t n, int K) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * K) return;
  p[e] = fma(b[e % K], p[e], z[e]);
}

hipError_t launch_xpby_cols(const double* z, const double* b, double* p, int64_t n, int K, hipStream_t s) {
  const int64_t tot = n * K;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_xpby_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, z, b, p, n, K);
  return hipGetLastError();
}

__global__ void k_nonfinite(const double* x, int64_t n, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) atomicOr(flag, 1);
}

hipError_t launch_count_nonfinite(const double* x, int64_t n, int* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

}  // namespace flsq
