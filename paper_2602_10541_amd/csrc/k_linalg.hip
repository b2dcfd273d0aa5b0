// Dense FP64 linear algebra for the regularised normal equations (A^T A + mu I) beta = A^T rhs.
//
// G is stored row-major and only its upper triangle is used.  The factor is upper
// triangular, G = U^T U, computed in place by a blocked right-looking Cholesky with
// block size kNb = 64:
//   1. factor the diagonal block and invert it  (one workgroup, in LDS)
//   2. block row: U_kj = U_kk^{-T} G_kj = X_kk^T G_kj   (batched MFMA GEMM, k_dense.hip)
//   3. trailing update G_ij -= U_ki^T U_kj       (FP64 MFMA 16x16x4, 64 x 64 tiles, i <= j)
// The off-diagonal blocks of X = U^{-1} are assembled afterwards level by level
// (X_12 = -X_11 U_12 X_22) with the same GEMM.
#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

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

// Block row: for each column j >= k0 + kNb solve U_kk^T y = g by forward substitution
// (backward stable, unlike multiplying by the explicit inverse of U_kk).  One column per
// thread, 64-thread workgroups so the (n - k1) columns spread over many CUs.  The
// triangle U_kk is read through its own read-only pointer: every address is wave-uniform,
// so its values arrive in scalar registers in wide batches instead of one LDS round trip
// per multiply-add.  The kernel writes only columns >= k1 of the block row, never U_kk.
__global__ __launch_bounds__(64) void k_trsm_row(double* __restrict__ Grow, const double* __restrict__ Ukk, int n,
                                                 int jend) {
  const int j = kNb + blockIdx.x * 64 + threadIdx.x;     // column offset from k0
  if (j >= jend) return;
  double y[kNb];
#pragma unroll
  for (int l = 0; l < kNb; ++l) y[l] = Grow[(int64_t)l * n + j];
#pragma unroll
  for (int l = 0; l < kNb; ++l) {
    y[l] = y[l] / Ukk[(int64_t)l * n + l];
#pragma unroll
    for (int m = l + 1; m < kNb; ++m) y[m] = fma(-Ukk[(int64_t)l * n + m], y[l], y[m]);
  }
#pragma unroll
  for (int l = 0; l < kNb; ++l) Grow[(int64_t)l * n + j] = y[l];
}

hipError_t launch_trsm_row(double* G, int n, int k0, hipStream_t s) {
  const int cols = n - k0 - kNb;
  if (cols <= 0) return hipSuccess;
  double* base = G + (int64_t)k0 * n + k0;
  // columns are addressed relative to k0; the valid range is j < n - k0
  hipLaunchKernelGGL(k_trsm_row, dim3((cols + 63) / 64), dim3(64), 0, s, base, (const double*)base, n, n - k0);
  return hipGetLastError();
}

// ------------------------------------------------------------------ equilibration
// d_i = 1 / sqrt(G_ii) (1 where G_ii <= 0); used to scale G to unit diagonal before the
// factorisation, and the inverse factor back: M^{-1} = (D X)(D X)^T.
__global__ void k_diag_rsqrt(const double* G, int n, double* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double g = G[(int64_t)i * n + i];
  d[i] = (g > 0.0) ? 1.0 / sqrt(g) : 1.0;
}

// dst_ij = d_i src_ij d_j on the upper triangle, plus diag_add + mu d_i^2 on the diagonal.
__global__ void k_scale_upper(const double* src, double* dst, int n, const double* d, double mu, double diag_add) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n || j < i) return;
  const int64_t o = (int64_t)i * n + j;
  double v = d[i] * src[o] * d[j];
  if (i == j) v += diag_add + mu * d[i] * d[i];
  dst[o] = v;
}

__global__ void k_scale_rows(double* X, int n, const double* d) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j < n) X[(int64_t)i * n + j] *= d[i];
}

hipError_t launch_equilibrate(const double* G, double* dst, int n, double* d, double mu, double diag_add,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_diag_rsqrt, dim3((n + 255) / 256), dim3(256), 0, s, G, n, d);
  hipLaunchKernelGGL(k_scale_upper, dim3((n + 255) / 256, n), dim3(256), 0, s, G, dst, n, d, mu, diag_add);
  return hipGetLastError();
}

hipError_t launch_scale_rows(double* X, int n, const double* d, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rows, dim3((n + 255) / 256, n), dim3(256), 0, s, X, n, d);
  return hipGetLastError();
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

__global__ void k_select_cols(const double* src, double* dst, int64_t n, int K, const double* mask) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * K) return;
  if (mask[e % K] != 0.0) dst[e] = src[e];
}

hipError_t launch_select_cols(const double* src, double* dst, int64_t n, int K, const double* mask, hipStream_t s) {
  const int64_t tot = n * K;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_select_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, dst, n, K, mask);
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
