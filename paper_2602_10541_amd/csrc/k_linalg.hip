// Dense FP64 helpers around the Cholesky factor of the regularised normal equations
// (A^T A + mu I) beta = A^T rhs: diagonal equilibration, copies, norms, and the small
// column-wise vector kernels of the CGLS / PCG iterations.  The factorisation itself is
// in k_chol.hip, the products with the explicit inverse factor in k_dense.hip.
#include <algorithm>

#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

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

hipError_t launch_equilibrate(const double* G, double* dst, int n, double* d, double mu, double diag_add,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_diag_rsqrt, dim3((n + 255) / 256), dim3(256), 0, s, G, n, d);
  hipLaunchKernelGGL(k_scale_upper, dim3((n + 255) / 256, n), dim3(256), 0, s, G, dst, n, d, mu, diag_add);
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
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_diag_max(const double* G, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_max, dim3(1), dim3(256), 0, s, G, n, out);
  return hipGetLastError();
}

// 64-bit fingerprint of the upper triangle of G (n x n row-major): the sum, modulo 2^64, of a
// mix (the splitmix64 finaliser) of each entry's bit pattern and its position.  Integer sums
// do not depend on their order, so the value is reproducible; stage 1 writes one partial per
// row (a workgroup per row), stage 2 sums them.
__device__ __forceinline__ unsigned long long fp_mix(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_fingerprint_rows(const double* G, int n, unsigned long long* part) {
  __shared__ unsigned long long red[256];
  const int i = blockIdx.x;
  unsigned long long h = 0;
  for (int j = i + (int)threadIdx.x; j < n; j += 256) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(G[(int64_t)i * n + j]);
    h += fp_mix(bits ^ ((unsigned long long)i << 32 | (unsigned)j));
  }
  red[threadIdx.x] = h;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[i] = red[0];
}

__global__ __launch_bounds__(256) void k_fingerprint_sum(const unsigned long long* part, int n,
                                                         unsigned long long* out) {
  __shared__ unsigned long long red[256];
  unsigned long long h = 0;
  for (int i = threadIdx.x; i < n; i += 256) h += part[i];
  red[threadIdx.x] = h;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_fingerprint_upper(const double* G, int n, unsigned long long* part, unsigned long long* out,
                                    hipStream_t s) {
  if (n <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fingerprint_rows, dim3(n), dim3(256), 0, s, G, n, part);
  hipLaunchKernelGGL(k_fingerprint_sum, dim3(1), dim3(256), 0, s, part, n, out);
  return hipGetLastError();
}

// Column dot products sum_i x[i][c] y[i][c]: stage 1 writes one partial per workgroup
// and column, stage 2 sums the partials in order (deterministic).
constexpr int kDotWg = 256;
constexpr int kDotBlocks = 512;

// Stage 1 of out[c] = sum_i x[i][c] y[i][c]: for columns in chunks of up to 256, thread t of
// a workgroup owns column c = t % kc and walks rows t / kc, t / kc + R, ... (R = 256 / kc rows
// per step, so a step reads R whole rows, coalesced); the R partial sums of a column are
// added in a fixed order.
__global__ __launch_bounds__(kDotWg) void k_dot_stage1(const double* __restrict__ x, const double* __restrict__ y,
                                                       int64_t n, int K, double* __restrict__ work) {
  __shared__ double red[kDotWg];
  const int t = threadIdx.x;
  for (int cb = 0; cb < K; cb += kDotWg) {
    const int kc = min(kDotWg, K - cb);
    const int R = kDotWg / kc;
    const int c = t % kc, r = t / kc;
    double s = 0.0;
    if (r < R)
      for (int64_t i = (int64_t)blockIdx.x * R + r; i < n; i += (int64_t)gridDim.x * R)
        s = fma(x[i * K + cb + c], y[i * K + cb + c], s);
    red[t] = s;
    __syncthreads();
    if (t < kc) {
      double acc = 0.0;
      for (int rr = 0; rr < R; ++rr) acc += red[rr * kc + t];
      work[(int64_t)(cb + t) * gridDim.x + blockIdx.x] = acc;
    }
    __syncthreads();
  }
}

// Weighted column sums: work[c][blk] = partial sums over the rows of sum_i u_i s_i Y[i][c], with
// s_i = X[i * ldx + xcol] (or 1 without X); same column-chunked layout as k_dot_stage1.
__global__ __launch_bounds__(kDotWg) void k_wsum_stage1(const double* __restrict__ Y, int64_t n, int K,
                                                        const double* __restrict__ u, const double* __restrict__ X,
                                                        int ldx, int xcol, double* __restrict__ work) {
  __shared__ double red[kDotWg];
  const int t = threadIdx.x;
  for (int cb = 0; cb < K; cb += kDotWg) {
    const int kc = min(kDotWg, K - cb);
    const int R = kDotWg / kc;
    const int c = t % kc, r = t / kc;
    double s = 0.0;
    if (r < R)
      for (int64_t i = (int64_t)blockIdx.x * R + r; i < n; i += (int64_t)gridDim.x * R) {
        const double w = X ? u[i] * X[i * ldx + xcol] : u[i];
        s = fma(w, Y[i * K + cb + c], s);
      }
    red[t] = s;
    __syncthreads();
    if (t < kc) {
      double acc = 0.0;
      for (int rr = 0; rr < R; ++rr) acc += red[rr * kc + t];
      work[(int64_t)(cb + t) * gridDim.x + blockIdx.x] = acc;
    }
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
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// Small products (n K <= kDotSmallMax): one 1024-thread workgroup per product writes the column
// sums directly.  Thread t owns column c = t % kc of a chunk of kc columns and walks rows
// t / kc, t / kc + R, ... with R the largest power of two with R kc <= 1024; the R partials of a
// column are then added pairwise in a fixed tree.  Several products go in one launch.
constexpr int kDotSmallWg = 1024;
constexpr int64_t kDotSmallMax = 32768;

__global__ __launch_bounds__(kDotSmallWg) void k_dot_small(DotBatch b) {
  __shared__ double red[kDotSmallWg];
  const int pi = blockIdx.x;
  const double* __restrict__ x = b.x[pi];
  const double* __restrict__ y = b.y[pi];
  const int64_t n = b.n[pi];
  const int K = b.K;
  const int t = threadIdx.x;
  for (int cb = 0; cb < K; cb += kDotSmallWg) {
    const int kc = min(kDotSmallWg, K - cb);
    int R = 1;
    while (R * 2 * kc <= kDotSmallWg) R *= 2;
    const int c = t % kc, r = t / kc;
    double s = 0.0;
    if (r < R)
      for (int64_t i = r; i < n; i += R) s = fma(x[i * K + cb + c], y[i * K + cb + c], s);
    red[t] = s;
    __syncthreads();
    for (int h = R / 2; h > 0; h >>= 1) {
      if (r < h) red[r * kc + c] += red[(r + h) * kc + c];
      __syncthreads();
    }
    if (t < kc) b.out[pi][cb + t] = red[t];
    __syncthreads();
  }
}

// Large products of a batch in one pair of launches: product p = blockIdx.y, its partials in
// work[p][c][blk] (the kDotBlocks x K doubles of one product's work are shared out among the
// batch), then summed per column as in k_dot_stage2.
__global__ __launch_bounds__(kDotWg) void k_dot_stage1_batch(DotBatch b, int nblk, double* __restrict__ work) {
  __shared__ double red[kDotWg];
  const int p = blockIdx.y;
  const double* __restrict__ x = b.x[p];
  const double* __restrict__ y = b.y[p];
  const int64_t n = b.n[p];
  const int K = b.K;
  double* w = work + (int64_t)p * K * nblk;
  const int t = threadIdx.x;
  for (int cb = 0; cb < K; cb += kDotWg) {
    const int kc = min(kDotWg, K - cb);
    const int R = kDotWg / kc;
    const int c = t % kc, r = t / kc;
    double s = 0.0;
    if (r < R)
      for (int64_t i = (int64_t)blockIdx.x * R + r; i < n; i += (int64_t)nblk * R)
        s = fma(x[i * K + cb + c], y[i * K + cb + c], s);
    red[t] = s;
    __syncthreads();
    if (t < kc) {
      double acc = 0.0;
      for (int rr = 0; rr < R; ++rr) acc += red[rr * kc + t];
      w[(int64_t)(cb + t) * nblk + blockIdx.x] = acc;
    }
    __syncthreads();
  }
}

__global__ void k_dot_stage2_batch(DotBatch b, int nblk, const double* __restrict__ work) {
  __shared__ double red[256];
  const int c = blockIdx.x, p = blockIdx.y;
  const double* w = work + ((int64_t)p * b.K + c) * nblk;
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) s += w[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) b.out[p][c] = red[0];
}

hipError_t launch_dot_batch(const DotBatch& b, double* work, hipStream_t s) {
  if (b.count < 1 || b.count > kDotBatchMax || b.K < 1) return hipErrorInvalidValue;
  bool small = true;
  int64_t nmax = 0;
  for (int p = 0; p < b.count; ++p) {
    small = small && b.n[p] * b.K <= kDotSmallMax;
    nmax = std::max(nmax, b.n[p] * b.K);
  }
  if (small) {
    hipLaunchKernelGGL(k_dot_small, dim3(b.count), dim3(kDotSmallWg), 0, s, b);
    return hipGetLastError();
  }
  if (b.count == 1) return launch_dot_cols(b.x[0], b.y[0], b.n[0], b.K, b.out[0], work, s);
  // the work of one product (kDotBlocks x K doubles) holds every product's partials
  const int64_t nb = (nmax + kDotWg - 1) / kDotWg;
  const int cap = kDotBlocks / b.count;
  const int nblk = (int)(nb < cap ? (nb > 0 ? nb : 1) : cap);
  hipLaunchKernelGGL(k_dot_stage1_batch, dim3(nblk, b.count), dim3(kDotWg), 0, s, b, nblk, work);
  hipLaunchKernelGGL(k_dot_stage2_batch, dim3(b.K, b.count), dim3(256), 0, s, b, nblk, work);
  return hipGetLastError();
}

hipError_t launch_dot_cols(const double* x, const double* y, int64_t n, int K, double* out, double* work,
                           hipStream_t s) {
  if (n * K <= kDotSmallMax && K >= 1) {
    DotBatch b{};
    b.x[0] = x;
    b.y[0] = y;
    b.n[0] = n;
    b.out[0] = out;
    b.count = 1;
    b.K = K;
    hipLaunchKernelGGL(k_dot_small, dim3(1), dim3(kDotSmallWg), 0, s, b);
    return hipGetLastError();
  }
  const int64_t nb = (n * K + kDotWg - 1) / kDotWg;   // one step of a workgroup reads kDotWg entries
  const int nblk = (int)(nb < kDotBlocks ? (nb > 0 ? nb : 1) : kDotBlocks);
  hipLaunchKernelGGL(k_dot_stage1, dim3(nblk), dim3(kDotWg), 0, s, x, y, n, K, work);
  hipLaunchKernelGGL(k_dot_stage2, dim3(K), dim3(256), 0, s, work, nblk, K, out);
  return hipGetLastError();
}

hipError_t launch_wsum_cols(const double* Y, int64_t n, int K, const double* u, const double* X, int ldx, int xcol,
                           double* out, double* work, hipStream_t s) {
  const int64_t nb = (n * K + kDotWg - 1) / kDotWg;
  const int nblk = (int)(nb < kDotBlocks ? (nb > 0 ? nb : 1) : kDotBlocks);
  hipLaunchKernelGGL(k_wsum_stage1, dim3(nblk), dim3(kDotWg), 0, s, Y, n, K, u, X, ldx, xcol, work);
  hipLaunchKernelGGL(k_dot_stage2, dim3(K), dim3(256), 0, s, work, nblk, K, out);
  return hipGetLastError();
}

__global__ void k_axpy_cols(ColScalars a, const double* x, double* y, int64_t n, int K, double sign) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * K) return;
  y[e] = fma(sign * a.v[e % K], x[e], y[e]);
}

hipError_t launch_axpy_cols(const ColScalars& a, const double* x, double* y, int64_t n, int K, double sign,
                            hipStream_t s) {
  const int64_t tot = n * K;
  if (tot == 0) return hipSuccess;
  if (K < 1 || K > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_axpy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a, x, y, n, K, sign);
  return hipGetLastError();
}

// CG steps with their scalars kept on the device (the host reads them once per iteration for
// its stopping decisions instead of round-tripping each one).  The step length of column k:
// alpha_k = gam_k / (d1_k + mu d2_k) for active columns with both positive, else 0 (d2 nullable).
__device__ __forceinline__ double cg_alpha_of(int k, const double* gam, const double* d1, const double* d2, double mu,
                                              uint64_t active) {
  const double dl = d1[k] + (d2 ? mu * d2[k] : 0.0);
  return (((active >> k) & 1ull) && dl > 0.0 && gam[k] > 0.0) ? gam[k] / dl : 0.0;
}

// y_q += sign_q alpha_c x_q (grid.y = q) with alpha from the device dots; alpha_out receives the
// step lengths for the host.  With keep given, the columns
// of y_0 selected by keep_mask are first copied to keep: the best-iterate copy the host decided
// after the previous step, taken before this step changes y_0.
__global__ void k_cg_step(const double* __restrict__ gam, const double* __restrict__ d1, const double* d2, double mu,
                          uint64_t active, double* __restrict__ alpha_out, AxpyBatch b, double* keep,
                          uint64_t keep_mask) {
  const int q = blockIdx.y;
  if (q == 0 && blockIdx.x == 0 && (int)threadIdx.x < b.K)
    alpha_out[threadIdx.x] = cg_alpha_of(threadIdx.x, gam, d1, d2, mu, active);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b.n[q] * b.K) return;
  const int k = (int)(e % b.K);
  const double a = cg_alpha_of(k, gam, d1, d2, mu, active);
  const double yo = b.y[q][e];
  if (q == 0 && keep && ((keep_mask >> k) & 1ull)) keep[e] = yo;
  b.y[q][e] = fma(b.sign[q] * a, b.x[q][e], yo);
}

hipError_t launch_cg_step(const double* gam, const double* d1, const double* d2, double mu, uint64_t active,
                          double* alpha_out, const AxpyBatch& b, double* keep, uint64_t keep_mask, hipStream_t s) {
  if (b.count < 1 || b.count > kAxpyBatchMax || b.K < 1 || b.K > 64) return hipErrorInvalidValue;
  int64_t mx = 0;
  for (int q = 0; q < b.count; ++q) mx = std::max<int64_t>(mx, b.n[q] * b.K);
  const unsigned bx = (unsigned)std::max<int64_t>((mx + 255) / 256, 1);
  hipLaunchKernelGGL(k_cg_step, dim3(bx, b.count), dim3(256), 0, s, gam, d1, d2, mu, active, alpha_out, b, keep,
                     keep_mask);
  return hipGetLastError();
}

// One workgroup's column dots of an n x K product in k_dot_small's order (K <= 64): column c's
// partials over rows r, r + R, ... (R the largest power of two with R K <= 1024), then a fixed
// pairwise tree; out[c] written by thread c, and the block synchronised on return.
__device__ void dot_cols_wg(const double* __restrict__ x, const double* __restrict__ y, int64_t n, int K,
                            double* __restrict__ out, double* red) {
  const int t = threadIdx.x;
  int R = 1;
  while (R * 2 * K <= kDotSmallWg) R *= 2;
  const int c = t % K, r = t / K;
  double s = 0.0;
  if (r < R)
    for (int64_t i = r; i < n; i += R) s = fma(x[i * K + c], y[i * K + c], s);
  red[t] = s;
  __syncthreads();
  for (int h = R / 2; h > 0; h >>= 1) {
    if (r < h) red[r * K + c] += red[(r + h) * K + c];
    __syncthreads();
  }
  if (t < K) out[t] = red[t];
  __syncthreads();
}

// The whole CG step of small systems in one workgroup: the dots of the step's products (the
// first launch_dot_batch), alpha and the updates (launch_cg_step), then the dots after the step
// (the second launch_dot_batch), each in the order the separate launches use.
__global__ __launch_bounds__(kDotSmallWg) void k_cg_step_small(CgStepSmall a) {
  __shared__ double red[kDotSmallWg];
  __shared__ double salpha[64];
  const int K = a.K, t = threadIdx.x;
  for (int q = 0; q < a.n_pre; ++q) dot_cols_wg(a.pre[q], a.pre[q], a.pre_n[q], K, a.pre_out[q], red);
  if (t < K) {
    const double al = cg_alpha_of(t, a.gam, a.d1, a.d2, a.mu, a.active);
    salpha[t] = al;
    a.alpha_out[t] = al;
  }
  __syncthreads();
  for (int q = 0; q < a.step.count; ++q) {
    const int64_t tot = a.step.n[q] * K;
    const double sg = a.step.sign[q];
    for (int64_t e = t; e < tot; e += kDotSmallWg) {
      const int k = (int)(e % K);
      const double yo = a.step.y[q][e];
      if (q == 0 && a.keep && ((a.keep_mask >> k) & 1ull)) a.keep[e] = yo;
      a.step.y[q][e] = fma(sg * salpha[k], a.step.x[q][e], yo);
    }
  }
  __syncthreads();
  for (int q = 0; q < a.n_post; ++q) dot_cols_wg(a.post[q], a.post[q], a.post_n[q], K, a.post_out[q], red);
}

bool cg_step_small_fits(const CgStepSmall& a) {
  if (a.K < 1 || a.K > 64) return false;
  for (int q = 0; q < a.n_pre; ++q)
    if (a.pre_n[q] * a.K > kDotSmallMax) return false;
  for (int q = 0; q < a.n_post; ++q)
    if (a.post_n[q] * a.K > kDotSmallMax) return false;
  for (int q = 0; q < a.step.count; ++q)
    if (a.step.n[q] * a.K > kDotSmallMax) return false;
  return true;
}

hipError_t launch_cg_step_small(const CgStepSmall& a, hipStream_t s) {
  if (!cg_step_small_fits(a) || a.n_pre > 4 || a.n_post > 2 || a.step.count < 1 || a.step.count > kAxpyBatchMax)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_step_small, dim3(1), dim3(kDotSmallWg), 0, s, a);
  return hipGetLastError();
}

// gam_new = g . z per column, beta = gam_new / gam_old (0 when gam_old <= 0), p = z + beta p;
// with gam_old null, p = z (the first direction; p is not read).  Small vectors
// (n K <= kDotSmallMax): one workgroup does all three, with k_dot_small's reduction order;
// larger ones take launch_dot_cols and one update launch.
__global__ __launch_bounds__(kDotSmallWg) void k_cg_direction_small(const double* __restrict__ g,
                                                                    const double* __restrict__ z, double* p, int64_t n,
                                                                    int K, const double* __restrict__ gam_old,
                                                                    double* __restrict__ gam_new) {
  __shared__ double red[kDotSmallWg];
  __shared__ double sbeta[64];
  const int t = threadIdx.x;
  int R = 1;
  while (R * 2 * K <= kDotSmallWg) R *= 2;
  const int c = t % K, r = t / K;
  double s = 0.0;
  if (r < R)
    for (int64_t i = r; i < n; i += R) s = fma(g[i * K + c], z[i * K + c], s);
  red[t] = s;
  __syncthreads();
  for (int h = R / 2; h > 0; h >>= 1) {
    if (r < h) red[r * K + c] += red[(r + h) * K + c];
    __syncthreads();
  }
  if (t < K) {
    const double gn = red[t], go = gam_old ? gam_old[t] : 0.0;
    gam_new[t] = gn;
    sbeta[t] = go > 0.0 ? gn / go : 0.0;
  }
  __syncthreads();
  if (gam_old)
    for (int64_t e = t; e < n * K; e += kDotSmallWg) p[e] = fma(sbeta[e % K], p[e], z[e]);
  else
    for (int64_t e = t; e < n * K; e += kDotSmallWg) p[e] = z[e];
}

__global__ void k_xpby_ratio(const double* __restrict__ z, const double* __restrict__ gam_new,
                             const double* __restrict__ gam_old, double* p, int64_t n, int K) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * K) return;
  if (!gam_old) {
    p[e] = z[e];
    return;
  }
  const int k = (int)(e % K);
  const double go = gam_old[k];
  const double beta = go > 0.0 ? gam_new[k] / go : 0.0;
  p[e] = fma(beta, p[e], z[e]);
}

hipError_t launch_cg_direction(const double* g, const double* z, double* p, int64_t n, int K, const double* gam_old,
                               double* gam_new, double* work, hipStream_t s) {
  if (K < 1 || K > 64) return hipErrorInvalidValue;
  if (n * K <= kDotSmallMax) {
    hipLaunchKernelGGL(k_cg_direction_small, dim3(1), dim3(kDotSmallWg), 0, s, g, z, p, n, K, gam_old, gam_new);
    return hipGetLastError();
  }
  hipError_t e = launch_dot_cols(g, z, n, K, gam_new, work, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_xpby_ratio, dim3((unsigned)((n * K + 255) / 256)), dim3(256), 0, s, z, gam_new, gam_old, p, n,
                     K);
  return hipGetLastError();
}

__global__ void k_select_cols(const double* src, double* dst, int64_t n, int K, uint64_t mask) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * K) return;
  if ((mask >> (e % K)) & 1ull) dst[e] = src[e];
}

hipError_t launch_select_cols(const double* src, double* dst, int64_t n, int K, uint64_t mask, hipStream_t s) {
  const int64_t tot = n * K;
  if (tot == 0 || mask == 0) return hipSuccess;
  if (K < 1 || K > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_select_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src, dst, n, K, mask);
  return hipGetLastError();
}

// NaN / Inf scan of several arrays in one launch: workgroup w of item q (grid.y) strides over
// the item's entries and writes flags[q * wgs + w] (0 or 1) itself, so nothing needs clearing.
__global__ __launch_bounds__(256) void k_finite_batch(FiniteBatch fb, int wgs, int* __restrict__ flags) {
  const int q = blockIdx.y, w = blockIdx.x;
  const double* __restrict__ x = fb.p[q];
  const int64_t n = x ? fb.n[q] : 0;
  int bad = 0;
  for (int64_t i = (int64_t)w * 256 + threadIdx.x; i < n; i += (int64_t)wgs * 256) bad |= !isfinite(x[i]);
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) flags[q * wgs + w] = bad ? 1 : 0;
}

int finite_batch_wgs(const FiniteBatch& fb) {
  int64_t mx = 1;
  for (int q = 0; q < fb.count; ++q)
    if (fb.p[q]) mx = std::max<int64_t>(mx, (fb.n[q] + 255) / 256);
  return (int)std::min<int64_t>(mx, kFiniteBatchWgs);
}

hipError_t launch_finite_batch(const FiniteBatch& fb, int* flags, hipStream_t s) {
  if (fb.count < 1 || fb.count > kFiniteBatchMax) return hipErrorInvalidValue;
  const int wgs = finite_batch_wgs(fb);
  hipLaunchKernelGGL(k_finite_batch, dim3(wgs, fb.count), dim3(256), 0, s, fb, wgs, flags);
  return hipGetLastError();
}


}  // namespace flsq
