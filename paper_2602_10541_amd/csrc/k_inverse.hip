// Kernels of the inverse heat-source application (Section 2.5: gradients through the
// pre-factored solve): Gaussian source right-hand sides for K hypotheses, the data
// misfit and its derivative, the chain rule through d rhs / d theta, and a batched
// Adam update of the K parameter vectors.
#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

// Rhs[i][h] = weight * a_h exp(-((x_i - cx_h)^2 + (y_i - cy_h)^2) / (2 w_h^2)) for i < n_src, else 0.
__global__ void k_source(const double* __restrict__ Xt, int64_t P, int64_t n_src, double weight,
                         const double* __restrict__ th, int K, double* __restrict__ Rhs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P * K) return;
  const int64_t i = e / K;
  const int h = (int)(e % K);
  double v = 0.0;
  if (i < n_src) {
    const double a = th[h * 4 + 0], cx = th[h * 4 + 1], cy = th[h * 4 + 2], w = th[h * 4 + 3];
    const double dx = Xt[i] - cx, dy = Xt[P + i] - cy;
    v = weight * a * exp(-(dx * dx + dy * dy) / (2.0 * w * w));
  }
  Rhs[e] = v;
}

hipError_t launch_source(const double* Xt, int64_t P, int64_t n_src, double weight, const double* thetas, int K,
                         double* Rhs, hipStream_t s) {
  const int64_t tot = P * K;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_source, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Xt, P, n_src, weight, thetas, K,
                     Rhs);
  return hipGetLastError();
}

// grad[h][p] = sum_{i < n_src} AL[i][h] * weight * d s(x_i; theta_h) / d theta_p,
//   ds/da = e, ds/dcx = a e dx / w^2, ds/dcy = a e dy / w^2, ds/dw = a e r^2 / w^3.
// Stage 1: workgroup (h, slab) writes 4 partial sums; stage 2 adds the slabs in order.
constexpr int kSrcSlabs = 64;

__global__ __launch_bounds__(256) void k_source_grad_stage1(const double* __restrict__ Xt, int64_t P, int64_t n_src,
                                                            double weight, const double* __restrict__ th, int K,
                                                            const double* __restrict__ AL,
                                                            double* __restrict__ work) {
  __shared__ double red[4][256];
  const int h = blockIdx.x;
  const int slab = blockIdx.y;
  const double a = th[h * 4 + 0], cx = th[h * 4 + 1], cy = th[h * 4 + 2], w = th[h * 4 + 3];
  const double iw2 = 1.0 / (w * w);
  double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
  for (int64_t i = (int64_t)slab * 256 + threadIdx.x; i < n_src; i += (int64_t)kSrcSlabs * 256) {
    const double dx = Xt[i] - cx, dy = Xt[P + i] - cy;
    const double r2 = dx * dx + dy * dy;
    const double e = exp(-0.5 * r2 * iw2);
    const double l = AL[i * K + h] * weight;
    g0 = fma(l, e, g0);
    g1 = fma(l, a * e * dx * iw2, g1);
    g2 = fma(l, a * e * dy * iw2, g2);
    g3 = fma(l, a * e * r2 * iw2 / w, g3);
  }
  red[0][threadIdx.x] = g0;
  red[1][threadIdx.x] = g1;
  red[2][threadIdx.x] = g2;
  red[3][threadIdx.x] = g3;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int p = 0; p < 4; ++p) red[p][threadIdx.x] += red[p][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) work[((int64_t)h * kSrcSlabs + slab) * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_source_grad_stage2(const double* __restrict__ work, int K, double* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= K * 4) return;
  const int h = e / 4, p = e % 4;
  double s = 0.0;
  for (int sl = 0; sl < kSrcSlabs; ++sl) s += work[((int64_t)h * kSrcSlabs + sl) * 4 + p];
  grad[e] = s;
}

hipError_t launch_source_grad_dot(const double* Xt, int64_t P, int64_t n_src, double weight, const double* thetas,
                                  int K, const double* AL, double* grad, double* work, hipStream_t s) {
  hipLaunchKernelGGL(k_source_grad_stage1, dim3(K, kSrcSlabs), dim3(256), 0, s, Xt, P, n_src, weight, thetas, K, AL,
                     work);
  hipLaunchKernelGGL(k_source_grad_stage2, dim3((K * 4 + 255) / 256), dim3(256), 0, s, work, K, grad);
  return hipGetLastError();
}

size_t source_grad_work_elems(int K) { return (size_t)K * kSrcSlabs * 4; }

// loss[h] = (1/n) sum_k (U[k][h] - d_k)^2 ; gu[k][h] = (2/n) (U[k][h] - d_k)
__global__ __launch_bounds__(256) void k_misfit(const double* __restrict__ U, const double* __restrict__ data,
                                                int64_t n_obs, int K, double* __restrict__ loss,
                                                double* __restrict__ gu) {
  __shared__ double red[256];
  const int h = blockIdx.x;
  const double inv = 1.0 / (double)n_obs;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < n_obs; k += 256) {
    const double r = U[k * K + h] - data[k];
    s = fma(r, r, s);
    gu[k * K + h] = 2.0 * inv * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[h] = red[0] * inv;
}

hipError_t launch_misfit(const double* U, const double* data, int64_t n_obs, int K, double* loss, double* gu,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_misfit, dim3(K), dim3(256), 0, s, U, data, n_obs, K, loss, gu);
  return hipGetLastError();
}

__global__ void k_combine_diff(const double* a, const double* b, double* out, int K) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < K) out[e] = a[e] - b[e];
}

hipError_t launch_combine_diff(const double* a, const double* b, double* out, int K, hipStream_t s) {
  hipLaunchKernelGGL(k_combine_diff, dim3((K + 255) / 256), dim3(256), 0, s, a, b, out, K);
  return hipGetLastError();
}

__global__ void k_adam(double* p, const double* g, double* m, double* v, int64_t n, int P, double lr, double b1,
                       double b2, double c1, double c2, double eps, int clamp_col, double clamp_min, double decay) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double gi = g[e];
  const double mi = b1 * m[e] + (1.0 - b1) * gi;
  const double vi = b2 * v[e] + (1.0 - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  double pi = p[e] * decay - lr * (mi / c1) / (sqrt(vi / c2) + eps);
  if (clamp_col >= 0 && (int)(e % P) == clamp_col && pi < clamp_min) pi = clamp_min;
  p[e] = pi;
}

hipError_t launch_adam(double* p, const double* g, double* m, double* v, int K, int P, int t, double lr, double b1,
                       double b2, double eps, int clamp_col, double clamp_min, double weight_decay, hipStream_t s) {
  const int64_t n = (int64_t)K * P;
  const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  const double decay = 1.0 - lr * weight_decay;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, P, lr, b1, b2, c1, c2,
                     eps, clamp_col, clamp_min, decay);
  return hipGetLastError();
}

}  // namespace flsq
