// Factorisation and inversion of one 64 x 64 diagonal block of the regularised Gram
// (blocked Cholesky, step 1 of the block loop in fastlsq.cpp).  Kept in its own file:
// the fully unrolled register code takes a while to compile.
#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

// ------------------------------------------------------------------ Cholesky
// Factor one diagonal block (right-looking, rows scaled by the pivot root), then invert
// it, X_kk = U_kk^{-1}, by back substitution.  X_kk goes to the diagonal block of X
// (n x n), which the block-row solve and the preconditioner use.
//
// One wave.  Lane j keeps column j of the block in registers (fully unrolled loops, so
// every index is static); row values move between lanes with v_readlane (a register
// broadcast, no memory).  A short last block (nbk < 64) is padded with the identity,
// which leaves the leading nbk x nbk factor and inverse unchanged.  Entries below the
// diagonal of a lane's column are scratch: they are never broadcast as U values.
__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffll), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__global__ __launch_bounds__(64) void k_potrf_diag(double* G, int n, int k0, int* info, double* X) {
  const int nbk = min(kNb, n - k0);
  const int j = threadIdx.x;
  double col[kNb];
#pragma unroll
  for (int i = 0; i < kNb; ++i) {
    double v = (i == j) ? 1.0 : 0.0;
    if (j < nbk && i < nbk && i <= j) v = G[(int64_t)(k0 + i) * n + k0 + j];
    col[i] = v;
  }
  // row l of U is (col[l] of every lane) after scaling by 1/sqrt(pivot)
#pragma unroll
  for (int l = 0; l < kNb; ++l) {
    double piv = lane_bcast(col[l], l);
    if (!(piv > 0.0) || !isfinite(piv)) {   // not positive definite (or NaN): record, keep going
      if (j == 0 && l < nbk && *info == 0) *info = k0 + l + 1;
      piv = 1.0;
    }
    const double dl = sqrt(piv);
    const double rdl = 1.0 / dl;
    const double ulj = (j > l) ? col[l] * rdl : ((j == l) ? dl : 0.0);
    col[l] = ulj;
#pragma unroll
    for (int i = l + 1; i < kNb; ++i) col[i] = fma(-lane_bcast(ulj, i), ulj, col[i]);
  }
#pragma unroll
  for (int i = 0; i < kNb; ++i)
    if (j < nbk && i <= j) G[(int64_t)(k0 + i) * n + k0 + j] = col[i];
  // X = U^{-1}: column j by back substitution, x_i = (e_ij - sum_{m > i} U_im x_m) / U_ii,
  // where U_im is lane m's col[i].
  double x[kNb];
#pragma unroll
  for (int i = kNb - 1; i >= 0; --i) {
    double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
    for (int m = i + 1; m < kNb; ++m) s = fma(-lane_bcast(col[i], m), x[m], s);
    x[i] = s / lane_bcast(col[i], i);
  }
#pragma unroll
  for (int i = 0; i < kNb; ++i)
    if (j < nbk && i < nbk) X[(int64_t)(k0 + i) * n + k0 + j] = x[i];
}

hipError_t launch_potrf_diag(double* G, int n, int k0, int* info, double* X, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(64), 0, s, G, n, k0, info, X);
  return hipGetLastError();
}

}  // namespace flsq
