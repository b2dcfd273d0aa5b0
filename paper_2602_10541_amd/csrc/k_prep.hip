// Operator folding, layout transforms, assembly to HBM and evaluation of u_N.
#include "flsq_device.h"
#include "flsq_launch.h"

#include <algorithm>

namespace flsq {

// Per feature j of one row block with weight w and operator sum_t c_t D^{alpha_t}:
//   S_j = w * norm * sum_t c_t W_j^{alpha_t} s(|alpha_t|),  s = +1, 0, -1, 0 for |alpha| = 0, 1, 2, 3 mod 4
//   C_j = w * norm * sum_t c_t W_j^{alpha_t} c(|alpha_t|),  c =  0, +1, 0, -1
// (Eq. (2): Phi_0..3 = sin, cos, -sin, -cos), so that A_ij = S_j sin z_ij + C_j cos z_ij.
// Folded to amplitude/phase: even-order operators keep (amp, ph) = (S, b); otherwise
// (amp, ph) = (hypot(S, C), b + atan2(C, S)).
__global__ void k_prep_block(OpTerms op, double scale, int d, int n, const double* __restrict__ W,
                             const double* __restrict__ b, double* amp, double* ph, float* amp32, float* ph32) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double S = 0.0, Cc = 0.0;
  bool even = true;
  for (int t = 0; t < op.n_terms; ++t) {
    double mono = 1.0;
    int ord = 0;
    for (int k = 0; k < d; ++k) {
      const int a = op.alpha[t][k];
      ord += a;
      const double wk = W[(int64_t)j * d + k];
      for (int p = 0; p < a; ++p) mono *= wk;
    }
    const double v = op.coef[t] * mono;
    switch (ord & 3) {
      case 0: S += v; break;
      case 1: Cc += v; break;
      case 2: S -= v; break;
      default: Cc -= v; break;
    }
    if (ord & 1) even = false;
  }
  S *= scale;
  Cc *= scale;
  double a, p;
  if (even) {
    a = S;
    p = b[j];
  } else {
    a = hypot(S, Cc);
    p = b[j] + atan2(Cc, S);
  }
  amp[j] = a;
  ph[j] = p;
  amp32[j] = (float)a;
  ph32[j] = (float)p;
}

hipError_t launch_prep_block(const OpTerms& op, double weight, double norm, int d, int n, const double* W,
                             const double* b, double* amp, double* ph, float* amp32, float* ph32, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_block, dim3((n + 255) / 256), dim3(256), 0, s, op, weight * norm, d, n, W, b, amp, ph,
                     amp32, ph32);
  return hipGetLastError();
}

// X (rows x d, row-major) -> Xt[k * ld_out + i] in FP64 and FP32.
__global__ void k_transpose(const double* __restrict__ X, int64_t rows, int d, double* Xt, float* Xt32,
                            int64_t ld_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  for (int k = 0; k < d; ++k) {
    const double v = X[i * d + k];
    Xt[(int64_t)k * ld_out + i] = v;
    if (Xt32) Xt32[(int64_t)k * ld_out + i] = (float)v;
  }
}

hipError_t launch_transpose(const double* X, int64_t rows, int d, double* Xt, float* Xt32, int64_t ld_out,
                            hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, X, rows, d, Xt, Xt32,
                     ld_out);
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void k_scale_copy(const double* src, double* dst, int64_t n, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src ? scale * src[i] : 0.0;
}

hipError_t launch_scale_copy(const double* src, double* dst, int64_t n, double scale, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n, scale);
  return hipGetLastError();
}

// The rows of up to kRowStageMax blocks in one launch (grid.y = block of the group): the
// transposed points in FP64 and FP32, the row-major copy, each row's block index and the
// weighted right-hand side (0 where a block has none).
__global__ void k_stage_rows(RowStage rs, int d, int64_t P, double* __restrict__ Xt, float* __restrict__ Xt32,
                             double* __restrict__ Xrm, int32_t* __restrict__ row_block, double* __restrict__ rhs_w) {
  const int b = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rs.rows[b]) return;
  const int64_t g = rs.row0[b] + i;
  const double* __restrict__ x = rs.x[b];
  for (int k = 0; k < d; ++k) {
    const double v = x[i * d + k];
    Xt[(int64_t)k * P + g] = v;
    Xt32[(int64_t)k * P + g] = (float)v;
    Xrm[g * d + k] = v;
  }
  row_block[g] = rs.block0 + b;
  rhs_w[g] = rs.rhs[b] ? rs.weight[b] * rs.rhs[b][i] : 0.0;
}

hipError_t launch_stage_rows(const RowStage& rs, int d, int64_t P, double* Xt, float* Xt32, double* Xrm,
                             int32_t* row_block, double* rhs_w, hipStream_t s) {
  if (rs.count < 1 || rs.count > kRowStageMax) return hipErrorInvalidValue;
  int64_t mx = 0;
  for (int b = 0; b < rs.count; ++b) mx = std::max(mx, rs.rows[b]);
  if (mx == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stage_rows, dim3((unsigned)((mx + 255) / 256), rs.count), dim3(256), 0, s, rs, d, P, Xt, Xt32,
                     Xrm, row_block, rhs_w);
  return hipGetLastError();
}

__global__ void k_to_f32(const double* src, float* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// A[i][j] with the same arithmetic as the fused Gram kernels (FP64 or FP32).
__global__ void k_assemble(Geo g, int fp32, void* A) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= g.n) return;
  const int blk = g.row_block[i];
  if (fp32) {
    float z = 0.f;
    for (int k = 0; k < g.d; ++k) z = fmaf(g.Wt32[(int64_t)k * g.n + j], g.Xt32[(int64_t)k * g.P + i], z);
    const float v = g.amp32[(int64_t)blk * g.n + j] * sin_f32(z + g.ph32[(int64_t)blk * g.n + j]);
    ((float*)A)[i * g.n + j] = v;
  } else {
    double z = 0.0;
    for (int k = 0; k < g.d; ++k) z = fma(g.Wt[(int64_t)k * g.n + j], g.Xt[(int64_t)k * g.P + i], z);
    const double v = g.amp[(int64_t)blk * g.n + j] * sin_f64(z + g.ph[(int64_t)blk * g.n + j]);
    ((double*)A)[i * g.n + j] = v;
  }
}

hipError_t launch_assemble(const Geo& g, int fp32, void* A, hipStream_t s) {
  int64_t r0 = 0;
  while (r0 < g.P) {  // grid.y is limited to 65535 rows per launch
    const int64_t rows = (g.P - r0 < 65535) ? g.P - r0 : 65535;
    Geo gg = g;
    // shift the row view: rows [r0, r0 + rows)
    gg.Xt = g.Xt + r0;
    gg.Xt32 = g.Xt32 + r0;
    gg.row_block = g.row_block + r0;
    void* Ab = fp32 ? (void*)((float*)A + r0 * g.n) : (void*)((double*)A + r0 * g.n);
    hipLaunchKernelGGL(k_assemble, dim3((g.n + 255) / 256, (unsigned)rows), dim3(256), 0, s, gg, fp32, Ab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    r0 += rows;
  }
  return hipSuccess;
}

// Feature records for the matrix-free passes: rec[g][j] = {W_j, amp_gj, ph_gj, 0, ...}, so
// that a wave reads everything it needs about one feature with a single scalar load.
__global__ void k_pack_features(const double* __restrict__ Wrm, const double* __restrict__ amp,
                                const double* __restrict__ ph, int n, int d, double* __restrict__ rec) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (j >= n) return;
  const int rs = frec_stride(d);
  double* r = rec + ((int64_t)g * n + j) * rs;
  for (int k = 0; k < d; ++k) r[k] = Wrm[(int64_t)j * d + k];
  r[d] = amp[(int64_t)g * n + j];
  r[d + 1] = ph[(int64_t)g * n + j];
  for (int k = d + 2; k < rs; ++k) r[k] = 0.0;
}

hipError_t launch_pack_features(const double* Wrm, const double* amp, const double* ph, int n_blocks, int n, int d,
                                double* rec, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_features, dim3((n + 255) / 256, n_blocks), dim3(256), 0, s, Wrm, amp, ph, n, d, rec);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Learnable bandwidth (reparameterisation W_j = L What_j): the weights from the base draws,
// a phase shift of a built system (d/dz of every entry: sin(z + ph) -> sin(z + ph + pi/2)),
// and the feature-scaled right-hand sides of the bilinear forms.
// ---------------------------------------------------------------------------------
__global__ void k_apply_lower(const double* __restrict__ What, int n, int d, LowerMat Lm, double* __restrict__ W) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int k = 0; k < d; ++k) {
    double s = 0.0;
    for (int m = 0; m <= k; ++m) s = fma(Lm.v[k * kMaxDim + m], What[(int64_t)j * d + m], s);
    W[(int64_t)j * d + k] = s;
  }
}

hipError_t launch_apply_lower(const double* What, int n, int d, const LowerMat& Lm, double* W, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply_lower, dim3((n + 255) / 256), dim3(256), 0, s, What, n, d, Lm, W);
  return hipGetLastError();
}

__global__ void k_add_phase(double* ph, int64_t count, double delta) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) ph[e] += delta;
}

hipError_t launch_add_phase(double* ph, int64_t count, double delta, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_phase, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, ph, count, delta);
  return hipGetLastError();
}

// V[j][c] = beta_j What_jc for c < d, lam_j What_j(c - d) for d <= c < 2d
__global__ void k_scaled_cols(const double* __restrict__ beta, const double* __restrict__ lam,
                              const double* __restrict__ What, int n, int d, double* __restrict__ V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * 2 * d) return;
  const int j = (int)(e / (2 * d)), c = (int)(e % (2 * d));
  V[e] = (c < d ? beta[j] : lam[j]) * What[(int64_t)j * d + (c < d ? c : c - d)];
}

hipError_t launch_scaled_cols(const double* beta, const double* lam, const double* What, int n, int d, double* V,
                              hipStream_t s) {
  const int64_t tot = (int64_t)n * 2 * d;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scaled_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, beta, lam, What, n, d, V);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Evaluation (Eq. (1)-(2)): out[q][a] = norm * sum_j beta_j W_j^{alpha_a} Phi_{|alpha_a|}(z_qj).
// coef[a][j] = norm * beta_j * W_j^{alpha_a} * (+1 | -1) with the sign of Phi folded in, so
// every output needs only sin z (even order) or cos z (odd order).
// ---------------------------------------------------------------------------------
__global__ void k_eval_coef(int d, int n, int n_alpha, const double* __restrict__ Wt, const double* __restrict__ b,
                            const double* __restrict__ beta, const uint8_t* __restrict__ alphas, double norm,
                            double* coef, float* coef32, float* Wt32, float* b32) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int a = 0; a < n_alpha; ++a) {
    double mono = 1.0;
    int ord = 0;
    for (int k = 0; k < d; ++k) {
      const int e = alphas[a * d + k];
      ord += e;
      for (int p = 0; p < e; ++p) mono *= Wt[(int64_t)k * n + j];
    }
    const double sgn = ((ord & 3) >= 2) ? -1.0 : 1.0;
    const double c = norm * beta[j] * mono * sgn;
    coef[(int64_t)a * n + j] = c;
    coef32[(int64_t)a * n + j] = (float)c;
  }
  // the FP32 kernel works with the phase in revolutions: W / 2 pi and b / 2 pi, scaled in FP64
  constexpr double kInv2Pi = 0.15915494309189533577;
  for (int k = 0; k < d; ++k) Wt32[(int64_t)k * n + j] = (float)(Wt[(int64_t)k * n + j] * kInv2Pi);
  b32[j] = (float)(b[j] * kInv2Pi);
}

constexpr int kEvalThreads = 256;
constexpr int kEvalFeat = 256;     // features staged per LDS round
constexpr int kEvalPts = 2;        // query points per thread

template <int D, typename T>
__global__ __launch_bounds__(kEvalThreads) void k_evaluate(int n, int n_alpha, int64_t n_q, const T* __restrict__ Wt,
                                                           const T* __restrict__ b, const T* __restrict__ coef,
                                                           uint32_t cos_mask, const T* __restrict__ xq,
                                                           T* __restrict__ out) {
  constexpr int kMaxA = 8;
  __shared__ T sF[kEvalFeat][D + 1 + kMaxA];
  const int64_t q0 = ((int64_t)blockIdx.x * kEvalThreads + threadIdx.x) * kEvalPts;
  T x[kEvalPts][D];
  T acc[kEvalPts][kMaxA];
#pragma unroll
  for (int p = 0; p < kEvalPts; ++p) {
    const int64_t q = q0 + p;
#pragma unroll
    for (int k = 0; k < D; ++k) x[p][k] = (q < n_q) ? xq[q * D + k] : T(0);
#pragma unroll
    for (int a = 0; a < kMaxA; ++a) acc[p][a] = T(0);
  }
  for (int j0 = 0; j0 < n; j0 += kEvalFeat) {
    __syncthreads();
    for (int e = threadIdx.x; e < kEvalFeat; e += kEvalThreads) {
      const int j = j0 + e;
      const bool ok = j < n;
#pragma unroll
      for (int k = 0; k < D; ++k) sF[e][k] = ok ? Wt[(int64_t)k * n + j] : T(0);
      sF[e][D] = ok ? b[j] : T(0);
#pragma unroll
      for (int a = 0; a < kMaxA; ++a) sF[e][D + 1 + a] = (ok && a < n_alpha) ? coef[(int64_t)a * n + j] : T(0);
    }
    __syncthreads();
    const int jn = (n - j0 < kEvalFeat) ? n - j0 : kEvalFeat;
    for (int jj = 0; jj < jn; ++jj) {
#pragma unroll
      for (int p = 0; p < kEvalPts; ++p) {
        T z = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) z = fma(sF[jj][k], x[p][k], z);
        z += sF[jj][D];
        T sv, cv;
        if constexpr (sizeof(T) == 8)
          sincos_f64(z, &sv, &cv);
        else
          sincos_f32(z, &sv, &cv);
#pragma unroll
        for (int a = 0; a < kMaxA; ++a)
          if (a < n_alpha) acc[p][a] = fma(sF[jj][D + 1 + a], ((cos_mask >> a) & 1u) ? cv : sv, acc[p][a]);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < kEvalPts; ++p) {
    const int64_t q = q0 + p;
    if (q < n_q)
#pragma unroll
      for (int a = 0; a < kMaxA; ++a)
        if (a < n_alpha) out[q * n_alpha + a] = acc[p][a];
  }
}

// FP32 evaluation.  The phase is formed in revolutions, z = (W / 2 pi) . x + b / 2 pi, reduced to
// [0, 1) by its fractional part (exact: z - floor z) and passed to the hardware sine and cosine
// (v_sin_f32 / v_cos_f32 take their argument in revolutions), one of each per (point, feature)
// pair.  Outputs are visited with the sine-type ones (even |alpha|) first, so each pair costs
// d multiply-adds for the phase, one reduction, two transcendental ops and one multiply-add per
// output.  (Contracting the outputs on the matrix cores instead, 16 points x 4 features per
// v_mfma_f32_16x16x4f32, was measured no faster on the 3D + t heat evaluation.)
struct EvalOrder {
  int n_sin;                 // outputs [0, n_sin) use sin z, the rest cos z
  int perm[8];               // visiting slot -> output column (and coefficient row)
};
constexpr int kEvalPts32 = 4;

// NS1 = 1: exactly one sine-type output (u and first derivatives, the usual query), fixed at
// compile time so no per-output select is issued; NS1 = 0 reads the split from ord.n_sin.
template <int D, int NA, int NS1>
__global__ __launch_bounds__(kEvalThreads) void k_evaluate_f32(int n, int64_t n_q,
                                                               const float* __restrict__ Wr,
                                                               const float* __restrict__ br,
                                                               const float* __restrict__ coef, EvalOrder ord,
                                                               const float* __restrict__ xq,
                                                               float* __restrict__ out) {
  __shared__ float sF[kEvalFeat][D + 1 + NA];
  const int64_t q0 = ((int64_t)blockIdx.x * kEvalThreads + threadIdx.x) * kEvalPts32;
  float x[kEvalPts32][D];
  float acc[kEvalPts32][NA];
#pragma unroll
  for (int p = 0; p < kEvalPts32; ++p) {
    const int64_t q = q0 + p;
#pragma unroll
    for (int k = 0; k < D; ++k) x[p][k] = (q < n_q) ? xq[q * D + k] : 0.f;
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[p][a] = 0.f;
  }
  for (int j0 = 0; j0 < n; j0 += kEvalFeat) {
    __syncthreads();
    for (int e = threadIdx.x; e < kEvalFeat; e += kEvalThreads) {
      const int j = j0 + e;
      const bool ok = j < n;
#pragma unroll
      for (int k = 0; k < D; ++k) sF[e][k] = ok ? Wr[(int64_t)k * n + j] : 0.f;
      sF[e][D] = ok ? br[j] : 0.f;
#pragma unroll
      for (int a = 0; a < NA; ++a) sF[e][D + 1 + a] = ok ? coef[(int64_t)ord.perm[a] * n + j] : 0.f;
    }
    __syncthreads();
    const int jn = (n - j0 < kEvalFeat) ? n - j0 : kEvalFeat;
    for (int jj = 0; jj < jn; ++jj) {
#pragma unroll
      for (int p = 0; p < kEvalPts32; ++p) {
        float z = sF[jj][D];
#pragma unroll
        for (int k = 0; k < D; ++k) z = fmaf(sF[jj][k], x[p][k], z);
        z = __builtin_amdgcn_fractf(z);
        const float sv = __builtin_amdgcn_sinf(z);
        const float cv = __builtin_amdgcn_cosf(z);
#pragma unroll
        for (int a = 0; a < NA; ++a)
          acc[p][a] = fmaf(sF[jj][D + 1 + a], (a < (NS1 ? 1 : ord.n_sin)) ? sv : cv, acc[p][a]);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < kEvalPts32; ++p) {
    const int64_t q = q0 + p;
    if (q < n_q)
#pragma unroll
      for (int a = 0; a < NA; ++a) out[q * NA + ord.perm[a]] = acc[p][a];
  }
}

template <int D>
hipError_t launch_evaluate_f32(const EvalArgs& a, const EvalOrder& ord, unsigned grid, hipStream_t s) {
  switch (a.n_alpha) {
#define FLSQ_EV32(NA)                                                                                       \
  case NA:                                                                                                 \
    if (ord.n_sin == 1)                                                                                    \
      hipLaunchKernelGGL((k_evaluate_f32<D, NA, 1>), dim3(grid), dim3(kEvalThreads), 0, s, a.n, a.n_q, a.Wt32,  \
                         a.b32, a.coef32, ord, (const float*)a.xq, (float*)a.out);                         \
    else                                                                                                   \
      hipLaunchKernelGGL((k_evaluate_f32<D, NA, 0>), dim3(grid), dim3(kEvalThreads), 0, s, a.n, a.n_q, a.Wt32,  \
                         a.b32, a.coef32, ord, (const float*)a.xq, (float*)a.out);                         \
    break;
    FLSQ_EV32(1) FLSQ_EV32(2) FLSQ_EV32(3) FLSQ_EV32(4) FLSQ_EV32(5) FLSQ_EV32(6) FLSQ_EV32(7) FLSQ_EV32(8)
#undef FLSQ_EV32
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define FLSQ_EVAL_CASE(DIM)                                                                              \
  case DIM:                                                                                              \
    if (a.fp32)                                                                                          \
      return launch_evaluate_f32<DIM>(a, ord, grid32, s);                                                \
    else                                                                                                 \
      hipLaunchKernelGGL((k_evaluate<DIM, double>), dim3(grid), dim3(kEvalThreads), 0, s, a.n, a.n_alpha, \
                         a.n_q, a.Wt, a.b, a.coef, mask, (const double*)a.xq, (double*)a.out);           \
    break;

hipError_t launch_evaluate(const EvalArgs& a, hipStream_t s) {
  const uint32_t mask = a.cos_mask;
  hipLaunchKernelGGL(k_eval_coef, dim3((a.n + 255) / 256), dim3(256), 0, s, a.d, a.n, a.n_alpha, a.Wt, a.b, a.beta,
                     a.alphas, a.norm, a.coef, a.coef32, a.Wt32, a.b32);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.n_q == 0) return e;
  EvalOrder ord{};
  int k = 0;
  for (int t = 0; t < a.n_alpha; ++t)
    if (!((mask >> t) & 1u)) ord.perm[k++] = t;
  ord.n_sin = k;
  for (int t = 0; t < a.n_alpha; ++t)
    if ((mask >> t) & 1u) ord.perm[k++] = t;
  for (; k < 8; ++k) ord.perm[k] = 0;
  const int64_t pts_per_wg = (int64_t)kEvalThreads * kEvalPts;
  const unsigned grid = (unsigned)((a.n_q + pts_per_wg - 1) / pts_per_wg);
  const int64_t pts_per_wg32 = (int64_t)kEvalThreads * kEvalPts32;
  const unsigned grid32 = (unsigned)((a.n_q + pts_per_wg32 - 1) / pts_per_wg32);
  switch (a.d) {
    FLSQ_EVAL_CASE(1) FLSQ_EVAL_CASE(2) FLSQ_EVAL_CASE(3) FLSQ_EVAL_CASE(4)
    FLSQ_EVAL_CASE(5) FLSQ_EVAL_CASE(6) FLSQ_EVAL_CASE(7) FLSQ_EVAL_CASE(8)
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace flsq
