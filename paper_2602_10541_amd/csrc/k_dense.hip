// Dense FP64 building blocks on gfx950 MFMA: a descriptor-batched GEMM, the explicit
// inverse of the upper Cholesky factor, and the triangular matrix-vector products that
// apply the preconditioner M^{-1} = U^{-1} U^{-T} = X X^T.
//
// With X = U^{-1} formed once per factorisation, every preconditioner application in the
// refinement is two bandwidth-bound passes over the triangle of X instead of 2 N / 64
// dependent block steps.
#include "flsq_device.h"
#include "flsq_launch.h"

#include <algorithm>

namespace flsq {

constexpr int kGT = 64;       // output tile (kGT x kGT) per workgroup
constexpr int kGK = 16;       // K slab staged in LDS

// C[M x N] = alpha * op(A)[M x K] * B[K x N] + beta * C, all row-major with leading
// dimensions; op(A) = A (lda >= K) or A^T (A stored K x M, lda >= M).
// Four waves in 2 x 2, each a 32 x 32 quarter as 2 x 2 blocks of v_mfma_f64_16x16x4f64.
__global__ __launch_bounds__(256) void k_gemm_batched(const GemmDesc* __restrict__ descs, double alpha, double beta,
                                                      int transA) {
  __shared__ double sA[kGK][kGT + 1];   // sA[k][m]
  __shared__ double sB[kGK][kGT + 1];   // sB[k][n]
  const GemmDesc D = descs[blockIdx.z];
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  if (m0 >= D.M || n0 >= D.N) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < D.K; k0 += kGK) {
    __syncthreads();
    for (int e = tid; e < kGK * kGT; e += 256) {
      int k, m;
      if (transA) {        // A stored K x M: read rows of A (coalesced along m)
        k = e / kGT;
        m = e % kGT;
      } else {             // A stored M x K: read rows of A (coalesced along k)
        m = e / kGK;
        k = e % kGK;
      }
      const int gk = k0 + k, gm = m0 + m;
      double v = 0.0;
      if (gk < D.K && gm < D.M) v = transA ? D.A[(int64_t)gk * D.lda + gm] : D.A[(int64_t)gm * D.lda + gk];
      sA[k][m] = v;
      const int kb = e / kGT, nb = e % kGT;
      const int gkb = k0 + kb, gn = n0 + nb;
      sB[kb][nb] = (gkb < D.K && gn < D.N) ? D.B[(int64_t)gkb * D.ldb + gn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kGK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = sA[k][wm * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = sB[k][wn * 32 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm * 32 + a * 16 + 4 * v + (lane >> 4);
        const int gn = n0 + wn * 32 + b * 16 + (lane & 15);
        if (gm < D.M && gn < D.N) {
          double* c = D.C + (int64_t)gm * D.ldc + gn;
          *c = (beta == 0.0) ? alpha * acc[a][b][v] : fma(alpha, acc[a][b][v], beta * *c);
        }
      }
}

hipError_t launch_gemm_batched(const GemmDesc* d_descs, int n_batch, int maxM, int maxN, double alpha, double beta,
                               int transA, hipStream_t s) {
  if (n_batch == 0 || maxM == 0 || maxN == 0) return hipSuccess;
  dim3 grid((maxN + kGT - 1) / kGT, (maxM + kGT - 1) / kGT, n_batch);
  hipLaunchKernelGGL(k_gemm_batched, grid, dim3(256), 0, s, d_descs, alpha, beta, transA);
  return hipGetLastError();
}

// ------------------------------------------------------------------ triangular-aware GEMM
// C = alpha A B per descriptor (row-major, no transposes) for the explicit inverse factor,
// where one operand is upper triangular: desc.tri = 1 means B[k][n] = 0 for k > n, so an
// output tile with columns < n0 + 128 needs k < n0 + 128; desc.tri = 2 means A[m][k] = 0 for
// k < m, so a tile with rows >= m0 needs k >= m0.  128 x 128 tiles, 4 waves in 2 x 2, each a
// 64 x 64 quarter as 4 x 4 blocks of v_mfma_f64_16x16x4f64; 16-deep K slices staged in LDS,
// the next slice fetched into registers while the current one is multiplied.
constexpr int kTT = 128;
constexpr int kTK = 16;
constexpr int kTPad = 2;   // LDS row padding (doubles): 1 leaves bank conflicts in the transposing stash

// blockIdx.z = desc * nsplit + split.  With nsplit == 1 the tile goes to C (times alpha);
// otherwise split s covers K range [s kper, (s + 1) kper) and its unscaled partial tile goes to
// part[(blockIdx.z * maxM + m) * maxN + n] (zeros where the range is empty), summed by
// k_gemm_tri_reduce.
// Two workgroups per CU (accumulators in VGPRs): measured 17% faster than one with AGPRs.
__global__ __launch_bounds__(256, 2) void k_gemm_tri(const GemmDesc* __restrict__ descs, double alpha, int nsplit,
                                                  int kper, int maxM, int maxN, double* __restrict__ part) {
  __shared__ double sA[2][kTK][kTT + kTPad];   // sA[buf][k][m]
  __shared__ double sB[2][kTK][kTT + kTPad];   // sB[buf][k][n]
  const int split = blockIdx.z % nsplit;
  const GemmDesc D = descs[blockIdx.z / nsplit];
  const int m0 = blockIdx.y * kTT, n0 = blockIdx.x * kTT;
  if (m0 >= D.M || n0 >= D.N) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int kbeg = 0, kend = D.K;
  if (D.tri == 1) kend = min(kend, n0 + kTT);
  if (D.tri == 2) kbeg = (m0 / kTK) * kTK;
  if (nsplit > 1) {
    kbeg = max(kbeg, split * kper);
    kend = min(kend, (split + 1) * kper);
  }
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // per slice each thread moves 8 entries of A (row m = e / 16, k = e % 16: 128-byte row pieces)
  // and 8 of B (row k = e / 128, column n = e % 128)
  constexpr int kQ = kTK * kTT / 256;
  double ra[kQ], rb[kQ];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = tid + 256 * q;
      const int m = e / kTK, k = e % kTK;
      const int gm = m0 + m, gk = k0 + k;
      ra[q] = (gm < D.M && gk < kend) ? D.A[(int64_t)gm * D.lda + gk] : 0.0;
      const int kb = e / kTT, nb = e % kTT;
      const int gkb = k0 + kb, gn = n0 + nb;
      rb[q] = (gkb < kend && gn < D.N) ? D.B[(int64_t)gkb * D.ldb + gn] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = tid + 256 * q;
      sA[buf][e % kTK][e / kTK] = ra[q];
      sB[buf][e / kTT][e % kTT] = rb[q];
    }
  };
  // Two LDS buffers: slice s is read from buffer s & 1 while slice s + 1 is stashed into
  // the other one and slice s + 2 is fetched into registers; one barrier per slice.
  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
    if (kbeg + kTK < kend) fetch(kbeg + kTK);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += kTK, buf ^= 1) {
#pragma unroll
    for (int kk = 0; kk < kTK / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = sA[buf][k][wm * 64 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = sB[buf][k][wn * 64 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (k0 + kTK < kend) {
      stash(buf ^ 1);   // slice k0 + kTK; that buffer's last reads were before the previous barrier
      if (k0 + 2 * kTK < kend) fetch(k0 + 2 * kTK);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm * 64 + a * 16 + 4 * v + (lane >> 4);
        const int gn = n0 + wn * 64 + b * 16 + (lane & 15);
        if (gm < D.M && gn < D.N) {
          if (nsplit == 1) D.C[(int64_t)gm * D.ldc + gn] = alpha * acc[a][b][v];
          else part[((int64_t)blockIdx.z * maxM + gm) * maxN + gn] = acc[a][b][v];
        }
      }
}

// C[m][n] = alpha * sum_s part[desc][s][m][n] in split order.
__global__ __launch_bounds__(256) void k_gemm_tri_reduce(const GemmDesc* __restrict__ descs, double alpha, int nsplit,
                                                         int maxM, int maxN, const double* __restrict__ part) {
  const GemmDesc D = descs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int m = (int)(e / maxN), n = (int)(e % maxN);
  if (m >= D.M || n >= D.N) return;
  const int64_t plane = (int64_t)maxM * maxN;
  const double* p = part + (int64_t)blockIdx.y * nsplit * plane + e;
  double acc = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) acc += p[sp * plane];
  D.C[(int64_t)m * D.ldc + n] = alpha * acc;
}

// Split count: about 1024 workgroups in all, K ranges of at least 64, partials within
// work_elems doubles.
int gemm_tri_splits(int n_batch, int maxM, int maxN, int maxK, size_t work_elems) {
  const int64_t tiles = (int64_t)((maxN + kTT - 1) / kTT) * ((maxM + kTT - 1) / kTT) * n_batch;
  int ns = (int)std::min<int64_t>(std::max<int64_t>(1, (1024 + tiles - 1) / std::max<int64_t>(tiles, 1)), 64);
  ns = std::min(ns, std::max(1, maxK / 64));
  while (ns > 1 && (size_t)ns * n_batch * (size_t)maxM * maxN > work_elems) --ns;
  return ns;
}

hipError_t launch_gemm_tri(const GemmDesc* d_descs, int n_batch, int maxM, int maxN, int maxK, double alpha,
                           double* work, size_t work_elems, hipStream_t s) {
  if (n_batch == 0 || maxM == 0 || maxN == 0) return hipSuccess;
  const int ns = work ? gemm_tri_splits(n_batch, maxM, maxN, maxK, work_elems) : 1;
  const int kper = ((maxK + ns - 1) / ns + kTK - 1) / kTK * kTK;
  dim3 grid((maxN + kTT - 1) / kTT, (maxM + kTT - 1) / kTT, n_batch * ns);
  hipLaunchKernelGGL(k_gemm_tri, grid, dim3(256), 0, s, d_descs, alpha, ns, kper, maxM, maxN, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ns == 1) return e;
  const int64_t plane = (int64_t)maxM * maxN;
  hipLaunchKernelGGL(k_gemm_tri_reduce, dim3((unsigned)((plane + 255) / 256), n_batch), dim3(256), 0, s, d_descs,
                     alpha, ns, maxM, maxN, work);
  return hipGetLastError();
}

// ------------------------------------------------------------------ split-K partial sums
// out[e] = sum_s part[s][e] for e < len, s < n_split.  Workgroup: 64 entries x 4 groups of
// splits (group g sums splits g, g + 4, ...); the group sums are added in a fixed order.
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int n_split, int64_t len,
                                                      double* __restrict__ out) {
  __shared__ double red[4][64];
  const int o = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + o;
  double s = 0.0;
  if (e < len)
    for (int sp = grp; sp < n_split; sp += 4) s += part[(int64_t)sp * len + e];
  red[grp][o] = s;
  __syncthreads();
  if (grp == 0 && e < len) out[e] = (red[0][o] + red[1][o]) + (red[2][o] + red[3][o]);
}

hipError_t launch_sum_partials(const double* part, int n_split, int64_t len, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)((len + 63) / 64)), dim3(256), 0, s, part, n_split, len, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ preconditioner application
// y = X^T v  (X upper triangular, n x n row-major): y_j = sum_{i <= j} X[i][j] v_i.
// Grid (column tiles, row splits): each thread owns a column, loops over its row range;
// partial sums go to work[split][j], reduced in order by k_sum_tv_splits.
constexpr int kTvSplits = 32;

__global__ __launch_bounds__(256) void k_trmv_t(const double* __restrict__ X, int n, const double* __restrict__ v,
                                                double* __restrict__ work) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int split = blockIdx.y;
  const int per = (n + kTvSplits - 1) / kTvSplits;
  const int i0 = split * per;
  const int i1 = min(n, i0 + per);
  if (j >= n) return;
  // rows i0 .. min(i1, j + 1) - 1 of column j; four independent partial sums keep four loads in
  // flight (the order of the terms is fixed, so the result does not depend on scheduling)
  const int iend = min(i1, j + 1);
  const double* col = X + j;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int i = i0;
  for (; i + 4 <= iend; i += 4) {
    s0 = fma(col[(int64_t)i * n], v[i], s0);
    s1 = fma(col[(int64_t)(i + 1) * n], v[i + 1], s1);
    s2 = fma(col[(int64_t)(i + 2) * n], v[i + 2], s2);
    s3 = fma(col[(int64_t)(i + 3) * n], v[i + 3], s3);
  }
  for (; i < iend; ++i) s0 = fma(col[(int64_t)i * n], v[i], s0);
  work[(int64_t)split * n + j] = (s0 + s1) + (s2 + s3);
}

// The kTvSplits partials of k_trmv_t, summed in split order: all loads of a column issued at
// once (unrolled), 64 columns per workgroup so that small n still spreads over several CUs.
__global__ __launch_bounds__(64) void k_sum_tv_splits(const double* __restrict__ work, int n, double* __restrict__ out) {
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= n) return;
  double v[kTvSplits];
#pragma unroll
  for (int sp = 0; sp < kTvSplits; ++sp) v[sp] = work[(int64_t)sp * n + j];
  double s = 0.0;
#pragma unroll
  for (int sp = 0; sp < kTvSplits; ++sp) s += v[sp];
  out[j] = s;
}

// z = X y: z_i = sum_{j >= i} X[i][j] y_j; one wave per row, lanes stride the row with four
// independent partial sums, then a fixed butterfly.
__global__ __launch_bounds__(256) void k_trmv_n(const double* __restrict__ X, int n, const double* __restrict__ y,
                                                double* __restrict__ z) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const double* row = X + (int64_t)i * n;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = i + lane;
  for (; j + 192 < n; j += 256) {
    s0 = fma(row[j], y[j], s0);
    s1 = fma(row[j + 64], y[j + 64], s1);
    s2 = fma(row[j + 128], y[j + 128], s2);
    s3 = fma(row[j + 192], y[j + 192], s3);
  }
  for (; j < n; j += 64) s0 = fma(row[j], y[j], s0);
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
  if (lane == 0) z[i] = s;
}

hipError_t launch_precond_apply(const double* X, int n, const double* v, double* tmp, double* work, double* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_trmv_t, dim3((n + 255) / 256, kTvSplits), dim3(256), 0, s, X, n, v, work);
  hipLaunchKernelGGL(k_sum_tv_splits, dim3((n + 63) / 64), dim3(64), 0, s, work, n, tmp);
  hipLaunchKernelGGL(k_trmv_n, dim3((n + 3) / 4), dim3(256), 0, s, X, n, tmp, out);
  return hipGetLastError();
}

size_t precond_work_elems(int n) { return (size_t)kTvSplits * n; }

// ------------------------------------------------------------------ multi-column preconditioner
// Z = X (X^T Y) for 2 <= K <= 64 columns, X upper triangular n x n, Y, T, Z n x K, all row-major.
// Both products run on 16-row output tiles (n_pad = n rounded up to 16, nt = n_pad / 16 tiles).
// Tile t of T = X^T Y contracts k in [0, 16 t + 16), tile t of Z = X T contracts k in
// [16 t, n_pad); either way a tile whose contraction holds v 16-blocks is cut into
// ceil(v / r) chunks of kc = 16 r indices, one workgroup each, so that the long tiles spread
// over many CUs.  Tasks are numbered by v, then chunk: tiles with v blocks start at task
// sum_{u < v} ceil(u / r).  A workgroup is 4 waves; wave w holds columns 16w .. 16w + 15 in one
// v_mfma_f64_16x16x4f64 accumulator and writes its chunk's partial tile to part[task][16][K];
// k_trimm_sum adds the chunks of each tile in chunk order (no atomics: the result does not
// depend on scheduling).
__host__ __device__ inline int64_t trimm_task0(int v, int r) {   // sum_{u = 1}^{v - 1} ceil(u / r)
  const int64_t t = v - 1, a = t / r, b = t % r;
  return r * a * (a + 1) / 2 + b * (a + 1);
}

__device__ inline void trimm_locate(int64_t task, int nt, int r, int* v_out, int* j_out) {
  int lo = 1, hi = nt;   // largest v with trimm_task0(v) <= task
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (trimm_task0(mid, r) <= task) lo = mid;
    else hi = mid - 1;
  }
  *v_out = lo;
  *j_out = (int)(task - trimm_task0(lo, r));
}

constexpr int kTrimmMaxKc = 512;

int trimm_kc(int n) {
  const int np = (n + 15) / 16 * 16;
  return np <= 2048 ? 128 : (np <= 4096 ? 256 : kTrimmMaxKc);
}

// part = chunk partials of X^T Y (TRANS = 1) or X T (TRANS = 0).  X^T Y reads rows of X
// (16 consecutive entries per lane group: coalesced) straight into the MFMA operand; X T needs
// X by columns, so the workgroup first copies its 16 x kc block of X into LDS transposed.
template <int TRANS, int KC>
__device__ __forceinline__ void trimm_body(const double* __restrict__ X, int n, const double* __restrict__ B, int K,
                                           int kc, double* __restrict__ part, double (*sX)[17]) {
  const int nt = (n + 15) >> 4, r = kc >> 4;
  int v, j;
  trimm_locate(blockIdx.x, nt, r, &v, &j);
  const int t = TRANS ? v - 1 : nt - v;
  const int i0 = 16 * t;
  const int kb = (TRANS ? 0 : i0) + j * kc;
  const int ke = min(kb + kc, TRANS ? 16 * v : 16 * nt);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (!TRANS) {
    const int len = ke - kb;
    for (int e = tid; e < 16 * len; e += 256) {
      const int row = e / len, kk = e - row * len;
      const int i = i0 + row, k = kb + kk;
      sX[kk][row] = (i < n && k < n && k >= i) ? X[(int64_t)i * n + k] : 0.0;
    }
    __syncthreads();
  }
  const int c0 = 16 * wave;
  if (c0 >= K) return;
  const int col = c0 + (lane & 15);
  const int m = lane & 15, kq = lane >> 4;
  f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
  constexpr int kBatch = 16;   // MFMA steps whose operands are loaded together
  for (int k4 = kb; k4 < ke; k4 += 4 * kBatch) {
    double a[kBatch], b[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int k = k4 + 4 * q + kq;
      const bool in = k < ke && k < n;
      if (TRANS) {
        const int i = i0 + m;
        a[q] = (in && i < n && k <= i) ? X[(int64_t)k * n + i] : 0.0;
      } else {
        a[q] = in ? sX[k - kb][m] : 0.0;
      }
      b[q] = (in && col < K) ? B[(int64_t)k * K + col] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc, 0, 0, 0);
  }
  double* out = part + (int64_t)blockIdx.x * 16 * K;
#pragma unroll
  for (int e = 0; e < 4; ++e) {   // FP64 16x16 accumulator: element e of lane group kq is row 4 e + kq
    const int row = 4 * e + kq;
    if (col < K) out[row * K + col] = acc[e];
  }
}

// X^T Y
__global__ __launch_bounds__(256) void k_trimm_t(const double* __restrict__ X, int n, const double* __restrict__ B,
                                                 int K, int kc, double* __restrict__ part) {
  trimm_body<1, 1>(X, n, B, K, kc, part, nullptr);
}

// X T: the workgroup's 16 x KC block of X staged transposed in LDS sized for KC
template <int KC>
__global__ __launch_bounds__(256) void k_trimm_n(const double* __restrict__ X, int n, const double* __restrict__ B,
                                                 int K, double* __restrict__ part) {
  __shared__ double sX[KC][17];
  trimm_body<0, KC>(X, n, B, K, KC, part, sX);
}

// out[16 t + m][c] = sum over the chunks of tile t, in chunk order: one thread per entry (grid
// x: tiles, grid y: 64-entry slices of the tile's 16 K entries), four chunk loads in flight.
template <int TRANS>
__global__ __launch_bounds__(64) void k_trimm_sum(const double* __restrict__ part, int n, int K, int kc,
                                                  double* __restrict__ out) {
  const int nt = (n + 15) >> 4, r = kc >> 4;
  const int t = blockIdx.x;
  const int e = blockIdx.y * 64 + threadIdx.x;
  if (e >= 16 * K || 16 * t + e / K >= n) return;
  const int v = TRANS ? t + 1 : nt - t;
  const int64_t task0 = trimm_task0(v, r);
  const int nch = (v + r - 1) / r;
  const double* p = part + task0 * 16 * K + e;
  const int64_t stride = (int64_t)16 * K;
  double s = 0.0;
  int ch = 0;
  for (; ch + 4 <= nch; ch += 4) {
    const double a = p[(ch + 0) * stride], b = p[(ch + 1) * stride], c = p[(ch + 2) * stride], d = p[(ch + 3) * stride];
    s += a;
    s += b;
    s += c;
    s += d;
  }
  for (; ch < nch; ++ch) s += p[ch * stride];
  out[(int64_t)16 * t * K + e] = s;
}

size_t chol_multi_work_elems(int n, int K) {
  const int nt = (n + 15) / 16, r = trimm_kc(n) / 16;
  return (size_t)trimm_task0(nt + 1, r) * 16 * K;
}

hipError_t launch_chol_solve_multi(const double* X, int n, const double* Y, int K, double* T, double* part, double* Z,
                                   hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (K < 2 || K > 64) return hipErrorInvalidValue;
  const int nt = (n + 15) / 16, kc = trimm_kc(n), r = kc / 16;
  const unsigned tasks = (unsigned)trimm_task0(nt + 1, r);
  const dim3 gsum(nt, (16 * K + 63) / 64);
  hipLaunchKernelGGL(k_trimm_t, dim3(tasks), dim3(256), 0, s, X, n, Y, K, kc, part);
  hipLaunchKernelGGL(k_trimm_sum<1>, gsum, dim3(64), 0, s, part, n, K, kc, T);
  if (kc == 128) hipLaunchKernelGGL(k_trimm_n<128>, dim3(tasks), dim3(256), 0, s, X, n, T, K, part);
  else if (kc == 256) hipLaunchKernelGGL(k_trimm_n<256>, dim3(tasks), dim3(256), 0, s, X, n, T, K, part);
  else hipLaunchKernelGGL(k_trimm_n<kTrimmMaxKc>, dim3(tasks), dim3(256), 0, s, X, n, T, K, part);
  hipLaunchKernelGGL(k_trimm_sum<0>, gsum, dim3(64), 0, s, part, n, K, kc, Z);
  return hipGetLastError();
}

// ------------------------------------------------------------------ kept-matrix products
// Split-contraction partials of the kept-matrix product summed in split order:
// out[e] = alpha sum_s part[s][e] + beta_y Y[e].
__global__ __launch_bounds__(256) void k_split_sum(const double* __restrict__ part, int nsplit, int64_t len,
                                                   const double* __restrict__ Y, double alpha, double beta_y,
                                                   double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double s = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) s += part[(int64_t)sp * len + e];
  out[e] = fma(alpha, s, Y ? beta_y * Y[e] : 0.0);
}

// ------------------------------------------------------------------ kept matrix in MFMA-operand order
// The kept matrices of a factor are stored in the order the FP64 16x16x4 MFMA reads its A
// operand: for row tile r (16 rows) and k-group q (4 indices), 64 consecutive doubles, lane
// l = 16 kq + m holding M[16 r + m][4 q + kq].  A wave then loads its operand for one MFMA
// step as one 512-byte coalesced read straight into registers.  Rows are padded with zeros to a
// multiple of 16 and the contraction to a multiple of 32 (whole k-slabs).
int64_t t16_groups(int64_t L) { return (L + 31) / 32 * 8; }   // k-groups of 4, padded to slabs of 32

size_t t16_elems(int64_t M, int64_t L) { return (size_t)((M + 15) / 16) * (size_t)t16_groups(L) * 64; }

__global__ __launch_bounds__(256) void k_to_t16(const double* __restrict__ src, int64_t M, int64_t L, int trans,
                                                int64_t G, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (M + 15) / 16 * G * 64;
  if (e >= total) return;
  const int lane = (int)(e & 63);
  const int64_t grp = e >> 6;
  const int64_t q = grp % G, r = grp / G;
  const int64_t row = 16 * r + (lane & 15), k = 4 * q + (lane >> 4);
  double v = 0.0;
  if (row < M && k < L) v = trans ? src[k * M + row] : src[row * L + k];
  dst[e] = v;
}

hipError_t launch_to_t16(const double* src, int64_t M, int64_t L, int trans, double* dst, hipStream_t s) {
  const int64_t total = (int64_t)t16_elems(M, L);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_t16, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src, M, L, trans,
                     t16_groups(L), dst);
  return hipGetLastError();
}

// out (M x K) = alpha Mt B + beta_y Y, Mt a kept matrix in operand order (M x L), B row-major
// L x K, K <= 64.  Workgroup: 4 waves on 4 row tiles (64 rows) and all 64 columns, one
// contraction range of kper indices (grid.z splits; with more than one, the unscaled partials
// go to part[split][M][K] and k_split_sum adds them in split order).  The B slab (32 x 64)
// goes through LDS, double-buffered, for the 4 waves to share; each wave loads its own A
// operand from HBM into registers two slabs ahead of its use.
constexpr int kT16Slab = 32;

__global__ __launch_bounds__(256) void k_gemm_t16(const double* __restrict__ Mt, int64_t M, int64_t L, int64_t G,
                                                  const double* __restrict__ B, int K, int64_t kper,
                                                  const double* __restrict__ Y, double alpha, double beta_y,
                                                  double* __restrict__ out, double* __restrict__ part) {
  __shared__ double sB[2][kT16Slab][64 + 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int64_t rt = (int64_t)blockIdx.x * 4 + wave;
  const bool rows_ok = rt * 16 < M;
  const int split = blockIdx.z;
  const int64_t kb = (int64_t)split * kper, ke = min(L, kb + kper);
  const double* Ap = Mt + (rows_ok ? rt : 0) * G * 64 + lane;
  double ra0[8], ra1[8], rb[8];
  auto fetch_a = [&](int64_t k0, double* r) {
    const int64_t q0 = k0 >> 2;
#pragma unroll
    for (int j = 0; j < 8; ++j) r[j] = rows_ok ? Ap[(q0 + j) * 64] : 0.0;
  };
  // B slab element f = 256 e + tid (row f / 64, column f % 64): each load instruction of a wave
  // reads one 512-byte row of B, and the LDS writes hit consecutive banks
  auto fetch_b = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int f = 256 * e + tid, c = f & 63;
      const int64_t gk = k0 + (f >> 6);
      rb[e] = (gk < ke && c < K) ? B[gk * K + c] : 0.0;
    }
  };
  auto stash_b = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int f = 256 * e + tid;
      sB[buf][f >> 6][f & 63] = rb[e];
    }
  };
  f64x4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f64x4{0.0, 0.0, 0.0, 0.0};
  auto compute = [&](int buf, const double* r) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 4 * j + kq;
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(r[j], sB[buf][k][16 * b + m], acc[b], 0, 0, 0);
    }
  };
  // A entries past ke inside the last slab multiply B rows that were loaded as zeros
  if (kb < ke) {
    fetch_a(kb, ra0);
    fetch_b(kb);
    stash_b(0);
    if (kb + kT16Slab < ke) {
      fetch_b(kb + kT16Slab);
      fetch_a(kb + kT16Slab, ra1);
    }
  }
  __syncthreads();
  for (int64_t k0 = kb; k0 < ke; k0 += 2 * kT16Slab) {
    compute(0, ra0);                                    // slab k0
    if (k0 + kT16Slab < ke) stash_b(1);                 // slab k0 + 32 (buffer 1 free since the last barrier)
    if (k0 + 2 * kT16Slab < ke) {
      fetch_b(k0 + 2 * kT16Slab);
      fetch_a(k0 + 2 * kT16Slab, ra0);
    }
    __syncthreads();
    if (k0 + kT16Slab >= ke) break;
    compute(1, ra1);                                    // slab k0 + 32
    if (k0 + 2 * kT16Slab < ke) stash_b(0);
    if (k0 + 3 * kT16Slab < ke) {
      fetch_b(k0 + 3 * kT16Slab);
      fetch_a(k0 + 3 * kT16Slab, ra1);
    }
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {   // element v of lane group kq: row 4 v + kq of the tile
      const int64_t row = 16 * rt + 4 * v + kq;
      const int c = 16 * b + m;
      if (row < M && c < K) {
        if (part) part[((int64_t)split * M + row) * K + c] = acc[b][v];
        else out[row * K + c] = fma(alpha, acc[b][v], Y ? beta_y * Y[row * K + c] : 0.0);
      }
    }
}

static int gemm_t16_splits(int64_t M, int64_t L) {
  const int64_t wgs = (M + 63) / 64;
  const int64_t want = (1536 + wgs - 1) / wgs;
  const int64_t cap = std::max<int64_t>(1, L / (4 * kT16Slab));
  return (int)std::max<int64_t>(1, std::min<int64_t>(std::min(want, cap), 64));
}

size_t gemm_t16_work_elems(int64_t M, int64_t L, int K) {
  const int ns = gemm_t16_splits(M, L);
  return ns > 1 ? (size_t)ns * (size_t)M * (size_t)K : 0;
}

hipError_t launch_gemm_t16(const double* Mt, int64_t M, int64_t L, const double* B, int K, const double* Y,
                           double alpha, double beta_y, double* out, double* part, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (K < 1 || K > 64) return hipErrorInvalidValue;
  const int ns = gemm_t16_splits(M, L);
  const int64_t kper = ((L + ns - 1) / ns + kT16Slab - 1) / kT16Slab * kT16Slab;
  const dim3 grid((unsigned)((M + 63) / 64), 1, (unsigned)ns);
  const int64_t G = t16_groups(L);
  if (ns == 1) {
    hipLaunchKernelGGL(k_gemm_t16, grid, dim3(256), 0, s, Mt, M, L, G, B, K, kper, Y, alpha, beta_y, out,
                       (double*)nullptr);
  } else {
    if (!part) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gemm_t16, grid, dim3(256), 0, s, Mt, M, L, G, B, K, kper, Y, alpha, beta_y, out, part);
    const int64_t len = M * K;
    hipLaunchKernelGGL(k_split_sum, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, part, ns, len, Y, alpha,
                       beta_y, out);
  }
  return hipGetLastError();
}

}  // namespace flsq
