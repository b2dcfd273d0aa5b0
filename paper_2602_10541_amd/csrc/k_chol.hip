// Blocked right-looking Cholesky G = U^T U of the regularised Gram (upper triangle,
// row-major, in place), with the inverse built alongside, one block row of W = U^{-T} per step.
//
// Block size kNb = 64.  For each block row k (host loop in fastlsq.cpp):
//   k_trsm_row       U_kj = U_kk^{-T} G_kj for every block column j > k (forward substitution),
//                    and block row k of W from the terms accumulated so far
//   k_syrk_potrf     G_ij -= U_ki^T U_kj over the trailing upper triangle and W_j -= U_kj^T W_k
//                    for the later block rows (FP64 MFMA); the workgroup that owns the next
//                    diagonal block factors it right after updating it
// Block 0 is factored by k_potrf before the loop; k_inv_transpose writes X = D W^T at the end.
//
// The 64 x 64 factorisation runs on one 256-thread workgroup and keeps the block in the
// FP64 MFMA 16x16x4 accumulator layout: wave q holds rows 16q .. 16q + 15 as four 16 x 16
// tiles (lane l, slot v: row 16q + 4v + l / 16, column 16c + l % 16).  Rows are factored four
// at a time by the wave that owns them: the group's four rows pass through LDS into a
// lane-per-column layout, where the four pivots and the couplings inside the group need only
// register reads; the finished rows are published to LDS, and after one barrier
// every wave applies their rank-4 update to its rows below the group as one MFMA per tile.
// The same layout lets the trailing-update kernel apply the last block row's update to the
// next diagonal block in registers and go straight on to its factorisation.
#include "flsq_device.h"
#include "flsq_launch.h"

#include <algorithm>

namespace flsq {

__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffll), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1 / sqrt(x) for x > 0: hardware estimate plus two Newton steps r <- r (3 - x r^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x, r * r, 1.5);
  return r * fma(-0.5 * x, r * r, 1.5);
}

// Diagonal block at k0 into the accumulator layout (wave q: rows 16q + 4v + l / 16, columns
// 16c + l % 16).  Only the upper triangle is read; a short last block (nbk < 64) is padded
// with the identity, which leaves the leading nbk x nbk factor unchanged.
__device__ __forceinline__ void potrf64_load(const double* G, int n, int k0, f64x4 acc[4]) {
  const int nbk = min(kNb, n - k0);
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const double* base = G + (int64_t)k0 * n + k0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * q + 4 * v + (lane >> 4), j = 16 * c + (lane & 15);
      const double g = base[(int64_t)min(i, nbk - 1) * n + min(j, nbk - 1)];   // in bounds, unconditional
      acc[c][v] = (i < nbk && j < nbk && i <= j) ? g : (i == j ? 1.0 : 0.0);
    }
}

// Factor the block held in acc (all 256 threads; S: kNb * kNb doubles of LDS, sbad: two ints
// of LDS) and store the upper triangle of U_kk at k0.
//
// Pivots below `boost` (> 0) are raised to it, the modified Cholesky of Gill and Murray: the
// factor is then exact for G + E with E diagonal, non-zero only at the raised pivots, so a
// Gram that rounding has pushed out of the positive definite cone still factors in one pass;
// their number is added to *nboost.  With boost = 0 a non-positive pivot is a failure instead.
// A failed (or non-finite) pivot is recorded in *info (1-based global index, first failure);
// the rows from it on are then not meaningful (the steps after the failure return at once and
// the attempt is repeated with a shift).  Entries below the diagonal are never stored.
__device__ __forceinline__ void potrf64_factor(f64x4 acc[4], double* G, int n, int k0, int* info, double* S,
                                               int* sbad, double boost, int* nboost) {
  const int nbk = min(kNb, n - k0);
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int r16 = lane & 15, k4 = lane >> 4;
  double* base = G + (int64_t)k0 * n + k0;
  const bool boosting = boost > 0.0;
  if (threadIdx.x == 0) {
    sbad[0] = -1;
    sbad[1] = 0;
  }
#pragma unroll
  for (int g = 0; g < kNb / 4; ++g) {
    const int L = 4 * g, q0 = g >> 2, v0 = g & 3;
    if (q == q0) {
      // rows L .. L + 3 (slot v0 of the four tiles) to one column per lane, through LDS
#pragma unroll
      for (int c = 0; c < 4; ++c) S[(L + k4) * kNb + 16 * c + r16] = acc[c][v0];
      double x[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) x[a] = S[(L + a) * kNb + lane];
      // the group's 4 x 4 pivot block as wave-uniform scalars: its factor is a short scalar chain
      // (one reciprocal square root per pivot), and the four rows follow from it lane-wise
      const double a00 = lane_bcast(x[0], L), a01 = lane_bcast(x[0], L + 1);
      const double a02 = lane_bcast(x[0], L + 2), a03 = lane_bcast(x[0], L + 3);
      const double a11 = lane_bcast(x[1], L + 1), a12 = lane_bcast(x[1], L + 2), a13 = lane_bcast(x[1], L + 3);
      const double a22 = lane_bcast(x[2], L + 2), a23 = lane_bcast(x[2], L + 3);
      const double a33 = lane_bcast(x[3], L + 3);
      // a pivot is raised to boost (boost > 0) or taken as it is: a failed one (non-finite, or
      // non-positive with boost = 0) is recorded below, off the chain, and the attempt abandoned
      const double d0 = a00;
      const double p0 = boosting ? fmax(d0, boost) : d0;
      const double r0 = rsqrt_nr(p0);
      const double u01 = a01 * r0, u02 = a02 * r0, u03 = a03 * r0;
      const double d1 = fma(-u01, u01, a11);
      const double p1 = boosting ? fmax(d1, boost) : d1;
      const double r1 = rsqrt_nr(p1);
      const double u12 = (a12 - u01 * u02) * r1, u13 = (a13 - u01 * u03) * r1;
      const double d2 = fma(-u12, u12, fma(-u02, u02, a22));
      const double p2 = boosting ? fmax(d2, boost) : d2;
      const double r2 = rsqrt_nr(p2);
      const double u23 = (a23 - u02 * u03 - u12 * u13) * r2;
      const double d3 = fma(-u23, u23, fma(-u13, u13, fma(-u03, u03, a33)));
      const double p3 = boosting ? fmax(d3, boost) : d3;
      const double r3 = rsqrt_nr(p3);
      // rows, lane = column: 0 left of the pivot, the pivot's square root on it
      const double U0 = x[0] * r0;
      const double U1 = (x[1] - u01 * U0) * r1;
      const double U2 = (x[2] - u02 * U0 - u12 * U1) * r2;
      const double U3 = (x[3] - u03 * U0 - u13 * U1 - u23 * U2) * r3;
      const double pr[4] = {p0 * r0, p1 * r1, p2 * r2, p3 * r3};
      const double Uv[4] = {U0, U1, U2, U3};
#pragma unroll
      for (int a = 0; a < 4; ++a) x[a] = (lane > L + a) ? Uv[a] : (lane == L + a ? pr[a] : 0.0);
#pragma unroll
      for (int a = 0; a < 4; ++a) S[(L + a) * kNb + lane] = x[a];
      const double dv[4] = {d0, d1, d2, d3};
      int bad = -1, raised = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int l = L + a;
        const bool low = !(dv[a] > boost);
        const bool fail = !isfinite(dv[a]) || (low && !boosting);
        raised += (low && !fail && l < nbk) ? 1 : 0;
        bad = (fail && bad < 0) ? l : bad;
      }
      if (lane == 0 && bad >= 0 && sbad[0] < 0) sbad[0] = bad;
      if (lane == 0) sbad[1] += raised;
    }
    __syncthreads();
    if (g + 1 < kNb / 4) {
      // rows below the group: tile (q, c) -= U_{L..L+3, rows}^T U_{L..L+3, cols}.  Rows at or
      // above the group (all of a wave above the owner) get a zero operand and stay as they
      // are; tiles below the diagonal (c < q) are never read.  Every wave issues the same four
      // products with no branch, which keeps the accumulators in place across the loop.
      const double ar = S[(L + k4) * kNb + 16 * q + r16];
      const double a_op = (16 * q + r16 > L + 3) ? -ar : 0.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double b_op = S[(L + k4) * kNb + 16 * c + r16];
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_op, b_op, acc[c], 0, 0, 0);
      }
    }
  }
  // every row of U_kk is final in S (the last group's barrier above); store the upper
  // triangle once, here: a global store inside the loop would make every barrier wait for it
#pragma unroll
  for (int r = 0; r < kNb / 4; ++r) {
    const int i = 4 * r + q;
    if (i < nbk && lane >= i && lane < nbk) base[(int64_t)i * n + lane] = S[i * kNb + lane];
  }
  const int bad = sbad[0];
  if (threadIdx.x == 0 && bad >= 0 && bad < nbk && *info == 0) *info = k0 + bad + 1;
  if (threadIdx.x == 0 && sbad[1] > 0) atomicAdd(nboost, sbad[1]);
}

__global__ __launch_bounds__(256) void k_potrf(double* G, int n, int k0, int* info, double boost, int* nboost) {
  __shared__ double S[kNb * kNb];
  __shared__ int sbad[2];
  f64x4 acc[4];
  potrf64_load(G, n, k0, acc);
  potrf64_factor(acc, G, n, k0, info, S, sbad, boost, nboost);
}

// Block row: y = U_kk^{-T} g for every column j >= k0 + kNb by forward substitution
// (backward stable, unlike a product with the explicit inverse of U_kk).  Written with the
// unit-diagonal factor: U_kk = D V, D = diag(U_kk), so y = D^{-1} z with z = V^{-T} g,
// z_m = g_m - sum_{l < m} V_lm z_l.
//
// The same launch finishes block row k of W = U^{-T} (the inverse of the lower factor U^T),
// which is built one block row per step alongside the factorisation (U^T W = I read one
// block row at a time): W_k = U_kk^{-T} (I_k - sum_{l < k} U_lk^T W_l).  The bracket has been
// accumulated in W by the trailing updates of the earlier steps (its block k holds the
// identity, taken implicitly); its columns 0 .. k0 + nbk are solved by the same substitution.
// Keeping W = X^T, not X = U^{-1}, makes every access of the inverse a row access, like G's.
//
// Lane m of a wave holds row m; each wave solves kTrsmCols columns at once (independent
// chains).  Step l reads z_l from lane l (a register broadcast) and every lane applies
// one multiply-add per column with its V_lm, which is zero for m <= l so the update
// needs no mask.  V (strictly upper, scaled rows; a short last block is padded with the
// identity) sits in LDS; the workgroup's 64 x 16 slab moves through LDS so that global
// accesses stay coalesced.  Workgroups [0, g_slabs) take 16 columns of G each, the rest 16
// columns of W each.
constexpr int kTrsmCols = 4;
constexpr int kTrsmWaves = 4;
constexpr int kTrsmSlab = kTrsmCols * kTrsmWaves;   // 16 columns per workgroup

__global__ __launch_bounds__(256) void k_trsm_row(double* G, double* W, int n, int k0, int g_slabs,
                                                  const int* info) {
  __shared__ double V[kNb][kNb + 1];
  __shared__ double Y[kNb][kTrsmSlab + 1];
  __shared__ double rinv[kNb];
  const int failed = *info;   // tested once the staging loads are in flight
  const int t = threadIdx.x;
  const int nbk = min(kNb, n - k0);
  const bool wpart = (int)blockIdx.x >= g_slabs;
  // G: columns from k0 + kNb; W: columns [0, k0 + nbk), the block k0 .. k0 + nbk the identity
  double* B = wpart ? W : G;
  const int jbase = wpart ? ((int)blockIdx.x - g_slabs) * kTrsmSlab : k0 + kNb + (int)blockIdx.x * kTrsmSlab;
  const int jend = wpart ? k0 + nbk : n;
  // Every load below reads a clamped, in-bounds address unconditionally and the padding is
  // selected afterwards, so all of them are in flight together (a conditional load would be
  // a branch with a wait of its own).
  // U_kk: thread t covers column t % 64 of rows t / 64 + 4 r (identity past nbk)
  double uv[kNb / 4], yv[kNb / 16];
  {
    const int c = t & 63, cc = min(c, nbk - 1);
#pragma unroll
    for (int r = 0; r < kNb / 4; ++r) {
      const int l = min((t >> 6) + 4 * r, nbk - 1);
      uv[r] = G[(int64_t)(k0 + l) * n + k0 + cc];
    }
  }
  // the slab: 16 threads per row, 16 rows per pass
  {
    const int c = t & (kTrsmSlab - 1);
    const int jc = min(jbase + c, jend - 1);
#pragma unroll
    for (int r = 0; r < kNb / 16; ++r) {
      const int l = min((t >> 4) + 16 * r, nbk - 1);
      yv[r] = B[(int64_t)(k0 + l) * n + jc];
    }
  }
  {
    const int c = t & 63;
#pragma unroll
    for (int r = 0; r < kNb / 4; ++r) {
      const int l = (t >> 6) + 4 * r;
      V[l][c] = (l < nbk && c < nbk) ? uv[r] : (l == c ? 1.0 : 0.0);
    }
  }
  {
    const int c = t & (kTrsmSlab - 1);
    const int j = jbase + c;
#pragma unroll
    for (int r = 0; r < kNb / 16; ++r) {
      const int l = (t >> 4) + 16 * r;
      double v = 0.0;
      if (j < jend && l < nbk) v = (wpart && j >= k0) ? (l == j - k0 ? 1.0 : 0.0) : yv[r];
      Y[l][c] = v;
    }
  }
  __syncthreads();
  if (failed != 0) return;   // a failed pivot: this attempt is abandoned
  if (t < kNb) rinv[t] = 1.0 / V[t][t];
  __syncthreads();
  // V_lm = U_lm / U_ll for m > l, 0 on and below the diagonal
  {
    const int c = t & 63;
#pragma unroll
    for (int r = 0; r < kNb / 4; ++r) {
      const int l = (t >> 6) + 4 * r;
      V[l][c] = (c > l) ? V[l][c] * rinv[l] : 0.0;
    }
  }
  __syncthreads();
  const int m = t & 63, w = t >> 6;
  double z[kTrsmCols];
#pragma unroll
  for (int c = 0; c < kTrsmCols; ++c) z[c] = Y[m][w * kTrsmCols + c];
#pragma unroll
  for (int l = 0; l < kNb - 1; ++l) {
    const double v = V[l][m];
#pragma unroll
    for (int c = 0; c < kTrsmCols; ++c) z[c] = fma(-v, lane_bcast(z[c], l), z[c]);
  }
  const double rm = rinv[m];
#pragma unroll
  for (int c = 0; c < kTrsmCols; ++c) Y[m][w * kTrsmCols + c] = z[c] * rm;
  __syncthreads();
  {
    const int c = t & (kTrsmSlab - 1);
    const int j = jbase + c;
    if (j < jend) {
#pragma unroll
      for (int r = 0; r < kNb / 16; ++r) {
        const int l = (t >> 4) + 16 * r;
        if (l < nbk) B[(int64_t)(k0 + l) * n + j] = Y[l][c];
      }
    }
  }
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

// Trailing update with the KR (64 or 128) just-solved panel rows k0 .. k0 + KR of U, over rows
// and columns [k1, n), k1 = k0 + KR: G_ij -= sum_l U_{k0+l,i} U_{k0+l,j}, i <= j, in 128 x 128
// tiles (ti <= tj), one workgroup per tile: wave w computes the 64 x 64 quadrant (w / 2, w % 2)
// with FP64 MFMA 16x16x4.  With W = U^{-T} given, the same launch applies the panel's terms of
// the inverse to the later block rows, W_j -= sum_l U_{k0+l,j}^T W_{k0+l} for the rows [k1, n)
// and the columns [0, k1), in 128 x 128 tiles after the triangle's; it has the triangle's form,
// with W's panel rows as the second operand.  With row_lim < n only the rows [k1, row_lim)
// (the next block row: tile row 0) are updated, in both G and W.
//
// Block rows are taken in pairs: the next block row alone (KR = 64, row_lim = k1 + 64), then,
// once it is solved too, the rest with both (KR = 128): the trailing matrix is read and written
// once per pair, which halves the HBM traffic of the updates at the cost of one small launch.
//
// The operands come straight from the panels into registers in the order the matrix cores
// consume them: the operand of k-step kk for 16 columns from c0 is one load whose lane l
// reads panel row 4 kk + l / 16, column c0 + l % 16 (four 128-byte pieces).  Each wave keeps
// the loads of the next two k-steps in flight while it multiplies, and nothing is staged in
// LDS, so two workgroups share a CU: one's loads overlap the other's products, and a step
// with up to twice as many tiles as CUs still runs in one round.
//
// Workgroup 0 owns the next diagonal block (quadrant (0, 0) of tile (0, 0), which the tile's
// own workgroup skips): it loads the block straight into the accumulator layout of the
// factorisation, applies the update there and factors it without a round trip through
// memory, so the critical path of a step is one update of one block plus its factorisation.
constexpr int kSyrkRing = 3;   // k-steps of operands held in registers (two in flight)

__device__ __forceinline__ double syrk_operand(const double* P, int n, int kk, int c0, int lane) {
  return P[(int64_t)(4 * kk + (lane >> 4)) * n + min(c0 + (lane & 15), n - 1)];
}

// One 64 x 64 quadrant: C[i0.., j0..] -= PA[:, i0..]^T PB[:, j0..] over the KR panel rows;
// only entries with i < row_end, j < col_end (and j >= i when TRI) are touched.  The old values are
// read after the products, 16 per lane at a time with the next 16 already in flight, from
// clamped in-bounds addresses (a conditional load would wait on its own); reading them up
// front instead delays the next diagonal block's loads, which are on the critical path.
template <bool TRI, int KR>
__device__ __forceinline__ void syrk_quadrant(double* C, const double* PA, const double* PB, int n, int i0, int j0,
                                              int row_end, int col_end, int lane) {
  const int r16 = lane & 15, k4 = lane >> 4;
  f64x4 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = f64x4{0.0, 0.0, 0.0, 0.0};
  double ra[kSyrkRing][4], rb[kSyrkRing][4];
  auto fetch = [&](int kk, int slot) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ra[slot][r] = syrk_operand(PA, n, kk, i0 + 16 * r, lane);
      rb[slot][r] = syrk_operand(PB, n, kk, j0 + 16 * r, lane);
    }
  };
  fetch(0, 0);
  fetch(1, 1);
#pragma unroll
  for (int kk = 0; kk < KR / 4; ++kk) {
    if (kk + 2 < KR / 4) fetch(kk + 2, (kk + 2) % kSyrkRing);
    const int s = kk % kSyrkRing;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[s][r], rb[s][c], acc[r][c], 0, 0, 0);
  }
  double old[2][16];
  auto load_old = [&](int r, int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 16 * r + 4 * v + k4;
        const int j = j0 + 16 * c + r16;
        old[buf][4 * c + v] = C[(int64_t)min(i, row_end - 1) * n + min(j, col_end - 1)];
      }
  };
  load_old(0, 0);
  load_old(1, 1);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int buf = r & 1;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 16 * r + 4 * v + k4;
        const int j = j0 + 16 * c + r16;
        if (i < row_end && j < col_end && (!TRI || j >= i)) C[(int64_t)i * n + j] = old[buf][4 * c + v] - acc[r][c][v];
      }
    if (r + 2 < 4) load_old(r + 2, buf);
  }
}

template <int KR>
__global__ __launch_bounds__(256, 2) void k_syrk_potrf(double* G, double* W, int n, int k0, int row_lim, int* info,
                                                       double boost, int* nboost) {
  __shared__ double S[kNb * kNb];
  __shared__ int sbad[2];
  const int failed = *info;   // a failed pivot abandons the attempt; tested once loads are out
  const int k1 = k0 + KR;
  const int nt = (n - k1 + 127) / 128;
  const bool strip = row_lim < n;
  const int ntri = strip ? nt : nt * (nt + 1) / 2;   // a strip keeps tile row 0 only
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double* P = G + (int64_t)k0 * n;   // the panel: rows k0 .. k0 + KR
  if (blockIdx.x == 0) {
    // the next diagonal block: its update in registers, then its factorisation.  Columns past
    // n read column n - 1 (clamped) and only touch the identity padding, which is never stored.
    f64x4 acc[4];
    potrf64_load(G, n, k1, acc);
    double ra[kSyrkRing], rb[kSyrkRing][4];
    auto fetch = [&](int kk, int slot) {
      ra[slot] = syrk_operand(P, n, kk, k1 + 16 * wave, lane);
#pragma unroll
      for (int c = 0; c < 4; ++c) rb[slot][c] = syrk_operand(P, n, kk, k1 + 16 * c, lane);
    };
    fetch(0, 0);
    fetch(1, 1);
    if (failed != 0) return;
    // all four tiles of every wave, with no branch: tiles below the diagonal (c < wave) take
    // the update too and are never read
#pragma unroll
    for (int kk = 0; kk < KR / 4; ++kk) {
      if (kk + 2 < KR / 4) fetch(kk + 2, (kk + 2) % kSyrkRing);
      const int s = kk % kSyrkRing;
      const double a = -ra[s];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, rb[s][c], acc[c], 0, 0, 0);
    }
    potrf64_factor(acc, G, n, k1, info, S, sbad, boost, nboost);
    return;
  }
  if (failed != 0) return;
  const int qi = wave >> 1, qj = wave & 1;
  const int b = (int)blockIdx.x - 1;
  if (b < ntri) {
    int ti = 0, tj = b;
    if (!strip) tri_coords(b, nt, &ti, &tj);
    const int i0 = k1 + ti * 128 + qi * 64, j0 = k1 + tj * 128 + qj * 64;
    // quadrant (0, 0) of tile (0, 0) is the next diagonal block (workgroup 0)
    const bool active = !(ti == tj && qi > qj) && !(ti == 0 && tj == 0 && qi == 0 && qj == 0) && i0 < row_lim &&
                        j0 < n;
    if (active) syrk_quadrant<true, KR>(G, P, P, n, i0, j0, row_lim, n, lane);
  } else {
    // W tile: rows [k1, row_lim) (the later block rows), columns [0, k1); a strip has one row
    const int wb = b - ntri;
    const int wr = strip ? 0 : wb % nt, wc = strip ? wb : wb / nt;
    const int i0 = k1 + wr * 128 + qi * 64, j0 = wc * 128 + qj * 64;
    if (i0 < row_lim && j0 < k1) syrk_quadrant<false, KR>(W, P, W + (int64_t)k0 * n, n, i0, j0, row_lim, k1, lane);
  }
}

// X = D W^T (X[i][j] = d_i W[j][i] for j >= i, 0 below the diagonal; d nullable = ones):
// 64 x 64 tiles through LDS, both sides read and written along rows.  Nothing is written when
// the factorisation's status (*info) reports a failed pivot.
__global__ __launch_bounds__(256) void k_inv_transpose(const double* __restrict__ W, const double* __restrict__ d,
                                                       int n, const int* __restrict__ info, double* __restrict__ X) {
  __shared__ double T[64][65];
  if (*info != 0) return;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;   // the tile X[i0.., j0..]
  const int t = threadIdx.x, c = t & 63;
  if (j0 + 63 < i0) {   // entirely below the diagonal
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = i0 + (t >> 6) + 4 * r, j = j0 + c;
      if (i < n && j < n) X[(int64_t)i * n + j] = 0.0;
    }
    return;
  }
  double w[16];   // all loads in flight together: clamped in-bounds addresses, padding selected after
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int j = j0 + (t >> 6) + 4 * r, i = i0 + c;   // W row j, column i
    w[r] = W[(int64_t)min(j, n - 1) * n + min(i, n - 1)];
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int jr = (t >> 6) + 4 * r;
    T[jr][c] = (i0 + c < n && j0 + jr < n) ? w[r] : 0.0;
  }
  double dv[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) dv[r] = d ? d[min(i0 + (t >> 6) + 4 * r, n - 1)] : 1.0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int ir = (t >> 6) + 4 * r;
    const int i = i0 + ir, j = j0 + c;
    if (i < n && j < n) X[(int64_t)i * n + j] = (j >= i) ? dv[r] * T[c][ir] : 0.0;
  }
}

hipError_t launch_potrf(double* G, int n, int k0, int* info, double boost, int* nboost, hipStream_t s) {
  hipLaunchKernelGGL(k_potrf, dim3(1), dim3(256), 0, s, G, n, k0, info, boost, nboost);
  return hipGetLastError();
}

hipError_t launch_trsm_row(double* G, double* W, int n, int k0, const int* info, hipStream_t s) {
  if (k0 < 0 || k0 >= n) return hipErrorInvalidValue;
  const int cols = n - k0 - kNb;
  const int g_slabs = cols > 0 ? (cols + kTrsmSlab - 1) / kTrsmSlab : 0;
  const int wcols = k0 + std::min(kNb, n - k0);
  const int w_slabs = W ? (wcols + kTrsmSlab - 1) / kTrsmSlab : 0;
  if (g_slabs + w_slabs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_trsm_row, dim3(g_slabs + w_slabs), dim3(256), 0, s, G, W, n, k0, g_slabs, info);
  return hipGetLastError();
}

hipError_t launch_syrk_potrf(double* G, double* W, int n, int k0, int kr, int row_lim, int* info, double boost,
                             int* nboost, hipStream_t s) {
  if (kr != 64 && kr != 128) return hipErrorInvalidValue;
  const int k1 = k0 + kr;
  const int rem = n - k1;
  if (rem <= 0) return hipSuccess;
  row_lim = std::min(std::max(row_lim, k1), n);
  const int nt = (rem + 127) / 128;
  const bool strip = row_lim < n;
  const int ntri = strip ? nt : nt * (nt + 1) / 2;
  const int wrows = strip ? 1 : nt;
  const int wt = W ? (k1 + 127) / 128 * wrows : 0;
  const dim3 grid(1 + ntri + wt);
  if (kr == 64)
    hipLaunchKernelGGL(k_syrk_potrf<64>, grid, dim3(256), 0, s, G, W, n, k0, row_lim, info, boost, nboost);
  else
    hipLaunchKernelGGL(k_syrk_potrf<128>, grid, dim3(256), 0, s, G, W, n, k0, row_lim, info, boost, nboost);
  return hipGetLastError();
}

hipError_t launch_inv_transpose(const double* W, const double* d, int n, const int* info, double* X, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((n + 63) / 64);
  hipLaunchKernelGGL(k_inv_transpose, dim3(nb, nb), dim3(256), 0, s, W, d, n, info, X);
  return hipGetLastError();
}


}  // namespace flsq
