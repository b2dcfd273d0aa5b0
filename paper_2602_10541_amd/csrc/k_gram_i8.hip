// Gram product A^T A from exact integer products on the int8 matrix cores.
//
// Every entry of A (Eq. (2)-(3), amplitude/phase form of flsq_device.h) is formed in
// FP64, scaled per feature to an integer a_ij = rint(A_ij 2^B / c_j) with |a_ij| <= 2^B
// (c_j bounds |A_ij| over all rows: max over blocks of |amp_gj| plus max |rho_i|), and
// represented by its balanced residues modulo a set of pairwise coprime odd moduli
// p_t <= 255, each of which fits in int8.  For every modulus the integer Gram
// sum_i r_ij r_il is exact in int32 (|r| <= 127, so up to 133 000 rows), and the
// Chinese remainder theorem recovers sum_i a_ij a_il exactly as long as the product of
// the moduli exceeds twice its magnitude.  The only rounding is that of A to B bits and
// of the final conversion to FP64: with B ~ 42 the Gram is as accurate as an FP64
// product, at int8 matrix-core rate.
//
//   k_i8_scale      c_j and 2^B / c_j per feature
//   k_i8_residues   residues of the scaled entries, int8, K-blocked [t][kb][feature][64 rows]
//   k_gram_i8       per modulus, the upper-triangle 256 x 256 tiles of R_t^T R_t (int32)
//   k_i8_crt        balanced mixed-radix (Garner) reconstruction, FP64 Horner, scaling
#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

constexpr int kI8Tile = 256;    // features per tile side
constexpr int kI8Kb = 64;       // rows per K block of the residue layout

// ------------------------------------------------------------------ scales
// rho_max (nullable): device scalar max_i |rho_i|.
__global__ void k_i8_scale(const double* amp, int n_blocks, int n, const double* rho_max, double two_b,
                           double* inv_scale, double* scale) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  double c = 0.0;
  for (int g = 0; g < n_blocks; ++g) c = fmax(c, fabs(amp[(int64_t)g * n + f]));
  if (rho_max) c += *rho_max;
  inv_scale[f] = (c > 0.0) ? two_b / c : 0.0;
  scale[f] = (c > 0.0) ? c / two_b : 0.0;
}

// max |x_i| over n entries (one workgroup; deterministic).
__global__ __launch_bounds__(1024) void k_absmax(const double* x, int64_t n, double* out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, fabs(x[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// ------------------------------------------------------------------ residues
// Workgroup: 32 features x one 64-row K block; thread (feature tid / 8, rows 8 (tid % 8) ..),
// so the eight threads of a feature store its 64 bytes per modulus side by side.
// R layout: R[((t * KB + kb) * n_pad + f) * 64 + r], zero for padded rows and features.
//
// Residue bytes: for the integer a (|a| <= 2^46, as B <= 46 for every admissible row count) and
// an odd modulus p, q = rint(a / p) is fma(a, 1/p, 1.5 * 2^52) - 1.5 * 2^52: the exact product
// lies within 2^-14 of a / p, which itself is at least 1 / (2p) away from any half-integer, so
// the single rounding of the fma gives q, and the low 32 bits of the biased double are q
// modulo 2^32.  The balanced residue a - p q lies in [-(p-1)/2, (p-1)/2], so its int8 byte is
// (a - p q) mod 256 = (a mod 2^32 + (256 - p) (q mod 2^24)) mod 256: one FP64 fma and one
// 24-bit integer multiply-add per entry and modulus.
//
// With Y given (P doubles), the same pass also forms the block's part of c = A^T Y from the
// FP64 entries before they are scaled: cpart[kb * n_pad + f] = sum over the block's rows (8
// rows per thread in order, then the eight threads of a feature pairwise), summed over kb by
// k_colsum_parts.
constexpr double kBias52 = 6755399441055744.0;   // 1.5 * 2^52

__device__ __forceinline__ unsigned low_word(double x) { return (unsigned)__double_as_longlong(x); }

// a * b + c on the low 24 bits of a and b (full-rate v_mad_u32_u24; written out because the
// compiler, seeing that only the low byte of the result is used, would otherwise widen the
// product to a quarter-rate 32-bit multiply).
__device__ __forceinline__ unsigned mad_u24(unsigned a, unsigned b, unsigned c) {
  unsigned d;
  asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
  return d;
}

template <int D>
__global__ __launch_bounds__(256) void k_i8_residues(Geo g, const double* rho, const double* inv_scale, I8Moduli M,
                                                     int n_pad, int KB, int8_t* R, const double* Y, double* cpart) {
  __shared__ double sX[D][kI8Kb];
  __shared__ double sRho[kI8Kb];
  __shared__ double sY[kI8Kb];
  __shared__ int sOff[kI8Kb];   // the row's block offset blk * n into amp and ph, -1 past the rows
  const int kb = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)kb * kI8Kb;
  for (int e = tid; e < D * kI8Kb; e += 256) {
    const int k = e / kI8Kb, r = e % kI8Kb;
    sX[k][r] = (i0 + r < g.P) ? g.Xt[(int64_t)k * g.P + i0 + r] : 0.0;
  }
  if (tid < kI8Kb) {
    const bool in = i0 + tid < g.P;
    sRho[tid] = (rho && in) ? rho[i0 + tid] : 0.0;
    sY[tid] = (Y && in) ? Y[i0 + tid] : 0.0;
    sOff[tid] = in ? g.row_block[i0 + tid] * g.n : -1;   // n_blocks * n < 2^31 (checked by the host)
  }
  __syncthreads();
  const SinPoly sp = sin_poly_sgpr();
  const int f = blockIdx.y * 32 + tid / 8;
  const int r0 = 8 * (tid % 8);
  const bool fvalid = f < g.n;
  double w[D];
#pragma unroll
  for (int k = 0; k < D; ++k) w[k] = fvalid ? g.Wt[(int64_t)k * g.n + f] : 0.0;
  const double isc = fvalid ? inv_scale[f] : 0.0;
  double a[8];
  unsigned alo[8];
  double cy = 0.0;
  const int fc = min(f, g.n - 1);
  const double* __restrict__ ph_f = g.ph + fc;
  const double* __restrict__ amp_f = g.amp + fc;
#pragma unroll
  for (int r = 0; r < 8; ++r) {   // branch-free: padded rows and features read a valid entry, then drop it
    const int off = sOff[r0 + r];
    const unsigned o = (unsigned)max(off, 0);
    double z = ph_f[o];
#pragma unroll
    for (int k = 0; k < D; ++k) z = fma(w[k], sX[k][r0 + r], z);
    const double e = (fvalid && off >= 0) ? (amp_f[o] + sRho[r0 + r]) * sin_f64(z, sp) : 0.0;
    cy = fma(e, sY[r0 + r], cy);
    const double v = rint(e * isc);
    a[r] = v;
    alo[r] = low_word(v + kBias52);
  }
  if (cpart) {   // the eight threads of a feature are adjacent lanes
    cy += __shfl_xor(cy, 1);
    cy += __shfl_xor(cy, 2);
    cy += __shfl_xor(cy, 4);
    if ((tid & 7) == 0) cpart[(int64_t)kb * n_pad + f] = cy;
  }
  int8_t* dst = R + ((int64_t)kb * n_pad + f) * kI8Kb + r0;
  const int64_t tstride = (int64_t)KB * n_pad * kI8Kb;
#pragma unroll
  for (int t = 0; t < kI8MaxMod; ++t) {   // unrolled: the moduli's scalar loads are issued up front
    if (t < M.n_mod) {
      const double ip = M.inv_p[t];
      const unsigned pc = 256u - (unsigned)M.ip[t];
      unsigned pk[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        unsigned word = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const unsigned q = low_word(fma(a[4 * h + e], ip, kBias52));
          const unsigned b = mad_u24(q, pc, alo[4 * h + e]);
          word |= (b & 0xffu) << (8 * e);
        }
        pk[h] = word;
      }
      *(uint2*)(dst + t * tstride) = make_uint2(pk[0], pk[1]);
    }
  }
}

// ------------------------------------------------------------------ int8 Gram tiles
// Workgroup = one upper tile (ti <= tj) of one modulus, 4 waves in 2 x 2, each wave a
// 128 x 128 quarter as 4 x 4 blocks of v_mfma_i32_32x32x32_i8.  Both operands are
// residues of the same matrix with rows on the contraction axis, so a lane's 16 bytes
// are 16 consecutive rows of one feature for the A and the B side alike.
//
// Tiles are taken in the order of J.order (4 x 4 super-tiles, modulus-major), and
// consecutive workgroup ids, which the hardware deals round-robin to the 8 XCDs, are
// remapped so that each XCD works through a contiguous stretch of that order: the
// workgroups resident on one XCD then share row and column panels in its L2.
//
// Pipeline: a ring of kI8Ring LDS slots, one 64-row K block each, filled by direct
// global-to-LDS loads (no staging registers) up to kI8Ring - 1 blocks ahead of the
// matrix cores.  Each wave waits for its own loads of a block with an explicit vmcnt and
// a plain s_barrier then makes every wave's loads visible.  A slot is refilled only after
// the barrier that follows the last reads of the block it held.  In a slot, panel p holds 256
// features x 4 granules of 16 bytes (16 rows each); granule g of feature f sits at
// position 4 f + (g ^ ((f >> 2) & 3)), so the 16-lane passes of the operand reads hit
// distinct LDS banks.
constexpr int kI8Ring = 4;
constexpr int kI8Slot = 2 * kI8Tile * kI8Kb;     // bytes per ring slot (two panels)

#define FLSQ_VMCNT(n) __builtin_amdgcn_s_waitcnt(((n) & 15) | (((n) >> 4) << 14) | (7 << 4) | (15 << 8))
#define FLSQ_SBARRIER() asm volatile("s_barrier" ::: "memory")

__device__ __forceinline__ int i8_swz(int f, int g) { return 4 * f + (g ^ ((f >> 2) & 3)); }

__device__ __forceinline__ void i8_dma(unsigned char* smem, const int8_t* baseA, const int8_t* baseB,
                                       int64_t kb_stride, int kb, int step, int wave, int lane) {
  unsigned char* slot = smem + (step % kI8Ring) * kI8Slot;
#pragma unroll
  for (int panel = 0; panel < 2; ++panel)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // one instruction of a wave fills 64 consecutive granules (1 KB) of the panel
      const int p = (q * 4 + wave) * 64 + lane;
      const int f = p >> 2, g = (p & 3) ^ ((f >> 2) & 3);
      const int8_t* src = (panel ? baseB : baseA) + (int64_t)kb * kb_stride + f * kI8Kb + g * 16;
      unsigned char* dst = slot + panel * (kI8Tile * kI8Kb) + (q * 4 + wave) * 1024;
      __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
}

// Operand fragments of one 32-row group (ks) of K block kb: 4 A and 4 B blocks.
__device__ __forceinline__ void i8_frags(i32x4 (&av)[4], i32x4 (&bv)[4], const unsigned char* smem, int kb, int ks,
                                         int wm, int wn, int lane) {
  const unsigned char* pA = smem + (kb % kI8Ring) * kI8Slot;
  const unsigned char* pB = pA + kI8Tile * kI8Kb;
  const int g = 2 * ks + (lane >> 5);
#pragma unroll
  for (int a = 0; a < 4; ++a) av[a] = *(const i32x4*)(pA + 16 * i8_swz(wm * 128 + a * 32 + (lane & 31), g));
#pragma unroll
  for (int b = 0; b < 4; ++b) bv[b] = *(const i32x4*)(pB + 16 * i8_swz(wn * 128 + b * 32 + (lane & 31), g));
}

__device__ __forceinline__ void i8_mma16(i32x16 (&acc)[4][4], const i32x4 (&av)[4], const i32x4 (&bv)[4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(av[a], bv[b], acc[a][b], 0, 0, 0);
}

__global__ __launch_bounds__(256, 1) void k_gram_i8(I8GemmJob J) {
  extern __shared__ __align__(16) unsigned char smem[];   // kI8Ring slots of kI8Slot bytes
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int total = J.n_tiles * J.n_mod;
  int wg = blockIdx.x;
  const int full = (total / 8) * 8;
  if (wg < full) wg = (wg % 8) * (total / 8) + wg / 8;
  const int t = wg / J.n_tiles;
  const int2 tc = J.order[wg % J.n_tiles];
  const int ti = tc.x, tj = tc.y;
  const int tile = ti * J.nt - ti * (ti - 1) / 2 + (tj - ti);   // row-major slot of (ti, tj)
  const int8_t* baseA = J.R + ((int64_t)t * J.KB * J.n_pad + (int64_t)ti * kI8Tile) * kI8Kb;
  const int8_t* baseB = J.R + ((int64_t)t * J.KB * J.n_pad + (int64_t)tj * kI8Tile) * kI8Kb;
  const int64_t kb_stride = (int64_t)J.n_pad * kI8Kb;

  i32x16 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0;

  const int nkb = J.KB;
  // Every step issues its refill, also past the last block: such a load re-reads block
  // nkb - 1 into the slot it is due (one no longer read), so the count of loads in flight is
  // the same at every wait and the loop body has no branch (the compiler then spreads the
  // refill's address arithmetic among the products: 5 % faster than conditional refills).
#pragma unroll
  for (int kb = 0; kb < kI8Ring - 1; ++kb) i8_dma(smem, baseA, baseB, kb_stride, min(kb, nkb - 1), kb, wave, lane);
  // Wait until block kb has landed in LDS for every wave: each wave's own loads of it are
  // done once at most those of the two later blocks already issued remain.
  auto block_ready = [&]() {
    FLSQ_VMCNT(16);
    FLSQ_SBARRIER();
  };
  i32x4 a0[4], b0[4], a1[4], b1[4];
  block_ready();
  i8_dma(smem, baseA, baseB, kb_stride, min(kI8Ring - 1, nkb - 1), kI8Ring - 1, wave, lane);
  i8_frags(a0, b0, smem, 0, 0, wm, wn, lane);
  // Per block: the second group's fragments load under the first group's products; the
  // next block's barrier, its refill of the slot freed by the previous block, and its
  // first fragments happen under the second group's products.
  // (the last block is peeled off so that the loop body has no join between the loads of
  // the next block's fragments and their use: the LDS counter then waits for exactly the
  // fragments each group needs)
  for (int kb = 0; kb + 1 < nkb; ++kb) {
    i8_frags(a1, b1, smem, kb, 1, wm, wn, lane);
    i8_mma16(acc, a0, b0);
    block_ready();
    i8_dma(smem, baseA, baseB, kb_stride, min(kb + kI8Ring, nkb - 1), kb + kI8Ring, wave, lane);
    i8_frags(a0, b0, smem, kb + 1, 0, wm, wn, lane);
    i8_mma16(acc, a1, b1);
  }
  i8_frags(a1, b1, smem, nkb - 1, 1, wm, wn, lane);
  i8_mma16(acc, a0, b0);
  i8_mma16(acc, a1, b1);
  FLSQ_VMCNT(0);   // the refills past the last block land before the workgroup ends
  // 32 x 32 block layout: slot v is row 8 (v / 4) + 4 (lane / 32) + v % 4, column lane % 32
  int32_t* out = J.out + ((int64_t)t * J.n_tiles + tile) * (kI8Tile * kI8Tile);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = wm * 128 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = wn * 128 + b * 32 + (lane & 31);
        out[row * kI8Tile + col] = acc[a][b][v];
      }
}

// ------------------------------------------------------------------ reconstruction
// Balanced remainders r = x - p rint(x / p) in [-(p-1)/2, (p-1)/2] (p odd): x / p is never a
// half-integer, and the rounded quotient lies within far less than 1/(2p) of the exact
// one, so rint is exact; the remainder is then exact in the format (|x| < 2^24 for FP32).
__device__ __forceinline__ int bal_mod_f64(int x, double p, double ip) {
  const double fx = (double)x;
  return (int)fma(-p, rint(fx * ip), fx);
}
__device__ __forceinline__ float bal_modf(float y, float p, float ip) { return fmaf(-p, rintf(y * ip), y); }

// One thread per upper-triangle entry (j <= l) of G (n x n row-major): balanced Garner
// digits v_k of the residues, X = v_0 + p_0 (v_1 + p_1 (v_2 + ...)) evaluated from the top
// in FP64 (a small |X| has leading zero digits, so nothing cancels), G_jl = X s_j s_l.
__global__ void k_i8_crt(I8CrtJob J) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (l >= J.n || l < j) return;
  const int ti = j / kI8Tile, tj = l / kI8Tile;
  const int tile = ti * J.nt - ti * (ti - 1) / 2 + (tj - ti);
  const int64_t e = (int64_t)tile * (kI8Tile * kI8Tile) + (j % kI8Tile) * kI8Tile + (l % kI8Tile);
  const int64_t tstride = (int64_t)J.n_tiles * (kI8Tile * kI8Tile);
  float v[kI8MaxMod];
#pragma unroll
  for (int k = 0; k < kI8MaxMod; ++k) {
    if (k < J.M.n_mod) {
      const float pk = J.M.pf[k], ipk = J.M.inv_pf[k];
      // |sum| < 2^31: the first reduction in FP64; the digit recurrence stays in FP32, where
      // every value is an integer below 2^16 in magnitude (|x - v| < 255, cinv < 255), so
      // each product and remainder is exact
      float x = (float)bal_mod_f64(J.Gt[k * tstride + e], J.M.p[k], J.M.inv_p[k]);
#pragma unroll
      for (int m = 0; m < kI8MaxMod; ++m)
        if (m < k) x = bal_modf((x - v[m]) * J.M.cinvf[m][k], pk, ipk);
      v[k] = x;
    }
  }
  double X = 0.0;
#pragma unroll
  for (int k = kI8MaxMod - 1; k >= 0; --k)
    if (k < J.M.n_mod) X = fma(X, J.M.p[k], (double)v[k]);
  double gv = X * J.scale[j] * J.scale[l];
  if (j == l) gv += J.diag_add;
  J.G[(int64_t)j * J.n + l] = gv;
  if (J.mirror && j != l) J.G[(int64_t)l * J.n + j] = gv;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_i8_scale(const double* amp, int n_blocks, int n, const double* rho, int64_t P, double* rho_max,
                           int B, double* inv_scale, double* scale, hipStream_t s) {
  if (rho) hipLaunchKernelGGL(k_absmax, dim3(1), dim3(1024), 0, s, rho, P, rho_max);
  hipLaunchKernelGGL(k_i8_scale, dim3((n + 255) / 256), dim3(256), 0, s, amp, n_blocks, n,
                     rho ? (const double*)rho_max : nullptr, ldexp(1.0, B), inv_scale, scale);
  return hipGetLastError();
}

// c[f] = sum over kb of cpart[kb * n_pad + f], f < n: 64 features per workgroup, sixteen waves
// each summing every sixteenth kb, the sixteen sums then added in a fixed order.
__global__ __launch_bounds__(1024) void k_colsum_parts(const double* __restrict__ cpart, int KB, int n_pad, int n,
                                                       double* __restrict__ c) {
  __shared__ double red[16][64];
  const int fl = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int f = blockIdx.x * 64 + fl;
  double acc = 0.0;
  if (f < n) {
#pragma unroll 4
    for (int kb = grp; kb < KB; kb += 16) acc += cpart[(int64_t)kb * n_pad + f];
  }
  red[grp][fl] = acc;
  __syncthreads();
  if (grp == 0 && f < n) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += red[q][fl];
    c[f] = t;
  }
}

hipError_t launch_i8_residues(const Geo& g, const double* rho, const double* inv_scale, const I8Moduli& M, int n_pad,
                              int KB, int8_t* R, const double* Y, double* cpart, double* c, hipStream_t s) {
  const dim3 grid(KB, n_pad / 32);
  if ((Y == nullptr) != (cpart == nullptr) || (cpart == nullptr) != (c == nullptr)) return hipErrorInvalidValue;
  switch (g.d) {
#define FLSQ_I8R(D) \
  case D:           \
    hipLaunchKernelGGL(k_i8_residues<D>, grid, dim3(256), 0, s, g, rho, inv_scale, M, n_pad, KB, R, Y, cpart); break;
    FLSQ_I8R(1) FLSQ_I8R(2) FLSQ_I8R(3) FLSQ_I8R(4) FLSQ_I8R(5) FLSQ_I8R(6) FLSQ_I8R(7) FLSQ_I8R(8)
#undef FLSQ_I8R
    default:
      return hipErrorInvalidValue;
  }
  if (c) hipLaunchKernelGGL(k_colsum_parts, dim3((g.n + 63) / 64), dim3(1024), 0, s, cpart, KB, n_pad, g.n, c);
  return hipGetLastError();
}

size_t i8_gemm_lds_bytes() { return (size_t)kI8Ring * kI8Slot; }

hipError_t launch_gram_i8(const I8GemmJob& J, hipStream_t s) {
  if (J.KB < 1) return hipErrorInvalidValue;   // the pipeline reads block KB - 1
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_gram_i8, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)i8_gemm_lds_bytes());
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(k_gram_i8, dim3(J.n_tiles * J.n_mod), dim3(256), i8_gemm_lds_bytes(), s, J);
  return hipGetLastError();
}

// The same reconstruction for the library's fixed set of 13 moduli, with every modulus,
// reciprocal and Garner inverse a compile-time constant: the generic kernel reads the 78
// inverses from its arguments through scalar loads between the dependent multiply-adds.
// The arithmetic (operations, operands and their order) is the generic kernel's.
constexpr int kCrtMods[13] = {255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199};

struct CrtInv {
  int v[13][13];
};
constexpr CrtInv crt_inverses() {
  CrtInv t{};
  for (int a = 0; a < 13; ++a)
    for (int k = a + 1; k < 13; ++k)
      for (int x = 1; x < kCrtMods[k]; ++x)
        if ((kCrtMods[a] % kCrtMods[k]) * x % kCrtMods[k] == 1) {
          t.v[a][k] = x;
          break;
        }
  return t;
}
constexpr CrtInv kCrtInv = crt_inverses();

template <int K, int M>
__device__ __forceinline__ float crt_inner(float x, const float (&v)[13]) {
  if constexpr (M < K) {
    constexpr float pk = (float)kCrtMods[K];
    constexpr float ipk = 1.0f / pk;
    constexpr float ci = (float)kCrtInv.v[M][K];
    return crt_inner<K, M + 1>(bal_modf((x - v[M]) * ci, pk, ipk), v);
  } else {
    return x;
  }
}

template <int K>
__device__ __forceinline__ void crt_digits(float (&v)[13], const int (&g)[13]) {
  constexpr double p = (double)kCrtMods[K];
  constexpr double ip = 1.0 / p;
  v[K] = crt_inner<K, 0>((float)bal_mod_f64(g[K], p, ip), v);
  if constexpr (K + 1 < 13) crt_digits<K + 1>(v, g);
}

__global__ void k_i8_crt13(I8CrtJob J) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (l >= J.n || l < j) return;
  const int ti = j / kI8Tile, tj = l / kI8Tile;
  const int tile = ti * J.nt - ti * (ti - 1) / 2 + (tj - ti);
  const int64_t e = (int64_t)tile * (kI8Tile * kI8Tile) + (j % kI8Tile) * kI8Tile + (l % kI8Tile);
  const int64_t tstride = (int64_t)J.n_tiles * (kI8Tile * kI8Tile);
  int g[13];
#pragma unroll
  for (int k = 0; k < 13; ++k) g[k] = J.Gt[k * tstride + e];
  float v[13];
  crt_digits<0>(v, g);
  double X = 0.0;
#pragma unroll
  for (int k = 12; k >= 0; --k) X = fma(X, (double)kCrtMods[k], (double)v[k]);
  double gv = X * J.scale[j] * J.scale[l];
  if (j == l) gv += J.diag_add;
  J.G[(int64_t)j * J.n + l] = gv;
  if (J.mirror && j != l) J.G[(int64_t)l * J.n + j] = gv;
}

hipError_t launch_i8_crt(const I8CrtJob& J, hipStream_t s) {
  bool fixed = J.M.n_mod == 13;
  for (int t = 0; fixed && t < 13; ++t) fixed = J.M.ip[t] == kCrtMods[t];
  for (int a = 0; fixed && a < 13; ++a)
    for (int k = a + 1; k < 13; ++k) fixed = fixed && J.M.cinv[a][k] == kCrtInv.v[a][k];
  if (fixed)
    hipLaunchKernelGGL(k_i8_crt13, dim3((J.n + 255) / 256, J.n), dim3(256), 0, s, J);
  else
    hipLaunchKernelGGL(k_i8_crt, dim3((J.n + 255) / 256, J.n), dim3(256), 0, s, J);
  return hipGetLastError();
}

void i8_tile_order(int nt, int2* out) {
  int k = 0;
  for (int si = 0; si < nt; si += 4)
    for (int sj = si; sj < nt; sj += 4)
      for (int ti = si; ti < si + 4 && ti < nt; ++ti)
        for (int tj = sj; tj < sj + 4 && tj < nt; ++tj)
          if (ti <= tj) out[k++] = make_int2(ti, tj);
}

int i8_tile() { return kI8Tile; }
int i8_kblock() { return kI8Kb; }

}  // namespace flsq
