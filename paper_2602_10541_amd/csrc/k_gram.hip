// Fused assembly + Gram product on gfx950 MFMA.
//
// G = A^T A over the stacked rows of Eq. (3), where every entry of A comes from the
// closed form of Eq. (2) (folded into amp * sin(W.x + ph), see flsq_device.h).  A is
// never written to memory: each workgroup builds a KC-row slab of A for its two
// 128-feature column sets in LDS and feeds it straight to the matrix cores.
//
// Work decomposition ("stream-K"): the upper-triangle tiles of G times the row chunks
// form a linear space of units; each persistent workgroup takes an equal contiguous
// range.  A range covers at most a few tiles; the partial tile of each covered segment
// is written to a workspace slot, and a deterministic reduction sums the slots of each
// tile in workgroup order.  All workgroups carry the same amount of MFMA work, so there
// is no tail wave, and results are bit-reproducible run to run.
#include "flsq_device.h"
#include "flsq_launch.h"

namespace flsq {

constexpr int kTile = 128;       // features per tile side
constexpr int kChunk = 32;       // rows per LDS slab
constexpr int kThreads = 256;    // 4 waves, 2 x 2 over the tile

struct GramJob {
  Geo g;
  const double* rho;         // per-row additive amplitude (nullable)
  const float* rho32;
  const Chunk* chunks;
  int n_chunks;
  int nt;                    // tiles per side
  int64_t total_units;       // n_tiles * n_chunks
  int64_t units_per_wg;
  int max_seg;
  void* partial;             // [n_wg * max_seg][kTile * kTile], double or float
};

__device__ __forceinline__ void tile_coords(int t, int nt, int* ti, int* tj) {
  int r = 0;
  int rowlen = nt;
  while (t >= rowlen) {
    t -= rowlen;
    ++r;
    --rowlen;
  }
  *ti = r;
  *tj = r + t;
}

// ------------------------------------------------------------------ FP64
template <int D>
__global__ __launch_bounds__(kThreads, 2) void k_gram_f64(GramJob J) {
  __shared__ double sA[2][kChunk][kTile];
  __shared__ double sX[D][kChunk];
  __shared__ double sRho[kChunk];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int n = J.g.n;
  const int64_t P = J.g.P;

  int64_t u = (int64_t)blockIdx.x * J.units_per_wg;
  const int64_t u_end = min(u + J.units_per_wg, J.total_units);
  int seg = 0;
  while (u < u_end) {
    const int tile = (int)(u / J.n_chunks);
    const int c0 = (int)(u % J.n_chunks);
    const int c1 = (int)min((int64_t)J.n_chunks, (int64_t)c0 + (u_end - u));
    int ti, tj;
    tile_coords(tile, J.nt, &ti, &tj);
    const bool diag = (ti == tj);

    // Each thread owns one feature of the J set (rows of G) or of the L set (columns).
    const int fl = tid % kTile;
    const int set = tid / kTile;                       // 0: J features, 1: L features
    const int f = (diag || set == 0) ? ti * kTile + fl : tj * kTile + fl;
    const bool fvalid = f < n;
    double w[D];
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = fvalid ? J.g.Wt[(int64_t)k * n + f] : 0.0;

    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

    for (int c = c0; c < c1; ++c) {
      const Chunk ch = J.chunks[c];
      __syncthreads();   // previous slab fully consumed
      for (int e = tid; e < D * kChunk; e += kThreads) {
        const int k = e / kChunk, r = e % kChunk;
        sX[k][r] = (r < ch.nrows) ? J.g.Xt[(int64_t)k * P + ch.row0 + r] : 0.0;
      }
      if (tid < kChunk) sRho[tid] = (J.rho && tid < ch.nrows) ? J.rho[ch.row0 + tid] : 0.0;
      __syncthreads();
      const double amp = fvalid ? J.g.amp[(int64_t)ch.block * n + f] : 0.0;
      const double ph = fvalid ? J.g.ph[(int64_t)ch.block * n + f] : 0.0;
      // assemble the slab: off-diagonal tiles build both sets (32 rows each thread),
      // diagonal tiles build one set with the rows split over the two thread halves.
      const int r_begin = diag ? set * (kChunk / 2) : 0;
      const int r_count = diag ? kChunk / 2 : kChunk;
      const int dst = diag ? 0 : set;
#pragma unroll 2
      for (int rr = 0; rr < r_count; ++rr) {
        const int r = r_begin + rr;
        double z = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) z = fma(w[k], sX[k][r], z);
        const double v = (r < ch.nrows) ? (amp + sRho[r]) * sin_f64(z + ph) : 0.0;
        sA[dst][r][fl] = v;
      }
      __syncthreads();
      const int lset = diag ? 0 : 1;
#pragma unroll 1
      for (int kk = 0; kk < kChunk / 4; ++kk) {
        const int row = kk * 4 + (lane >> 4);
        double av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = sA[0][row][wm * 64 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = sA[lset][row][wn * 64 + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    // write the partial tile: slot v of a 16x16 block is row 4 v + lane / 16, column lane % 16
    double* out = (double*)J.partial + ((int64_t)blockIdx.x * J.max_seg + seg) * (kTile * kTile);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = wm * 64 + a * 16 + 4 * v + (lane >> 4);
          const int col = wn * 64 + b * 16 + (lane & 15);
          out[row * kTile + col] = acc[a][b][v];
        }
    ++seg;
    u += (c1 - c0);
  }
}

// ------------------------------------------------------------------ FP32
// Same decomposition with FP32 entries and v_mfma_f32_32x32x2_f32; each wave owns a
// 64 x 64 quarter of the tile as 2 x 2 blocks of 32 x 32.
template <int D>
__global__ __launch_bounds__(kThreads, 2) void k_gram_f32(GramJob J) {
  __shared__ float sA[2][kChunk][kTile];
  __shared__ float sX[D][kChunk];
  __shared__ float sRho[kChunk];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int n = J.g.n;
  const int64_t P = J.g.P;

  int64_t u = (int64_t)blockIdx.x * J.units_per_wg;
  const int64_t u_end = min(u + J.units_per_wg, J.total_units);
  int seg = 0;
  while (u < u_end) {
    const int tile = (int)(u / J.n_chunks);
    const int c0 = (int)(u % J.n_chunks);
    const int c1 = (int)min((int64_t)J.n_chunks, (int64_t)c0 + (u_end - u));
    int ti, tj;
    tile_coords(tile, J.nt, &ti, &tj);
    const bool diag = (ti == tj);
    const int fl = tid % kTile;
    const int set = tid / kTile;
    const int f = (diag || set == 0) ? ti * kTile + fl : tj * kTile + fl;
    const bool fvalid = f < n;
    float w[D];
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = fvalid ? J.g.Wt32[(int64_t)k * n + f] : 0.f;

    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    for (int c = c0; c < c1; ++c) {
      const Chunk ch = J.chunks[c];
      __syncthreads();
      for (int e = tid; e < D * kChunk; e += kThreads) {
        const int k = e / kChunk, r = e % kChunk;
        sX[k][r] = (r < ch.nrows) ? J.g.Xt32[(int64_t)k * P + ch.row0 + r] : 0.f;
      }
      if (tid < kChunk) sRho[tid] = (J.rho32 && tid < ch.nrows) ? J.rho32[ch.row0 + tid] : 0.f;
      __syncthreads();
      const float amp = fvalid ? J.g.amp32[(int64_t)ch.block * n + f] : 0.f;
      const float ph = fvalid ? J.g.ph32[(int64_t)ch.block * n + f] : 0.f;
      const int r_begin = diag ? set * (kChunk / 2) : 0;
      const int r_count = diag ? kChunk / 2 : kChunk;
      const int dst = diag ? 0 : set;
#pragma unroll 4
      for (int rr = 0; rr < r_count; ++rr) {
        const int r = r_begin + rr;
        float z = 0.f;
#pragma unroll
        for (int k = 0; k < D; ++k) z = fmaf(w[k], sX[k][r], z);
        const float v = (r < ch.nrows) ? (amp + sRho[r]) * sin_f32(z + ph) : 0.f;
        sA[dst][r][fl] = v;
      }
      __syncthreads();
      const int lset = diag ? 0 : 1;
#pragma unroll
      for (int kk = 0; kk < kChunk / 2; ++kk) {
        const int row = kk * 2 + (lane >> 5);
        float av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = sA[0][row][wm * 64 + a * 32 + (lane & 31)];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = sA[lset][row][wn * 64 + b * 32 + (lane & 31)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    // slot v of a 32x32 block is row 8 (v / 4) + 4 (lane / 32) + v % 4, column lane % 32
    float* out = (float*)J.partial + ((int64_t)blockIdx.x * J.max_seg + seg) * (kTile * kTile);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm * 64 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          const int col = wn * 64 + b * 32 + (lane & 31);
          out[row * kTile + col] = acc[a][b][v];
        }
    ++seg;
    u += (c1 - c0);
  }
}

// ------------------------------------------------------------------ BF16x3
// Same decomposition as the FP32 kernel; each FP32 entry a is split into bf16 parts
// hi = bf16(a), lo = bf16(a - hi) (round to nearest even; a - hi is exact in FP32), and
// the Gram is accumulated in FP32 from three v_mfma_f32_32x32x16_bf16 products per block,
// hi.hi + hi.lo + lo.hi (the dropped lo.lo term and the bf16 rounding of lo leave about
// 2^-16 relative per product).  Slabs are stored feature-major, 8 consecutive rows of one
// feature per 16-byte operand; a 16-byte pad per feature row keeps the operand reads of
// 16 consecutive features on distinct LDS banks.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBfPitch = kChunk + 8;   // bf16 elements per feature row (80 bytes)

__device__ __forceinline__ unsigned bf16_bits_rne(float v) {
  const unsigned u = __float_as_uint(v);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

template <int D>
__global__ __launch_bounds__(kThreads, 2) void k_gram_bf16x3(GramJob J) {
  __shared__ __align__(16) unsigned short sH[2][kTile][kBfPitch];
  __shared__ __align__(16) unsigned short sL[2][kTile][kBfPitch];
  __shared__ float sX[D][kChunk];
  __shared__ float sRho[kChunk];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int n = J.g.n;
  const int64_t P = J.g.P;

  int64_t u = (int64_t)blockIdx.x * J.units_per_wg;
  const int64_t u_end = min(u + J.units_per_wg, J.total_units);
  int seg = 0;
  while (u < u_end) {
    const int tile = (int)(u / J.n_chunks);
    const int c0 = (int)(u % J.n_chunks);
    const int c1 = (int)min((int64_t)J.n_chunks, (int64_t)c0 + (u_end - u));
    int ti, tj;
    tile_coords(tile, J.nt, &ti, &tj);
    const bool diag = (ti == tj);
    const int fl = tid % kTile;
    const int set = tid / kTile;
    const int f = (diag || set == 0) ? ti * kTile + fl : tj * kTile + fl;
    const bool fvalid = f < n;
    float w[D];
#pragma unroll
    for (int k = 0; k < D; ++k) w[k] = fvalid ? J.g.Wt32[(int64_t)k * n + f] : 0.f;

    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

    for (int c = c0; c < c1; ++c) {
      const Chunk ch = J.chunks[c];
      __syncthreads();
      for (int e = tid; e < D * kChunk; e += kThreads) {
        const int k = e / kChunk, r = e % kChunk;
        sX[k][r] = (r < ch.nrows) ? J.g.Xt32[(int64_t)k * P + ch.row0 + r] : 0.f;
      }
      if (tid < kChunk) sRho[tid] = (J.rho32 && tid < ch.nrows) ? J.rho32[ch.row0 + tid] : 0.f;
      __syncthreads();
      const float amp = fvalid ? J.g.amp32[(int64_t)ch.block * n + f] : 0.f;
      const float ph = fvalid ? J.g.ph32[(int64_t)ch.block * n + f] : 0.f;
      const int r_begin = diag ? set * (kChunk / 2) : 0;
      const int r_count = diag ? kChunk / 2 : kChunk;
      const int dst = diag ? 0 : set;
      for (int r8 = 0; r8 < r_count; r8 += 8) {
        unsigned hw[4], lw[4];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int r = r_begin + r8 + q;
          float z = 0.f;
#pragma unroll
          for (int k = 0; k < D; ++k) z = fmaf(w[k], sX[k][r], z);
          const float v = (r < ch.nrows) ? (amp + sRho[r]) * sin_f32(z + ph) : 0.f;
          const unsigned hb = bf16_bits_rne(v);
          const unsigned lb = bf16_bits_rne(v - __uint_as_float(hb << 16));
          if (q & 1) {
            hw[q >> 1] |= hb << 16;
            lw[q >> 1] |= lb << 16;
          } else {
            hw[q >> 1] = hb;
            lw[q >> 1] = lb;
          }
        }
        *(u32x4*)&sH[dst][fl][r_begin + r8] = u32x4{hw[0], hw[1], hw[2], hw[3]};
        *(u32x4*)&sL[dst][fl][r_begin + r8] = u32x4{lw[0], lw[1], lw[2], lw[3]};
      }
      __syncthreads();
      const int lset = diag ? 0 : 1;
#pragma unroll
      for (int ks = 0; ks < kChunk / 16; ++ks) {
        const int k0 = ks * 16 + 8 * (lane >> 5);
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int fa = wm * 64 + a * 32 + (lane & 31);
          ah[a] = *(const bf16x8*)&sH[0][fa][k0];
          al[a] = *(const bf16x8*)&sL[0][fa][k0];
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int fb = wn * 64 + b * 32 + (lane & 31);
          bh[b] = *(const bf16x8*)&sH[lset][fb][k0];
          bl[b] = *(const bf16x8*)&sL[lset][fb][k0];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          }
      }
    }
    // slot v of a 32x32 block is row 8 (v / 4) + 4 (lane / 32) + v % 4, column lane % 32
    float* out = (float*)J.partial + ((int64_t)blockIdx.x * J.max_seg + seg) * (kTile * kTile);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = wm * 64 + a * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          const int col = wn * 64 + b * 32 + (lane & 31);
          out[row * kTile + col] = acc[a][b][v];
        }
    ++seg;
    u += (c1 - c0);
  }
}

// ------------------------------------------------------------------ reduction
// For tile t, sum its partial slots (listed in slot_ptr / slots, in workgroup order)
// in FP64 and store the upper triangle of G (row-major n x n, lda = n).  With `mirror`,
// the lower triangle receives the transpose of the upper one (exactly symmetric G).
template <typename T>
__global__ __launch_bounds__(256) void k_gram_reduce(const T* partial, const int32_t* slot_ptr,
                                                     const int32_t* slots, int nt, int n, double* G,
                                                     int mirror, double diag_add) {
  __shared__ double tr[32][33];
  const int t = blockIdx.x;
  int ti, tj;
  tile_coords(t, nt, &ti, &tj);
  const int s0 = slot_ptr[t], s1 = slot_ptr[t + 1];
  const int tid = threadIdx.x;
  // 32 x 32 sub-blocks so the mirrored store can be transposed through LDS
  for (int sb = 0; sb < (kTile / 32) * (kTile / 32); ++sb) {
    const int br = (sb / (kTile / 32)) * 32, bc = (sb % (kTile / 32)) * 32;
    for (int e = tid; e < 32 * 32; e += 256) {
      const int r = e / 32, c = e % 32;
      double s = 0.0;
      for (int q = s0; q < s1; ++q) s += (double)partial[(int64_t)slots[q] * (kTile * kTile) + (br + r) * kTile + bc + c];
      const int gi = ti * kTile + br + r, gj = tj * kTile + bc + c;
      if (gi == gj) s += diag_add;
      // in a diagonal tile only the upper triangle is taken (the kernels may round the two
      // triangles differently); the lower one is its mirror
      if (gi < n && gj < n && gj >= gi) G[(int64_t)gi * n + gj] = s;
      tr[r][c] = s;
    }
    __syncthreads();
    if (mirror) {
      for (int e = tid; e < 32 * 32; e += 256) {
        const int r = e / 32, c = e % 32;   // store G[tj*T + bc + r][ti*T + br + c] = tile[br + c][bc + r]
        const int gi = tj * kTile + bc + r, gj = ti * kTile + br + c;
        if (gi < n && gj < n && gi > gj) G[(int64_t)gi * n + gj] = tr[c][r];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ launchers
int gram_tile() { return kTile; }
int gram_chunk_rows() { return kChunk; }

int gram_occupancy(int prec) {
  int occ = 0;
  hipError_t e;
  if (prec == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_gram_f64<6>, kThreads, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_gram_f32<6>, kThreads, 0);
  return (e == hipSuccess && occ > 0) ? occ : 1;
}

#define FLSQ_GRAM_CASE(DIM, KER)                                                        \
  case DIM:                                                                             \
    hipLaunchKernelGGL((KER<DIM>), dim3(n_wg), dim3(kThreads), 0, stream, job);        \
    break;

hipError_t launch_gram(const GramLaunch& L, hipStream_t stream) {
  GramJob job;
  job.g = L.g;
  job.rho = L.rho;
  job.rho32 = L.rho32;
  job.chunks = L.chunks;
  job.n_chunks = L.n_chunks;
  job.nt = L.nt;
  job.total_units = L.total_units;
  job.units_per_wg = L.units_per_wg;
  job.max_seg = L.max_seg;
  job.partial = L.partial;
  const int n_wg = L.n_wg;
  if (L.prec == 0) {
    switch (L.g.d) {
      FLSQ_GRAM_CASE(1, k_gram_f64) FLSQ_GRAM_CASE(2, k_gram_f64) FLSQ_GRAM_CASE(3, k_gram_f64)
      FLSQ_GRAM_CASE(4, k_gram_f64) FLSQ_GRAM_CASE(5, k_gram_f64) FLSQ_GRAM_CASE(6, k_gram_f64)
      FLSQ_GRAM_CASE(7, k_gram_f64) FLSQ_GRAM_CASE(8, k_gram_f64)
      default: return hipErrorInvalidValue;
    }
  } else if (L.prec == 1) {
    switch (L.g.d) {
      FLSQ_GRAM_CASE(1, k_gram_f32) FLSQ_GRAM_CASE(2, k_gram_f32) FLSQ_GRAM_CASE(3, k_gram_f32)
      FLSQ_GRAM_CASE(4, k_gram_f32) FLSQ_GRAM_CASE(5, k_gram_f32) FLSQ_GRAM_CASE(6, k_gram_f32)
      FLSQ_GRAM_CASE(7, k_gram_f32) FLSQ_GRAM_CASE(8, k_gram_f32)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (L.g.d) {
      FLSQ_GRAM_CASE(1, k_gram_bf16x3) FLSQ_GRAM_CASE(2, k_gram_bf16x3) FLSQ_GRAM_CASE(3, k_gram_bf16x3)
      FLSQ_GRAM_CASE(4, k_gram_bf16x3) FLSQ_GRAM_CASE(5, k_gram_bf16x3) FLSQ_GRAM_CASE(6, k_gram_bf16x3)
      FLSQ_GRAM_CASE(7, k_gram_bf16x3) FLSQ_GRAM_CASE(8, k_gram_bf16x3)
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

// prec: 0 FP64 partials, otherwise FP32 partials
hipError_t launch_gram_reduce(int prec, const void* partial, const int32_t* slot_ptr, const int32_t* slots,
                              int nt, int n, double* G, int mirror, double diag_add, hipStream_t stream) {
  const int n_tiles = nt * (nt + 1) / 2;
  if (prec == 0)
    hipLaunchKernelGGL(k_gram_reduce<double>, dim3(n_tiles), dim3(256), 0, stream, (const double*)partial,
                       slot_ptr, slots, nt, n, G, mirror, diag_add);
  else
    hipLaunchKernelGGL(k_gram_reduce<float>, dim3(n_tiles), dim3(256), 0, stream, (const float*)partial,
                       slot_ptr, slots, nt, n, G, mirror, diag_add);
  return hipGetLastError();
}

}  // namespace flsq
