// Device-side building blocks shared by the gfx950 kernels of the FastLSQ hot path.
//
// Trigonometric functions are written here from their mathematics so their
// accuracy is known and testable:
//   * range reduction by multiples of pi (or pi/2) with the two-constant
//     Cody-Waite scheme (W. J. Cody and W. Waite, "Software Manual for the
//     Elementary Functions", 1980): pi is split into its double (float) rounding
//     PI_A and the remainder PI_B, and both products are subtracted with fused
//     multiply-adds;
//   * on the reduced interval, the FP64 sine's polynomial is fitted in the Chebyshev sense
//     (sin_poly_fit.py); the others are Taylor polynomials truncated where the first omitted
//     term is below the format's rounding unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flsq {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMaxDim = 8;

// ---------------------------------------------------------------------------------
// FP64.  sin(x) for |x| < 2^30.  x = k pi + r, |r| <= pi/2, sin x = (-1)^k sin r.
// sin r = r + r^3 g(r^2), g a degree-7 polynomial fitted to (sin sqrt(t) - sqrt(t)) / t^(3/2)
// on [0, (pi/2)^2] in the Chebyshev sense (sin_poly_fit.py beside this file): fit error 3.4e-19,
// evaluation error in double at most 1.9e-16 on [0, pi/2], as for the Taylor series to r^21
// with two multiply-adds fewer.
// ---------------------------------------------------------------------------------
// The coefficients of g, highest degree first.
struct SinPoly {
  double c[8];
};
__device__ __forceinline__ SinPoly sin_poly() {
  return SinPoly{{2.7314447669863995e-15, -7.643970296798572e-13, 1.6058977312464087e-10, -2.5052107616996182e-08,
                  2.7557319219163234e-06, -0.00019841269841254974, 0.008333333333333316, -0.16666666666666666}};
}
// The same values, held in scalar registers: in straight-line code with many sines the compiler
// would otherwise rebuild each 64-bit constant in vector registers at every use (two moves per
// coefficient and sine).
__device__ __forceinline__ SinPoly sin_poly_sgpr() {
  SinPoly q = sin_poly();
#pragma unroll
  for (int i = 0; i < 8; ++i) asm volatile("" : "+s"(q.c[i]));
  return q;
}

__device__ __forceinline__ double sin_f64(double x, const SinPoly& q) {
  const double kInvPi = 0.31830988618379067154;    // 1/pi rounded to double
  const double kPiA = 3.141592653589793116;        // pi rounded to double
  const double kPiB = 1.2246467991473532072e-16;   // pi - kPiA
  const double k = rint(x * kInvPi);
  double r = fma(-k, kPiA, x);
  r = fma(-k, kPiB, r);
  const double r2 = r * r;
  double p = q.c[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) p = fma(p, r2, q.c[i]);
  const double s = fma(r * r2, p, r);
  return (static_cast<int>(k) & 1) ? -s : s;   // |k| < 2^31 for |x| < 2^30: the conversion is exact
}

__device__ __forceinline__ double sin_f64(double x) { return sin_f64(x, sin_poly()); }

// sin and cos together for |x| < 2^30: x = k pi/2 + r, |r| <= pi/4.
// sin to r^17 (omitted (pi/4)^19/19! < 1e-19), cos to r^18 (omitted (pi/4)^20/20! < 1e-21).
__device__ __forceinline__ void sincos_f64(double x, double* s_out, double* c_out) {
  const double k2Pi = 0.63661977236758134308;      // 2/pi
  const double kPiA = 1.5707963267948965580;       // pi/2 rounded to double
  const double kPiB = 6.1232339957367660359e-17;   // pi/2 - kPiA
  const double k = rint(x * k2Pi);
  double r = fma(-k, kPiA, x);
  r = fma(-k, kPiB, r);
  const double r2 = r * r;
  double ps = 1.0 / 355687428096000.0;             // 1/17!
  ps = fma(ps, r2, -1.0 / 1307674368000.0);
  ps = fma(ps, r2, 1.0 / 6227020800.0);
  ps = fma(ps, r2, -1.0 / 39916800.0);
  ps = fma(ps, r2, 1.0 / 362880.0);
  ps = fma(ps, r2, -1.0 / 5040.0);
  ps = fma(ps, r2, 1.0 / 120.0);
  ps = fma(ps, r2, -1.0 / 6.0);
  const double s = fma(r * r2, ps, r);
  double pc = 1.0 / 6402373705728000.0;            // 1/18!
  pc = fma(pc, r2, -1.0 / 20922789888000.0);       // -1/16!
  pc = fma(pc, r2, 1.0 / 87178291200.0);           // 1/14!
  pc = fma(pc, r2, -1.0 / 479001600.0);            // -1/12!
  pc = fma(pc, r2, 1.0 / 3628800.0);               // 1/10!
  pc = fma(pc, r2, -1.0 / 40320.0);                // -1/8!
  pc = fma(pc, r2, 1.0 / 720.0);                   // 1/6!
  pc = fma(pc, r2, -1.0 / 24.0);                   // -1/4!
  pc = fma(pc, r2, 0.5);
  const double c = fma(-r2, pc, 1.0);
  const int q = static_cast<int>(k) & 3;           // |k| < 2^31 for |x| < 2^30
  const double sv = (q & 1) ? c : s;
  const double cv = (q & 1) ? s : c;
  *s_out = (q & 2) ? -sv : sv;
  *c_out = ((q + 1) & 2) ? -cv : cv;
}

// ---------------------------------------------------------------------------------
// FP32.  sin(x) for |x| < 2^16.  x = k pi + r; Taylor of sin to r^13
// (omitted (pi/2)^15/15! < 7e-10).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ float sin_f32(float x) {
  const float kInvPi = 0.318309886f;
  const float kPiA = 3.14159274101257324f;         // pi rounded to float
  const float kPiB = -8.74227800037248566e-8f;     // pi - kPiA
  const float k = rintf(x * kInvPi);
  float r = fmaf(-k, kPiA, x);
  r = fmaf(-k, kPiB, r);
  const float r2 = r * r;
  float p = 1.0f / 6227020800.0f;                  // 1/13!
  p = fmaf(p, r2, -1.0f / 39916800.0f);
  p = fmaf(p, r2, 1.0f / 362880.0f);
  p = fmaf(p, r2, -1.0f / 5040.0f);
  p = fmaf(p, r2, 1.0f / 120.0f);
  p = fmaf(p, r2, -1.0f / 6.0f);
  const float s = fmaf(r * r2, p, r);
  return (static_cast<int>(k) & 1) ? -s : s;
}

// sin and cos together: x = k pi/2 + r, |r| <= pi/4; sin to r^9 (omitted < 2e-9),
// cos to r^10 (omitted < 1.2e-10).
__device__ __forceinline__ void sincos_f32(float x, float* s_out, float* c_out) {
  const float k2Pi = 0.636619772f;
  const float kPiA = 1.57079637050628662f;         // pi/2 rounded to float
  const float kPiB = -4.37113900018624283e-8f;     // pi/2 - kPiA
  const float k = rintf(x * k2Pi);
  float r = fmaf(-k, kPiA, x);
  r = fmaf(-k, kPiB, r);
  const float r2 = r * r;
  float ps = 1.0f / 362880.0f;
  ps = fmaf(ps, r2, -1.0f / 5040.0f);
  ps = fmaf(ps, r2, 1.0f / 120.0f);
  ps = fmaf(ps, r2, -1.0f / 6.0f);
  const float s = fmaf(r * r2, ps, r);
  float pc = 1.0f / 3628800.0f;
  pc = fmaf(pc, r2, -1.0f / 40320.0f);
  pc = fmaf(pc, r2, 1.0f / 720.0f);
  pc = fmaf(pc, r2, -1.0f / 24.0f);
  pc = fmaf(pc, r2, 0.5f);
  const float c = fmaf(-r2, pc, 1.0f);
  const int q = static_cast<int>(k) & 3;
  const float sv = (q & 1) ? c : s;
  const float cv = (q & 1) ? s : c;
  *s_out = (q & 2) ? -sv : sv;
  *c_out = ((q + 1) & 2) ? -cv : cv;
}

// ---------------------------------------------------------------------------------
// Problem geometry as the kernels see it (device pointers, structure-of-arrays).
//
// Entry of the stacked matrix for row i in block g and feature j (Eq. (2)-(3)):
//   A_ij = (amp[g][j] + rho_i) * sin(W_j . x_i + ph[g][j])
// The host folds every operator into this amplitude/phase form:
//   S_j sin z + C_j cos z = R_j sin(z + psi_j),  R = hypot(S, C), psi = atan2(C, S),
// and for operators with only even-order terms (C = 0) keeps amp = S (signed), ph = b,
// which is the form that admits the per-row Newton coefficient rho_i.
// ---------------------------------------------------------------------------------
struct Geo {
  int d;
  int n;                 // features
  int64_t P;             // rows of the stacked system
  int n_blocks;
  const double* Wt;      // d x n
  const float* Wt32;
  const double* amp;     // n_blocks x n
  const double* ph;
  const float* amp32;
  const float* ph32;
  const double* Xt;      // d x P
  const double* Xrm;     // P x d (row-major copy)
  const float* Xt32;
  const int32_t* row_block;   // P
  const double* frec;         // n_blocks x n records {W_j (d), amp_gj, ph_gj, 0...}, frec_stride(d) doubles each
};

// Doubles per feature record: 8 up to d = 6 (one 64-byte scalar load), else 16.
__host__ __device__ constexpr int frec_stride(int d) { return d + 2 <= 8 ? 8 : 16; }

// A run of rows that lies inside one block: rows [row0, row0 + nrows).
struct Chunk {
  int32_t row0;
  int32_t nrows;
  int32_t block;
  int32_t pad;
};

}  // namespace flsq
