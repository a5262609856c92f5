// rlx_gauss.hpp -- standard normals from a field pair of a RANLUX++ step
// (Box-Muller), shared by librlx.so's bulk kernels and the device-side
// engine of rlx_engine.h, and compiled for the host by the tests.
//
// The paper leaves distributions to the framework around the engine
// (section 2.4); the transform used here takes the step's aligned field pair
// (v1, v2) (48 bits each, section 2.3) as u1 = v1 2^-48 and u2 = v2 2^-48 and
// returns
//     r cos(2 pi u2) and r sin(2 pi u2),   r = sqrt(-2 ln(1 - u1)).
//
// Everything is written in binary64 basic operations, fused multiply-adds,
// rint, division and sqrt, all correctly rounded on the device and on the
// host, with contraction switched off, so a host build gives the device's
// bits.  Accuracy (checked against a 40-digit evaluation on the host):
//
//  * ln w for w = 1 - u1 in [2^-48, 1] (exact): w = 2^e m with m in
//    [sqrt(1/2), sqrt(2)) by integer arithmetic on the high word (adding the
//    distance from sqrt(1/2)'s high word to 1.0's carries mantissas at or
//    above it into the next exponent); with f = m - 1 (exact) and
//    s = f / (2 + f), ln m = 2 atanh s = 2s + 2s z P(z), z = s^2,
//    P(z) = sum_k z^k / (2k + 3), |s| < 0.1716.  Since 2s = f - s f this is
//    f - s (f - 2 z P(z)): the leading term f is exact and the correction is
//    at most a fifth of it.  e ln 2 is added as e LN2_HI (exact: LN2_HI has
//    46 significant bits, |e| <= 48) plus e LN2_LO.  Ten terms of P leave a
//    truncation below 10^-18 relative.
//
//  * 2 pi u2 = (pi / 2) t with t = 4 u2 = v2 2^-46 in [0, 4) (exact); with
//    j = rint(t) and y = t - j in [-1/2, 1/2] (exact), the angle is
//    j pi/2 + phi, phi = (pi / 2) y in [-pi/4, pi/4], formed as p + d with
//    pi/2 split in two doubles (d is the product's rounding error plus the
//    low part).  sin p and cos p are their Taylor series (through p^17 and
//    p^16; the first omitted terms are below 10^-19 and 3 10^-18), then
//    corrected by d (sin(p + d) = sin p + d cos p, cos(p + d) = cos p -
//    d sin p to first order), then rotated by j quarter turns.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlx {
namespace gauss {

#define RLX_GAUSS_HD __host__ __device__ __forceinline__

RLX_GAUSS_HD double from_bits(uint32_t lo, uint32_t hi) {
  const uint64_t b = ((uint64_t)hi << 32) | lo;
  double v;
  __builtin_memcpy(&v, &b, 8);
  return v;
}

RLX_GAUSS_HD uint64_t to_bits(double v) {
  uint64_t b;
  __builtin_memcpy(&b, &v, 8);
  return b;
}

// ln 2 = LN2_HI + LN2_LO, LN2_HI = floor(ln 2 2^46) 2^-46.
constexpr double LN2_HI = 0x1.62e42fefa3980p-1;
constexpr double LN2_LO = 0x1.bcd5e4f1d9cc0p-47;
// pi / 2 = PIO2_HI + PIO2_LO, each rounded to nearest.
constexpr double PIO2_HI = 0x1.921fb54442d18p+0;
constexpr double PIO2_LO = 0x1.1a62633145c07p-54;
// High word of sqrt(1/2) (0x3FE6A09E667F3BCD).
constexpr uint32_t SQRT_HALF_HI = 0x3FE6A09Eu;

// ln w for w in [2^-48, 1], w a multiple of 2^-48.
RLX_GAUSS_HD double log_unit(double w) {
#pragma clang fp contract(off)
  const uint64_t b = to_bits(w);
  uint32_t hi = (uint32_t)(b >> 32) + (0x3FF00000u - SQRT_HALF_HI);
  const int e = (int)(hi >> 20) - 0x3FF;
  hi = (hi & 0x000FFFFFu) + SQRT_HALF_HI;
  const double f = from_bits((uint32_t)b, hi) - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double P = 1.0 / 21;
  P = __builtin_fma(P, z, 1.0 / 19);
  P = __builtin_fma(P, z, 1.0 / 17);
  P = __builtin_fma(P, z, 1.0 / 15);
  P = __builtin_fma(P, z, 1.0 / 13);
  P = __builtin_fma(P, z, 1.0 / 11);
  P = __builtin_fma(P, z, 1.0 / 9);
  P = __builtin_fma(P, z, 1.0 / 7);
  P = __builtin_fma(P, z, 1.0 / 5);
  P = __builtin_fma(P, z, 1.0 / 3);
  const double c = s * __builtin_fma(-2.0 * z, P, f);  // s (f - 2 z P), 2z exact
  const double de = (double)e;
  return __builtin_fma(de, LN2_HI, f - __builtin_fma(-de, LN2_LO, c));
}

// cos(2 pi u2) and sin(2 pi u2) for t = 4 u2 in [0, 4), t a multiple of
// 2^-46.
RLX_GAUSS_HD void cos_sin_quarter_turns(double t, double& co, double& si) {
#pragma clang fp contract(off)
  const double j = __builtin_rint(t);
  const double y = t - j;
  const double p = y * PIO2_HI;
  const double d = __builtin_fma(y, PIO2_LO, __builtin_fma(y, PIO2_HI, -p));
  const double z = p * p;
  double S = 1.0 / 355687428096000.0;   // sin: 1/17!, -1/15!, ..., -1/3!
  S = __builtin_fma(S, z, -1.0 / 1307674368000.0);
  S = __builtin_fma(S, z, 1.0 / 6227020800.0);
  S = __builtin_fma(S, z, -1.0 / 39916800.0);
  S = __builtin_fma(S, z, 1.0 / 362880.0);
  S = __builtin_fma(S, z, -1.0 / 5040.0);
  S = __builtin_fma(S, z, 1.0 / 120.0);
  S = __builtin_fma(S, z, -1.0 / 6.0);
  double C = 1.0 / 20922789888000.0;    // cos: 1/16!, -1/14!, ..., -1/2!
  C = __builtin_fma(C, z, -1.0 / 87178291200.0);
  C = __builtin_fma(C, z, 1.0 / 479001600.0);
  C = __builtin_fma(C, z, -1.0 / 3628800.0);
  C = __builtin_fma(C, z, 1.0 / 40320.0);
  C = __builtin_fma(C, z, -1.0 / 720.0);
  C = __builtin_fma(C, z, 1.0 / 24.0);
  C = __builtin_fma(C, z, -0.5);
  const double sp = __builtin_fma(p * z, S, p);
  const double cp = __builtin_fma(z, C, 1.0);
  const double sn = __builtin_fma(d, cp, sp);
  const double cs = __builtin_fma(-d, sp, cp);
  // rotate by q = j mod 4 quarter turns: (c, s) -> (-s, c) per turn
  const uint32_t q = (uint32_t)(int)j;
  const bool swap = (q & 1u) != 0;
  const double a = swap ? sn : cs;
  const double bb = swap ? cs : sn;
  const uint64_t neg_c = (uint64_t)(((q + 1u) >> 1) & 1u) << 63;  // q = 1, 2
  const uint64_t neg_s = (uint64_t)((q >> 1) & 1u) << 63;         // q = 2, 3
  const uint64_t ab = to_bits(a) ^ neg_c, bbb = to_bits(bb) ^ neg_s;
  __builtin_memcpy(&co, &ab, 8);
  __builtin_memcpy(&si, &bbb, 8);
}

// The two normals of the field pair held in words (w0, w1, w2) (bits 0..47
// are v1, bits 48..95 v2): co = r cos(2 pi u2), si = r sin(2 pi u2).
RLX_GAUSS_HD void box_muller(uint32_t w0, uint32_t w1, uint32_t w2, double& co, double& si) {
#pragma clang fp contract(off)
  // 0x403 << 52 | v1 is 16 + v1 2^-48 and 0x405 << 52 | v2 is 64 + v2 2^-46:
  // the subtractions are exact
  const double u1 = from_bits(w0, (w1 & 0xFFFFu) | 0x40300000u) - 16.0;
  const double t = from_bits((w1 >> 16) | (w2 << 16), (w2 >> 16) | 0x40500000u) - 64.0;
  const double r = __builtin_sqrt(-2.0 * log_unit(1.0 - u1));
  double c, s;
  cos_sin_quarter_turns(t, c, s);
  co = r * c;
  si = r * s;
}

#undef RLX_GAUSS_HD

}  // namespace gauss
}  // namespace rlx
