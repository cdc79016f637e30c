// Hyperbolic tangent of the hidden layer, shared by the feature, evaluation
// and adjoint-evaluation kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace ddelm {

// tanh|z| = e / (e + 2) with e = expm1(2|z|), and expm1 by argument
// reduction (Tang's method, without a table): x = 2|z| = k ln2 + r with
// |r| <= ln2 / 2, expm1(x) = 2^k (e^r - 1) + (2^k - 1), where
// e^r - 1 = r + r^2 (1/2! + r/3! + ... + r^11/13!) is the Taylor series cut
// after r^13 (the remainder is below 1e-17 relative).  There is no
// cancellation for small |z| (k = 0 gives e^r - 1 directly).  ln2 is split
// into a 32-bit head (k ln2_hi is exact for the |k| <= 58 met here) and a
// tail.  1/(e + 2) comes from the hardware reciprocal refined by two
// Newton-Raphson steps y <- y + y (1 - d y).  For |z| > 20 tanh differs from
// +-1 by less than 1e-17.  The error is a few ulps, like a library tanh, at
// about a third of the instructions of expm1 and an IEEE division.
__device__ __forceinline__ double tanh_fast(double z) {
  constexpr double kInvLn2 = 1.4426950408889634;
  constexpr double kLn2Hi = 0.6931471803691238;       // ln2 rounded to 32 significant bits
  constexpr double kLn2Lo = 1.9082149292705877e-10;   // ln2 - kLn2Hi
  const double a = fabs(z);
  const double x = 2.0 * a;
  const double k = rint(x * kInvLn2);
  const double r = fma(-k, kLn2Lo, fma(-k, kLn2Hi, x));
  double p = 1.6059043836821613e-10;                  // 1/13!
  p = fma(p, r, 2.08767569878681e-09);                // 1/12!
  p = fma(p, r, 2.505210838544172e-08);               // 1/11!
  p = fma(p, r, 2.755731922398589e-07);               // 1/10!
  p = fma(p, r, 2.7557319223985893e-06);              // 1/9!
  p = fma(p, r, 2.48015873015873e-05);                // 1/8!
  p = fma(p, r, 0.0001984126984126984);               // 1/7!
  p = fma(p, r, 0.001388888888888889);                // 1/6!
  p = fma(p, r, 0.008333333333333333);                // 1/5!
  p = fma(p, r, 0.041666666666666664);                // 1/4!
  p = fma(p, r, 0.16666666666666666);                 // 1/3!
  p = fma(p, r, 0.5);                                 // 1/2!
  const double q = fma(r * r, p, r);                  // e^r - 1
  const double s = ldexp(1.0, (int)k);
  const double e = fma(s, q, s - 1.0);                // expm1(x)
  const double d = e + 2.0;
  double y = __builtin_amdgcn_rcp(d);
  y = fma(fma(-d, y, 1.0), y, y);
  y = fma(fma(-d, y, 1.0), y, y);
  return a > 20.0 ? copysign(1.0, z) : copysign(e * y, z);
}

}  // namespace ddelm
