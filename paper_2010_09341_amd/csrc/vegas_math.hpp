// vegas_math.hpp — binary64 elementary functions written for the kernels
// (shorter than the general library ones: no special-case handling the
// kernels do not need).
#pragma once

#include <hip/hip_runtime.h>

namespace vegas {

// e^x in binary64 (the binary64 Gaussian evaluates one per event, the
// refinement one per bin). Cody and Waite's reduction: x = n ln2 + r with
// n = rint(x / ln2), the product n ln2 taken in two parts (a head with
// trailing zero bits, so that n times it is exact, and a tail),
// |r| <= ln2/2 + tiny; e^r from its Taylor series to
// degree 13 (truncation below 5e-18 relative), evaluated by Horner's rule;
// then the scaling by 2^n, which also gives 0 below about -745 and infinity
// above about 709.8. x below -1100 (-inf included) is taken as -1100, which
// gives 0; x must not be NaN (it would give 0 too) and x up to 1e9 keeps n in
// range. Within 3 ulp of e^x (the tests check it against the C library).
__host__ __device__ inline double exp_f64(double x) {
  x = fmax(x, -1100.0);
  const double ln2_hi = 6.93147180369123816490e-01;  // 0x3FE62E42FEE00000
  const double ln2_lo = 1.90821492927058770002e-10;  // ln2 - ln2_hi
  const double n = rint(x * 1.44269504088896338700e+00);  // x / ln2
  double r = fma(-n, ln2_hi, x);
  r = fma(-n, ln2_lo, r);
  // 1/k! for k = 13 .. 2
  double p = 1.0 / 6227020800.0;
  p = fma(p, r, 1.0 / 479001600.0);
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)n);
}

// ln x in binary64 for finite x > 0 (subnormals included). x = m 2^k with
// m in [1/sqrt2, sqrt2); ln m = 2 atanh(s) with s = (m - 1)/(m + 1),
// |s| <= 0.1716, from the odd series 2 s (1 + s^2/3 + s^4/5 + ... + s^20/21)
// (truncation below 2e-18 relative), evaluated by Horner's rule in s^2; then
// k ln2 added in two parts as in exp_f64. Within 2 ulp of ln x (the tests
// check it against the C library).
__host__ __device__ inline double log_f64(double x) {
  const double ln2_hi = 6.93147180369123816490e-01;  // as in exp_f64
  const double ln2_lo = 1.90821492927058770002e-10;
  int k;
  double m = frexp(x, &k);  // x = m 2^k, m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    k -= 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  // 1/(2j+1) for j = 10 .. 1, then 1
  double q = 1.0 / 21.0;
  q = fma(q, z, 1.0 / 19.0);
  q = fma(q, z, 1.0 / 17.0);
  q = fma(q, z, 1.0 / 15.0);
  q = fma(q, z, 1.0 / 13.0);
  q = fma(q, z, 1.0 / 11.0);
  q = fma(q, z, 1.0 / 9.0);
  q = fma(q, z, 1.0 / 7.0);
  q = fma(q, z, 1.0 / 5.0);
  q = fma(q, z, 1.0 / 3.0);
  // ln m = 2s + 2s z q
  const double two_s = 2.0 * s;
  const double lnm = fma(two_s * z, q, two_s);
  const double kd = (double)k;
  return fma(kd, ln2_hi, fma(kd, ln2_lo, lnm));
}

// x^a for finite x > 0 as e^(a ln x) (the refinement's compression): a few
// ulp of ln x, times |a ln x|, relative.
__host__ __device__ inline double pow_pos(double x, double a) { return exp_f64(a * log_f64(x)); }

// sin(2 pi u) and cos(2 pi u) for 0 <= u <= 1 (RAMBO's azimuth, u in turns).
// The reduction is exact in turns: n = rint(4u) quarter turns, r = u - n/4 in
// [-1/8, 1/8] (u and n/4 are both multiples of u's ulp, so the subtraction
// loses nothing), theta = 2 pi r with |theta| <= pi/4; then the Taylor series
// of sin to theta^17 and of cos to theta^16 (truncation below 1e-19),
// evaluated by Horner's rule in theta^2, and the quadrant's signs and swap.
// Within a few ulp of the exact values (the tests check it against 40-digit
// arithmetic); near u = 1/2 and 1 it is more accurate than sin(2 pi u) of a
// rounded argument 2 pi u.
__host__ __device__ inline void sincos_turns_f64(double u, double* s, double* c) {
  const double n = rint(4.0 * u);
  const double r = fma(-0.25, n, u);
  const double th = r * 6.28318530717958647693;
  const double z = th * th;
  // sin: theta (1 - z/3! + z^2/5! - ... + z^8/17!)
  double ps = 1.0 / 355687428096000.0;  // 1/17!
  ps = fma(ps, -z, 1.0 / 1307674368000.0);
  ps = fma(ps, -z, 1.0 / 6227020800.0);
  ps = fma(ps, -z, 1.0 / 39916800.0);
  ps = fma(ps, -z, 1.0 / 362880.0);
  ps = fma(ps, -z, 1.0 / 5040.0);
  ps = fma(ps, -z, 1.0 / 120.0);
  ps = fma(ps, -z, 1.0 / 6.0);
  const double sn = fma(th * -z, ps, th);  // th - th z (1/3! - ...)
  // cos: 1 - z/2! + z^2/4! - ... + z^8/16!
  double pc = 1.0 / 20922789888000.0;  // 1/16!
  pc = fma(pc, -z, 1.0 / 87178291200.0);
  pc = fma(pc, -z, 1.0 / 479001600.0);
  pc = fma(pc, -z, 1.0 / 3628800.0);
  pc = fma(pc, -z, 1.0 / 40320.0);
  pc = fma(pc, -z, 1.0 / 720.0);
  pc = fma(pc, -z, 1.0 / 24.0);
  pc = fma(pc, -z, 0.5);
  const double cs = fma(-z, pc, 1.0);
  // quadrant q = n mod 4: (sin, cos) = (sn, cs), (cs, -sn), (-sn, -cs), (-cs, sn)
  const int q = (int)n & 3;
  const double a = (q & 1) ? cs : sn;
  const double b = (q & 1) ? sn : cs;
  *s = (q & 2) ? -a : a;
  *c = ((q + 1) & 2) ? -b : b;
}

}  // namespace vegas
