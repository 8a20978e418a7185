// FP64 log, exp and erf for the op-list kernels.
//
// Both are branch-free (every lane of a wave runs the same instructions)
// and keep their working precision in plain doubles; the constants come
// from gen_dmath.py.  Measured against the host C library they stay
// within a few ulp over the whole double range.
#pragma once
#include <hip/hip_runtime.h>

#include "dmath_coef.h"

namespace dfx {

// p(x) for coefficients c[0] + c[1] x + ... (Horner's rule)
template <int N> __device__ __forceinline__ double dm_poly(const double (&c)[N], double x) {
  double p = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) p = __builtin_fma(p, x, c[i]);
  return p;
}

// 1 / d to about an ulp: the hardware estimate refined by two Newton steps
__device__ __forceinline__ double dm_recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __builtin_fma(-d, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-d, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Natural logarithm.  x = 2^k m with m in [sqrt(1/2), sqrt(2)); with
// f = m - 1 and s = f / (2 + f), log m = 2 atanh(s) = 2s + s R(s^2), and
// 2s = f - s f, so log m = f - (f^2/2 - s (f^2/2 + R)) keeps the leading
// term f exact.  ln 2 is split so that k ln2_hi is exact.
__device__ __forceinline__ double dm_log(double x) {
  int k = __builtin_amdgcn_frexp_exp(x);
  double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1), denormals included
  const bool lo = m < dmc::SQRT_HALF;
  m = lo ? m + m : m;
  k = lo ? k - 1 : k;
  const double f = m - 1.0;  // exact
  const double d = 2.0 + f;
  const double r = dm_recip(d);
  double s = f * r;
  s = __builtin_fma(__builtin_fma(-d, s, f), r, s);  // one correction of the quotient
  const double z = s * s;
  const double R = z * dm_poly(dmc::LOG_Q, z);
  const double hfsq = 0.5 * (f * f);
  const double lm = f - (hfsq - s * (hfsq + R));
  const double dk = (double)k;
  double y = __builtin_fma(dk, dmc::LN2_HI, __builtin_fma(dk, dmc::LN2_LO, lm));
  // +inf -> +inf; +-0 -> -inf; negative or NaN -> NaN
  y = x == __builtin_inf() ? x : y;
  y = x == 0.0 ? -__builtin_inf() : y;
  y = x < 0.0 ? __builtin_nan("") : y;
  return x != x ? x : y;
}

// exp(y) for finite y in [-746, 710]: y = n ln 2 + r with |r| <= ln2 / 2,
// exp y = 2^n E(r), one rounding in the final scaling
__device__ __forceinline__ double dm_exp_mid(double y) {
  const double n = __builtin_rint(y * dmc::INV_LN2);
  double r = __builtin_fma(-n, dmc::LN2_HI, y);
  r = __builtin_fma(-n, dmc::LN2_LO, r);
  return __builtin_amdgcn_ldexp(dm_poly(dmc::EXP_E, r), (int)n);
}

// Exponential over the whole double range: x is clamped to [-746, 710]
// (beyond, the result is 0 or inf anyway), reduced to x = n ln 2 + r with
// |r| <= ln2 / 2, and scaled by one ldexp, which also rounds results in
// the overflow and denormal range.
__device__ __forceinline__ double dm_exp(double x) {
  const double xc = x < -746.0 ? -746.0 : (x > 710.0 ? 710.0 : x);
  const double y = dm_exp_mid(xc);
  return x != x ? x : y;
}

// Error function.  |x| < 0.84375: erf x = x P(x^2).  Above: erf |x| =
// 1 - erfc |x| with erfc x = exp(-x^2) H(t), t = 1 / (1 + p x), a form in
// which erfc x exp(x^2) is smooth enough for one polynomial up to x = 6;
// from there on 1 - erfc rounds to 1 (erfc 6 < 2^-55), so |x| is clamped.
// Both forms are evaluated and the result selected.
__device__ __forceinline__ double dm_erf(double x) {
  const double ax = __builtin_fabs(x);
  const double ys = x * dm_poly(dmc::ERF_P, x * x);
  const double xc = ax < dmc::ERF_ONE ? ax : dmc::ERF_ONE;
  const double t = dm_recip(__builtin_fma(dmc::ERFC_P, xc, 1.0));
  const double ec = dm_exp_mid(-(xc * xc)) * dm_poly(dmc::ERFC_H, t);
  const double yl = __builtin_copysign(1.0 - ec, x);
  const double y = ax < dmc::ERF_SPLIT ? ys : yl;
  return x != x ? x : y;
}

}  // namespace dfx
