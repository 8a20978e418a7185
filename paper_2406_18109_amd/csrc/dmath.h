// FP64 log, exp and erf for the op-list kernels.
//
// All are branch-free (every lane of a wave runs the same instructions)
// and keep their working precision in plain doubles; the constants come
// from gen_dmath.py.  Measured against the host C library they stay
// within a few ulp over the whole double range.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "dmath_coef.h"

namespace dfx {

// Every function works on N values at once, statement by statement, so
// that one materialised coefficient serves N fused multiply-adds and the N
// dependency chains interleave; the arithmetic on each value is the same
// for any N.
// A scheduling barrier after each Horner step keeps the N multiply-adds of
// the step together; otherwise the scheduler serialises the chains again
// and the coefficients are rematerialised for each value.
#ifndef DFX_DM_SCHED
#define DFX_DM_SCHED 1
#endif
#define DM_EACH(...) _Pragma("unroll") for (int j = 0; j < N; ++j) { __VA_ARGS__ }

// p = c[0] + c[1] x + ... (Horner's rule)
template <int N, int M>
__device__ __forceinline__ void dm_poly(const double (&c)[M], const double (&x)[N], double (&p)[N]) {
  DM_EACH(p[j] = c[M - 1];)
#pragma unroll
  for (int i = M - 2; i >= 0; --i) {
    DM_EACH(p[j] = __builtin_fma(p[j], x[j], c[i]);)
#if DFX_DM_SCHED
    if constexpr (N > 1) __builtin_amdgcn_sched_barrier(0);
#endif
  }
}

// 1 / d to about an ulp: the hardware estimate refined by two Newton steps
template <int N> __device__ __forceinline__ void dm_recip(const double (&d)[N], double (&r)[N]) {
  DM_EACH(r[j] = __builtin_amdgcn_rcp(d[j]);)
  DM_EACH(r[j] = __builtin_fma(r[j], __builtin_fma(-d[j], r[j], 1.0), r[j]);)
  DM_EACH(r[j] = __builtin_fma(r[j], __builtin_fma(-d[j], r[j], 1.0), r[j]);)
}

// Natural logarithm.  x = 2^k m with m in [sqrt(1/2), sqrt(2)); with
// f = m - 1 and s = f / (2 + f), log m = 2 atanh(s) = 2s + s R(s^2), and
// 2s = f - s f, so log m = f - (f^2/2 - s (f^2/2 + R)) keeps the leading
// term f exact.  ln 2 is split so that k ln2_hi is exact.
template <int N> __device__ __forceinline__ void dm_log(double (&v)[N]) {
  double f[N], d[N], r[N], s[N], z[N], q[N];
  int k[N];
  DM_EACH(
    const int e = __builtin_amdgcn_frexp_exp(v[j]);
    double m = __builtin_amdgcn_frexp_mant(v[j]);  // [0.5, 1), denormals included
    const bool lo = m < dmc::SQRT_HALF;
    m = lo ? m + m : m;
    k[j] = lo ? e - 1 : e;
    f[j] = m - 1.0;  // exact
    d[j] = 2.0 + f[j];)
  dm_recip(d, r);
  DM_EACH(
    const double s0 = f[j] * r[j];
    s[j] = __builtin_fma(__builtin_fma(-d[j], s0, f[j]), r[j], s0);  // one correction of the quotient
    z[j] = s[j] * s[j];)
  dm_poly(dmc::LOG_Q, z, q);
  DM_EACH(
    const double x = v[j];
    const double R = z[j] * q[j];
    const double hfsq = 0.5 * (f[j] * f[j]);
    const double lm = f[j] - (hfsq - s[j] * (hfsq + R));
    const double dk = (double)k[j];
    double y = __builtin_fma(dk, dmc::LN2_HI, __builtin_fma(dk, dmc::LN2_LO, lm));
    // +inf -> +inf; +-0 -> -inf; negative or NaN -> NaN
    y = x == __builtin_inf() ? x : y;
    y = x == 0.0 ? -__builtin_inf() : y;
    y = x < 0.0 ? __builtin_nan("") : y;
    v[j] = x != x ? x : y;)
}

// exp(y) for finite y in [-746, 710]: y = n ln 2 + r with |r| <= ln2 / 2,
// exp y = 2^n E(r), one rounding in the final scaling
template <int N> __device__ __forceinline__ void dm_exp_mid(const double (&y)[N], double (&out)[N]) {
  double n[N], r[N], e[N];
  DM_EACH(
    n[j] = __builtin_rint(y[j] * dmc::INV_LN2);
    r[j] = __builtin_fma(-n[j], dmc::LN2_LO, __builtin_fma(-n[j], dmc::LN2_HI, y[j]));)
  dm_poly(dmc::EXP_E, r, e);
  DM_EACH(out[j] = __builtin_amdgcn_ldexp(e[j], (int)n[j]);)
}

// Exponential over the whole double range: x is clamped to [-746, 710]
// (beyond, the result is 0 or inf anyway), reduced to x = n ln 2 + r with
// |r| <= ln2 / 2, and scaled by one ldexp, which also rounds results in
// the overflow and denormal range.
template <int N> __device__ __forceinline__ void dm_exp(double (&v)[N]) {
  double xc[N], y[N];
  DM_EACH(xc[j] = v[j] < -746.0 ? -746.0 : (v[j] > 710.0 ? 710.0 : v[j]);)
  dm_exp_mid(xc, y);
  DM_EACH(v[j] = v[j] != v[j] ? v[j] : y[j];)
}

// Error function.  |x| < 0.84375: erf x = x P(x^2).  Above: erf |x| =
// 1 - erfc |x| with erfc x = exp(-x^2) H(t), t = 1 / (1 + p x), a form in
// which erfc x exp(x^2) is smooth enough for one polynomial up to x = 6;
// from there on 1 - erfc rounds to 1 (erfc 6 < 2^-55), so |x| is clamped.
// Both forms are evaluated and the result selected.
template <int N> __device__ __forceinline__ void dm_erf(double (&v)[N]) {
  double u[N], p[N], d[N], t[N], h[N], w[N], e[N];
  DM_EACH(
    const double ax = __builtin_fabs(v[j]);
    const double xc = ax < dmc::ERF_ONE ? ax : dmc::ERF_ONE;
    u[j] = v[j] * v[j];
    d[j] = __builtin_fma(dmc::ERFC_P, xc, 1.0);
    w[j] = -(xc * xc);)
  dm_poly(dmc::ERF_P, u, p);
  dm_recip(d, t);
  dm_poly(dmc::ERFC_H, t, h);
  dm_exp_mid(w, e);
  DM_EACH(
    const double x = v[j];
    const double ys = x * p[j];
    const double yl = __builtin_copysign(1.0 - e[j] * h[j], x);
    const double y = __builtin_fabs(x) < dmc::ERF_SPLIT ? ys : yl;
    v[j] = x != x ? x : y;)
}

#undef DM_EACH

}  // namespace dfx
