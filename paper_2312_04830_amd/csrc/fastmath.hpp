// Double-precision exp, expm1, log and reciprocal for the property kernels.
//
// The device library's general routines guard every special case (overflow, subnormal
// scaling, NaN and infinity paths); the property path only evaluates them on finite,
// moderate arguments, so these versions keep just the arithmetic:
//   exp   — Cody & Waite argument reduction x = k ln2 + r, |r| <= ln2/2, with ln2 split
//           into a 24-bit head (k * head exact) and a tail; e^r by its Taylor series to
//           r^13 (truncation < 5e-18 relative); scaling by 2^k with ldexp.
//   expm1 — the same series without its constant term for |x| < ln2/2, exp(x) - 1 beyond.
//   log   — x = m 2^e with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(f), f = (m-1)/(m+1),
//           |f| <= 0.1716, by the odd series of atanh to f^21 (truncation < 1e-18).
//   rcp   — hardware reciprocal refined by two Newton-Raphson steps.
// Results are within a few units in the last place for the arguments the kernels use; a
// host build of the same code is checked against long-double libm in the test-suite.
// NaN propagates; exp underflows to 0 below -745.2 and overflows above 709.78; log of a
// non-positive argument is NaN.
#pragma once

#include <cmath>

#if defined(__HIP_DEVICE_COMPILE__)
#define FM_QUAL __device__ __forceinline__
#else
#define FM_QUAL inline
#endif
#if defined(__HIPCC__)
#define FM_HD __host__ __device__
#else
#define FM_HD
#endif

namespace props {
namespace fm {

constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2Hi = 0.6931471526622772;      // ln 2 rounded to 24 significant bits
constexpr double kLn2Lo = 2.7897668087737545e-08;  // ln 2 - kLn2Hi
constexpr double kSqrtHalf = 0.7071067811865476;

// 1/n! for n = 13 .. 2 (Horner order), exact rationals rounded to double
constexpr double kInvFact[12] = {
    1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0,
    1.0 / 362880.0,     1.0 / 40320.0,     1.0 / 5040.0,     1.0 / 720.0,
    1.0 / 120.0,        1.0 / 24.0,        1.0 / 6.0,        1.0 / 2.0};

// sum_{n>=2} r^(n-2) / n!  (so e^r = 1 + r + r^2 * tail(r))
FM_HD inline double exp_tail(double r)
{
    double p = kInvFact[0];
#pragma unroll
    for (int i = 1; i < 12; i++) p = std::fma(p, r, kInvFact[i]);
    return p;
}

FM_HD inline double exp(double x)
{
    double k = std::rint(x * kLog2e);
    k = std::fmin(std::fmax(k, -1100.0), 1100.0);
    double r = std::fma(-k, kLn2Hi, x);
    r = std::fma(-k, kLn2Lo, r);
    const double p = std::fma(r * r, exp_tail(r), r) + 1.0;
    const double y = std::ldexp(p, (int)k);
    return (x < -745.2) ? 0.0 : ((x > 709.78) ? HUGE_VAL : y);
}

FM_HD inline double expm1(double x)
{
    if (std::fabs(x) < 0.34657359027997264) return std::fma(x * x, exp_tail(x), x);
    return exp(x) - 1.0;
}

FM_HD inline double log(double x)
{
    int e;
    double m = std::frexp(x, &e);          // m in [0.5, 1)
    if (m < kSqrtHalf) {
        m *= 2.0;
        e -= 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double f2 = f * f;
    // atanh(f)/f = sum f^(2j) / (2j + 1), j = 0..10
    double s = 1.0 / 21.0;
    s = std::fma(s, f2, 1.0 / 19.0);
    s = std::fma(s, f2, 1.0 / 17.0);
    s = std::fma(s, f2, 1.0 / 15.0);
    s = std::fma(s, f2, 1.0 / 13.0);
    s = std::fma(s, f2, 1.0 / 11.0);
    s = std::fma(s, f2, 1.0 / 9.0);
    s = std::fma(s, f2, 1.0 / 7.0);
    s = std::fma(s, f2, 1.0 / 5.0);
    s = std::fma(s, f2, 1.0 / 3.0);
    const double t = 2.0 * f;
    const double ed = (double)e;
    // log x = e ln2 + 2 f (1 + f2 s), tail term added first
    const double y = std::fma(ed, kLn2Hi, std::fma(t * f2, s, std::fma(ed, kLn2Lo, t)));
    return (x > 0.0) ? y : NAN;
}

FM_HD inline double rcp(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    double e = std::fma(-x, r, 1.0);
    r = std::fma(r, e, r);
    e = std::fma(-x, r, 1.0);
    return std::fma(r, e, r);
#else
    return 1.0 / x;
#endif
}

}  // namespace fm
}  // namespace props
