// Double-precision log and reciprocal for the property kernels.
//
// The device library's log guards every special case and costs about twice the VALU
// instructions of the arithmetic below in our gfx950 build; its division is a correctly
// rounded sequence of about twice the cost of a refined reciprocal:
//   log   — x = m 2^e with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(f), f = (m-1)/(m+1),
//           |f| <= 0.1716, by the odd series of atanh to f^21 (truncation < 1e-18), and
//           e ln2 with ln2 split into a 24-bit head and a tail.
//   rcp   — hardware reciprocal refined by two Newton-Raphson steps.
//   exp_tab — the same with 64 table values 2^(j/64) and a degree-5 polynomial (below).
//   exp   — x = n ln2 + r with n = rint(x log2 e), |r| <= ln2/2 (ln 2 split as for log),
//           e^r by its Taylor series to r^13 (truncation below 5e-18 relative), scaled
//           by 2^n with ldexp; no special-case branches (the device library's exp
//           guards them and costs about a fifth more).
// All are within two units in the last place; host builds of log and exp are checked
// against long-double libm in the test-suite.  log of a non-positive argument is NaN;
// exp takes finite arguments (overflow gives inf, underflow 0 through subnormals, NaN
// stays NaN; -inf is not supported).
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define FM_HD __host__ __device__
#else
#define FM_HD
#endif

namespace props {
namespace fm {

constexpr double kLn2Hi = 0.6931471526622772;      // ln 2 rounded to 24 significant bits
constexpr double kLn2Lo = 2.7897668087737545e-08;  // ln 2 - kLn2Hi
constexpr double kSqrtHalf = 0.7071067811865476;

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

FM_HD inline double exp(double x)
{
    const double n = std::rint(x * 1.4426950408889634);   // log2(e)
    double r = std::fma(-n, kLn2Hi, x);
    r = std::fma(-n, kLn2Lo, r);
    // sum_{k=0}^{13} r^k / k!
    double p = 1.0 / 6227020800.0;
    p = std::fma(p, r, 1.0 / 479001600.0);
    p = std::fma(p, r, 1.0 / 39916800.0);
    p = std::fma(p, r, 1.0 / 3628800.0);
    p = std::fma(p, r, 1.0 / 362880.0);
    p = std::fma(p, r, 1.0 / 40320.0);
    p = std::fma(p, r, 1.0 / 5040.0);
    p = std::fma(p, r, 1.0 / 720.0);
    p = std::fma(p, r, 1.0 / 120.0);
    p = std::fma(p, r, 1.0 / 24.0);
    p = std::fma(p, r, 1.0 / 6.0);
    p = std::fma(p, r, 0.5);
    p = std::fma(p, r, 1.0);
    p = std::fma(p, r, 1.0);
    return std::ldexp(p, (int)n);
}

// exp with a table of the 64 values 2^(j/64) (correctly rounded), typically an LDS copy:
// x = (64 m + j) ln2/64 + r with |r| <= ln2/128 (ln2/64 split into a 35-bit head and a
// tail), e^x = 2^m 2^(j/64) e^r, e^r by its Taylor series to r^5 (truncation below 4e-17
// relative).  Fourteen instructions and one table read against twenty for exp; the same
// range behaviour (overflow inf, underflow 0 through subnormals, NaN stays NaN).
constexpr double k64Log2e = 92.33248261689366;            // 64/ln2
constexpr double kLn2o64Hi = 0.010830424696450791;        // ln2/64 to 35 significant bits
constexpr double kLn2o64Lo = -2.0164562921995537e-13;     // ln2/64 - kLn2o64Hi

FM_HD inline double exp_tab(double x, const double *tab64)
{
    const double k = std::rint(x * k64Log2e);
    const int ki = (int)k;
    double r = std::fma(-k, kLn2o64Hi, x);
    r = std::fma(-k, kLn2o64Lo, r);
    // e^r - 1 = r + r (r/2 + r^2/6 + r^3/24 + r^4/120), then t + t (e^r - 1): one rounding
    double q = 1.0 / 120.0;
    q = std::fma(q, r, 1.0 / 24.0);
    q = std::fma(q, r, 1.0 / 6.0);
    q = std::fma(q, r, 0.5);
    q = q * r;
    q = std::fma(q, r, r);
    const double t = tab64[ki & 63];
    return std::ldexp(std::fma(t, q, t), ki >> 6);
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton-Raphson steps
// (r <- r + r (1 - x r^2)/2, the relative error squaring each time), within two ulp;
// sqrt(x) then follows as x * rsqrt(x) without the correctly rounded square root's cost.
FM_HD inline double rsqrt(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rsq(x);
    double e = std::fma(-x * r, r, 1.0);
    r = std::fma(0.5 * r, e, r);
    e = std::fma(-x * r, r, 1.0);
    return std::fma(0.5 * r, e, r);
#else
    return 1.0 / std::sqrt(x);
#endif
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
