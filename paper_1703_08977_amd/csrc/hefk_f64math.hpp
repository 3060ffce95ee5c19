// hefk_f64math.hpp -- binary64 elementary functions for the walker step, written
// for the arguments the step produces (finite, and positive where a logarithm or
// a root is taken), without the special-case handling of a general library:
//
//   log(x)      x = m 2^e, m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s),
//               s = (m - 1)/(m + 1), |s| <= 0.1716: 2 s (1 + z R(z)), z = s^2, with R a
//               degree-6 polynomial fitted to (atanh(s)/s - 1)/z.
//   sincos(2 pi u), u in [0, 1): x = 2u = k/2 + y, |y| <= 1/4 (exact), the angle k pi/2 + pi y:
//               sin(pi y) = y S(y^2), cos(pi y) = C(y^2), polynomials of degree 6 and 7
//               fitted to sin(pi y)/y and cos(pi y); quadrant k mod 4.
//   exp(x)      x <= 0: x = k ln 2 + r, |r| <= ln2/2 (two-part ln 2), a degree-11
//               polynomial fitted to e^r, then 2^k by exponent scaling.
//   expm1(x)    x <= 0: the same reduction, e^r - 1 = r + r^2 Q(r) with a degree-10
//               polynomial Q fitted to (e^r - 1 - r)/r^2, then 2^k (e^r - 1) + 2^k - 1.
// The polynomial coefficients (below) are weighted least-squares fits on those ranges in
// high precision, rounded to binary64 one at a time from the lowest order with the rest
// refitted (f64_coeffs.py prints them); their approximation errors are 0.003-0.35 units of
// 2^-53, below the rounding of the evaluation.
//   sqrt(x)     x >= 0: y ~ 1/sqrt(x) from the hardware seed, two Newton steps on
//               g = x y, h = y/2 (Goldschmidt's coupled iteration), x = 0 -> 0.
//   1/x         hardware reciprocal seed and two Newton steps, x = 0 -> inf.
//   sqrt and 1/sqrt of a squared distance together: the square root's iteration, then one
//               Newton step on its reciprocal half.
// sqrt_pos, rcp_nz and log_normal are the same arithmetic without the tests for
// zero and subnormal arguments: the walker step calls them where its arguments
// cannot be zero (a uniform of the noise, 1 + ..., a distance), and an argument
// that is zero after all (an electron exactly on the nucleus) gives NaN there,
// which marks the walker non-finite as the infinity of the tested form would.
// Each is within a few units in the last place of the correctly rounded value over
// those arguments.  Host builds use the same code (seeds from the C library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#ifndef HD
#define HD __host__ __device__ __forceinline__
#endif

namespace hefk {
namespace f64 {

// ---- polynomial coefficients (f64_coeffs.py) ----
// SIN_PI: degree 6 on [0.0, 0.0625], max error 0.351 x 2^-53 (relative)
constexpr double kSIN_PI0 = 0x1.921fb54442d18p+1;  // 3.1415926535897931
constexpr double kSIN_PI1 = -0x1.4abbce625be09p+2;  // -5.1677127800499045
constexpr double kSIN_PI2 = 0x1.466bc67754ffbp+1;  // 2.5501640398670111
constexpr double kSIN_PI3 = -0x1.32d2ccdfe8d0ap-1;  // -0.59926452859181834
constexpr double kSIN_PI4 = 0x1.50782d5e89456p-4;  // 0.082145859931715165
constexpr double kSIN_PI5 = -0x1.e2fe766f665bap-8;  // -0.0073699034832314606
constexpr double kSIN_PI6 = 0x1.e357bb6294ae5p-12;  // 0.00046095152189200148
// COS_PI: degree 7 on [0.0, 0.0625], max error 0.003 x 2^-53 (absolute)
constexpr double kCOS_PI0 = 0x1.0000000000000p+0;  // 1
constexpr double kCOS_PI1 = -0x1.3bd3cc9be45dep+2;  // -4.934802200544679
constexpr double kCOS_PI2 = 0x1.03c1f081b5a65p+2;  // 4.0587121264166841
constexpr double kCOS_PI3 = -0x1.55d3c7e3c2d7bp+0;  // -1.3352627688462622
constexpr double kCOS_PI4 = 0x1.e1f5067b057f8p-3;  // 0.23533062994891885
constexpr double kCOS_PI5 = -0x1.a6d1e6b52f412p-6;  // -0.025806880283870078
constexpr double kCOS_PI6 = 0x1.f9c840cb57470p-10;  // 0.001929406122904067
constexpr double kCOS_PI7 = -0x1.b14b5b3de0d19p-14;  // -0.00010330542587948625
// LOG_R: degree 6 on [0.0, 0.0294373], max error 0.012 x 2^-53 (relative to 1 + z R)
constexpr double kLOG_R0 = 0x1.5555555555594p-2;  // 0.33333333333333681
constexpr double kLOG_R1 = 0x1.999999997f77cp-3;  // 0.19999999999702911
constexpr double kLOG_R2 = 0x1.2492494235b74p-3;  // 0.14285714371973379
constexpr double kLOG_R3 = 0x1.c71c51dbbbd75p-4;  // 0.11111099220192051
constexpr double kLOG_R4 = 0x1.746646d7fcebcp-4;  // 0.090917851193632993
constexpr double kLOG_R5 = 0x1.39a108cae2047p-4;  // 0.076569589944598268
constexpr double kLOG_R6 = 0x1.2f0b96857276dp-4;  // 0.073985660527936495
// EXP: degree 11 on [-0.346574, 0.346574], max error 0.037 x 2^-53 (relative)
constexpr double kEXP0 = 0x1.0000000000000p+0;  // 1
constexpr double kEXP1 = 0x1.0000000000000p+0;  // 1
constexpr double kEXP2 = 0x1.000000000000bp-1;  // 0.50000000000000122
constexpr double kEXP3 = 0x1.555555555550fp-3;  // 0.16666666666666471
constexpr double kEXP4 = 0x1.55555555502a6p-5;  // 0.041666666666519789
constexpr double kEXP5 = 0x1.1111111122b4fp-7;  // 0.0083333333334586739
constexpr double kEXP6 = 0x1.6c16c18529f74p-10;  // 0.0013888888945902929
constexpr double kEXP7 = 0x1.a01a014493a95p-13;  // 0.00019841269581140757
constexpr double kEXP8 = 0x1.a01997cd32dd4p-16;  // 2.4801491055366002e-05
constexpr double kEXP9 = 0x1.71deec77b25ddp-19;  // 2.7557521738760222e-06
constexpr double kEXP10 = 0x1.28af3b651cd0bp-22;  // 2.7630897243072546e-07
constexpr double kEXP11 = 0x1.add741be6cfcap-26;  // 2.5020030264367061e-08
// EXPM1_Q: degree 10 on [-0.346574, 0.346574], max error 0.003 x 2^-53 (relative to e^r - 1)
constexpr double kEXPM1_Q0 = 0x1.0000000000000p-1;  // 0.5
constexpr double kEXPM1_Q1 = 0x1.5555555555559p-3;  // 0.16666666666666677
constexpr double kEXPM1_Q2 = 0x1.555555555554cp-5;  // 0.041666666666666602
constexpr double kEXPM1_Q3 = 0x1.111111110f65bp-7;  // 0.0083333333333214712
constexpr double kEXPM1_Q4 = 0x1.6c16c16c1b325p-10;  // 0.0013888888888928333
constexpr double kEXPM1_Q5 = 0x1.a01a01afff406p-13;  // 0.00019841269886447537
constexpr double kEXPM1_Q6 = 0x1.a01a018b42992p-16;  // 2.4801587227543639e-05
constexpr double kEXPM1_Q7 = 0x1.71ddf81dc16bbp-19;  // 2.7557243943457041e-06
constexpr double kEXPM1_Q8 = 0x1.27e5198d2f157p-22;  // 2.7557361976704003e-07
constexpr double kEXPM1_Q9 = 0x1.af5f0dedded80p-26;  // 2.5109114724470039e-08
constexpr double kEXPM1_Q10 = 0x1.1f1017eaef034p-29;  // 2.0886572380207129e-09


HD uint64_t bits(double x)
{
    uint64_t b;
    __builtin_memcpy(&b, &x, 8);
    return b;
}
HD double from_bits(uint64_t b)
{
    double x;
    __builtin_memcpy(&x, &b, 8);
    return x;
}

HD double rcp_seed(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcp(x);
#else
    return 1.0 / x;
#endif
}
HD double rsq_seed(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rsq(x);
#else
    return 1.0 / ::sqrt(x);
#endif
}

// 1/x for finite x != 0: seed and two Newton steps r <- r + r (1 - x r)
// (x = 0 gives NaN: the form for arguments that cannot be zero)
HD double rcp_nz(double x)
{
    double r = rcp_seed(x);
    double e = ::fma(-x, r, 1.0);
    r = ::fma(r, e, r);
    e = ::fma(-x, r, 1.0);
    r = ::fma(r, e, r);
    return r;
}

// 1/x, x = +-0 -> +-inf
HD double rcp(double x)
{
    const double r = rcp_nz(x);
    return x == 0.0 ? from_bits(bits(x) | 0x7FF0000000000000ull) : r;
}

// sqrt(x) for finite x > 0 (x = 0 gives NaN: the form for arguments that cannot be zero)
HD double sqrt_pos(double x)
{
    const double y = rsq_seed(x);
    double g = x * y, h = 0.5 * y;
    double r = ::fma(-g, h, 0.5);
    g = ::fma(g, r, g);
    h = ::fma(h, r, h);
    const double d = ::fma(-g, g, x);
    g = ::fma(d, h, g);
    return g;
}

// r = sqrt(q) and i = 1/r for finite q > 0 from one reciprocal square root seed: the coupled
// iteration of sqrt_pos gives r, and i = 2h, Newton-refined once against the final r
HD void dist_inv(double q, double& r, double& i)
{
    const double y = rsq_seed(q);
    double g = q * y, h = 0.5 * y;
    const double e = ::fma(-g, h, 0.5);
    g = ::fma(g, e, g);
    h = ::fma(h, e, h);
    const double d = ::fma(-g, g, q);
    r = ::fma(d, h, g);
    const double i0 = 2.0 * h;
    i = ::fma(i0, ::fma(-r, i0, 1.0), i0);
}

// sqrt(x), x >= 0
HD double sqrt(double x)
{
    const double g = sqrt_pos(x);
    return x == 0.0 ? 0.0 : g;
}

// log(x) - e_off ln 2 for finite x >= 2^-1000 (the exponent offset enters before the
// split multiplication by ln 2)
HD double log_scaled(double x, double e_off)
{
    const uint64_t b = bits(x);
    int e = (int)((b >> 52) & 0x7FF) - 1023;
    double m = from_bits((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);  // [1, 2)
    const bool big = m > 1.4142135623730951;
    m = big ? 0.5 * m : m;
    e = big ? e + 1 : e;
    const double s = (m - 1.0) * rcp_nz(m + 1.0);
    const double z = s * s;
    // R(z) ~ (atanh(s)/s - 1)/z = 1/3 + z/5 + z^2/7 + ...
    double p = kLOG_R6;
    p = ::fma(p, z, kLOG_R5);
    p = ::fma(p, z, kLOG_R4);
    p = ::fma(p, z, kLOG_R3);
    p = ::fma(p, z, kLOG_R2);
    p = ::fma(p, z, kLOG_R1);
    p = ::fma(p, z, kLOG_R0);
    const double lm = 2.0 * s + 2.0 * s * z * p;  // 2 s (1 + z p), the leading term kept apart
    const double ln2_hi = 6.93147180369123816490e-01;  // ln 2 split: high part has 21 trailing zero bits
    const double ln2_lo = 1.90821492927058770002e-10;
    const double fe = (double)e - e_off;
    return fe * ln2_hi + (lm + fe * ln2_lo);
}

// log(x) for finite x >= 2^-1000 (the form for arguments bounded away from zero and
// from the subnormal range, such as the uniforms of the noise)
HD double log_normal(double x) { return log_scaled(x, 0.0); }

// log(x), x > 0 finite (0 -> -inf); arguments below 2^-1000 are scaled by 2^100 first
HD double log(double x)
{
    const bool tiny = x < 0x1p-1000;
    const double r = log_scaled(tiny ? x * 0x1p100 : x, tiny ? 100.0 : 0.0);
    return x == 0.0 ? -INFINITY : r;
}

// -2 log(u) for the Box-Muller radius, u a uniform of the noise (u >= 2^-33)
HD double neg2log(double u) { return -2.0 * log_normal(u); }

// sin(2 pi u), cos(2 pi u) for u in [0, 1)
HD void sincos2pi(double u, double* s_out, double* c_out)
{
    const double x = 2.0 * u;            // exact
    const double k = ::rint(2.0 * x);    // quadrant index: x = k/2 + y
    const double y = ::fma(-0.5, k, x);  // exact, |y| <= 1/4: the angle is k pi/2 + pi y
    const double w = y * y;
    // sin(pi y) = y S(w), S(w) ~ pi - pi^3 w / 6 + ...
    double ps = kSIN_PI6;
    ps = ::fma(ps, w, kSIN_PI5);
    ps = ::fma(ps, w, kSIN_PI4);
    ps = ::fma(ps, w, kSIN_PI3);
    ps = ::fma(ps, w, kSIN_PI2);
    ps = ::fma(ps, w, kSIN_PI1);
    ps = ::fma(ps, w, kSIN_PI0);
    const double sn = y * ps;
    // cos(pi y) = C(w), C(w) ~ 1 - pi^2 w / 2 + ...; C(0) = kCOS_PI0 = 1
    double pc = kCOS_PI7;
    pc = ::fma(pc, w, kCOS_PI6);
    pc = ::fma(pc, w, kCOS_PI5);
    pc = ::fma(pc, w, kCOS_PI4);
    pc = ::fma(pc, w, kCOS_PI3);
    pc = ::fma(pc, w, kCOS_PI2);
    pc = ::fma(pc, w, kCOS_PI1);
    const double cs = ::fma(pc, w, kCOS_PI0);
    // angle = k pi/2 + t: odd quadrants exchange sin and cos; sin is negated in
    // quadrants 2, 3 and cos in quadrants 1, 2 (selects, no branches)
    const uint32_t q = (uint32_t)(int)k;
    const double a = (q & 1u) ? cs : sn;
    const double b = (q & 1u) ? sn : cs;
    // the sign flips as xors of the sign bit: bit 1 of q for sin, of q + 1 for cos
    *s_out = from_bits(bits(a) ^ ((uint64_t)(q & 2u) << 62));
    *c_out = from_bits(bits(b) ^ ((uint64_t)((q + 1u) & 2u) << 62));
}

// e^x for x <= 0 (and moderate x > 0)
HD double exp(double x)
{
    const double k = ::rint(x * 1.44269504088896340736);  // x / ln 2
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    const double r = ::fma(-k, ln2_lo, ::fma(-k, ln2_hi, x));  // |r| <= ln2 / 2
    double p = kEXP11;
    p = ::fma(p, r, kEXP10);
    p = ::fma(p, r, kEXP9);
    p = ::fma(p, r, kEXP8);
    p = ::fma(p, r, kEXP7);
    p = ::fma(p, r, kEXP6);
    p = ::fma(p, r, kEXP5);
    p = ::fma(p, r, kEXP4);
    p = ::fma(p, r, kEXP3);
    p = ::fma(p, r, kEXP2);
    p = ::fma(p, r, kEXP1);
    p = ::fma(p, r, kEXP0);
    return k < -1100.0 ? 0.0 : ::ldexp(p, (int)k);
}

// e^x - 1 for x <= 0: x = k ln 2 + r as in exp, e^r - 1 = r + r^2 Q(r)
// (no cancellation: the sum starts at r), then e^x - 1 = 2^k (e^r - 1) + (2^k - 1),
// whose second term is exact; k = 0 returns the series itself
HD double expm1_neg(double x)
{
    const double k = ::rint(x * 1.44269504088896340736);
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    const double r = ::fma(-k, ln2_lo, ::fma(-k, ln2_hi, x));  // |r| <= ln2 / 2
    double q = kEXPM1_Q10;
    q = ::fma(q, r, kEXPM1_Q9);
    q = ::fma(q, r, kEXPM1_Q8);
    q = ::fma(q, r, kEXPM1_Q7);
    q = ::fma(q, r, kEXPM1_Q6);
    q = ::fma(q, r, kEXPM1_Q5);
    q = ::fma(q, r, kEXPM1_Q4);
    q = ::fma(q, r, kEXPM1_Q3);
    q = ::fma(q, r, kEXPM1_Q2);
    q = ::fma(q, r, kEXPM1_Q1);
    q = ::fma(q, r, kEXPM1_Q0);
    const double em = ::fma(r * r, q, r);  // r + r^2 Q(r)
    const double p2 = k < -1100.0 ? 0.0 : ::ldexp(1.0, (int)k);  // 2^k
    return ::fma(p2, em, p2 - 1.0);
}

}  // namespace f64
}  // namespace hefk
