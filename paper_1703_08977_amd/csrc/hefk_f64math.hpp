// hefk_f64math.hpp -- binary64 elementary functions for the walker step, written
// for the arguments the step produces (finite, and positive where a logarithm or
// a root is taken), without the special-case handling of a general library:
//
//   log(x)      x = m 2^e, m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(s),
//               s = (m - 1)/(m + 1), |s| <= 0.1716, by its Taylor series to s^21.
//   sincos(2 pi u), u in [0, 1): x = 2u = k/2 + y, |y| <= 1/4, t = pi y,
//               Taylor series of sin t to t^17 and cos t to t^16, quadrant k mod 4.
//   exp(x)      x <= 0: x = k ln 2 + r, |r| <= ln2/2 (two-part ln 2), Taylor series
//               of e^r to r^13, then 2^k by exponent scaling.
//   expm1(x)    x <= 0: the same reduction, e^r - 1 by its series, 2^k (e^r - 1) + 2^k - 1.
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
    // sum_{k=0}^{10} z^k / (2k + 1); the next term, z^11 / 23 <= 7e-19, is below the rounding
    double p = 1.0 / 21.0;
    p = ::fma(p, z, 1.0 / 19.0);
    p = ::fma(p, z, 1.0 / 17.0);
    p = ::fma(p, z, 1.0 / 15.0);
    p = ::fma(p, z, 1.0 / 13.0);
    p = ::fma(p, z, 1.0 / 11.0);
    p = ::fma(p, z, 1.0 / 9.0);
    p = ::fma(p, z, 1.0 / 7.0);
    p = ::fma(p, z, 1.0 / 5.0);
    p = ::fma(p, z, 1.0 / 3.0);
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
    const double y = ::fma(-0.5, k, x);  // exact, |y| <= 1/4
    const double t = 3.14159265358979323846 * y;
    const double z = t * t;
    // sin t = t (1 + sum_{j=1}^{8} (-1)^j z^j / (2j+1)!)
    double ps = 1.0 / 355687428096000.0;         // + 1/17!
    ps = ::fma(ps, z, -1.0 / 1307674368000.0);   // - 1/15!
    ps = ::fma(ps, z, 1.0 / 6227020800.0);       // + 1/13!
    ps = ::fma(ps, z, -1.0 / 39916800.0);        // - 1/11!
    ps = ::fma(ps, z, 1.0 / 362880.0);           // + 1/9!
    ps = ::fma(ps, z, -1.0 / 5040.0);            // - 1/7!
    ps = ::fma(ps, z, 1.0 / 120.0);              // + 1/5!
    ps = ::fma(ps, z, -1.0 / 6.0);               // - 1/3!
    const double sn = ::fma(t * z, ps, t);
    // cos t = 1 + sum_{j=1}^{8} (-1)^j z^j / (2j)!; the next term, t^18 / 18! <= 3e-18, is below the rounding
    double pc = 1.0 / 20922789888000.0;          // + 1/16!
    pc = ::fma(pc, z, -1.0 / 87178291200.0);     // - 1/14!
    pc = ::fma(pc, z, 1.0 / 479001600.0);        // + 1/12!
    pc = ::fma(pc, z, -1.0 / 3628800.0);         // - 1/10!
    pc = ::fma(pc, z, 1.0 / 40320.0);            // + 1/8!
    pc = ::fma(pc, z, -1.0 / 720.0);             // - 1/6!
    pc = ::fma(pc, z, 1.0 / 24.0);               // + 1/4!
    pc = ::fma(pc, z, -0.5);                     // - 1/2!
    const double cs = ::fma(z, pc, 1.0);
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
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = ::fma(p, r, 1.0 / 479001600.0);
    p = ::fma(p, r, 1.0 / 39916800.0);
    p = ::fma(p, r, 1.0 / 3628800.0);
    p = ::fma(p, r, 1.0 / 362880.0);
    p = ::fma(p, r, 1.0 / 40320.0);
    p = ::fma(p, r, 1.0 / 5040.0);
    p = ::fma(p, r, 1.0 / 720.0);
    p = ::fma(p, r, 1.0 / 120.0);
    p = ::fma(p, r, 1.0 / 24.0);
    p = ::fma(p, r, 1.0 / 6.0);
    p = ::fma(p, r, 0.5);
    p = ::fma(p, r, 1.0);
    p = ::fma(p, r, 1.0);
    return k < -1100.0 ? 0.0 : ::ldexp(p, (int)k);
}

// e^x - 1 for x <= 0: x = k ln 2 + r as in exp, e^r - 1 by its Taylor series to r^13
// (no cancellation: the series starts at r), then e^x - 1 = 2^k (e^r - 1) + (2^k - 1),
// whose second term is exact; k = 0 returns the series itself
HD double expm1_neg(double x)
{
    const double k = ::rint(x * 1.44269504088896340736);
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    const double r = ::fma(-k, ln2_lo, ::fma(-k, ln2_hi, x));  // |r| <= ln2 / 2
    double q = 1.0 / 6227020800.0;  // 1/13!
    q = ::fma(q, r, 1.0 / 479001600.0);
    q = ::fma(q, r, 1.0 / 39916800.0);
    q = ::fma(q, r, 1.0 / 3628800.0);
    q = ::fma(q, r, 1.0 / 362880.0);
    q = ::fma(q, r, 1.0 / 40320.0);
    q = ::fma(q, r, 1.0 / 5040.0);
    q = ::fma(q, r, 1.0 / 720.0);
    q = ::fma(q, r, 1.0 / 120.0);
    q = ::fma(q, r, 1.0 / 24.0);
    q = ::fma(q, r, 1.0 / 6.0);
    q = ::fma(q, r, 0.5);
    const double em = ::fma(r * r, q, r);
    const double p2 = k < -1100.0 ? 0.0 : ::ldexp(1.0, (int)k);  // 2^k
    return ::fma(p2, em, p2 - 1.0);
}

}  // namespace f64
}  // namespace hefk
