// Host build of the binary64 step functions (hefk_f64math.hpp): prints the largest
// error in units of the last place against the C library over argument sweeps, and the
// relative error of the binary32 e^x - 1 of the step.
#include <cmath>
#include <cstdio>
#include <random>

#include "hefk_device.hpp"

static double ulp_err(double got, double ref)
{
    if (got == ref) return 0.0;
    const double u = std::nextafter(std::fabs(ref), INFINITY) - std::fabs(ref);
    return std::fabs(got - ref) / u;
}

int main()
{
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    double e_log = 0, e_sin = 0, e_cos = 0, e_exp = 0, e_sqrt = 0, e_rcp = 0, e_expm1 = 0, e_expm1f = 0, e_dr = 0, e_di = 0;
    long same = 0, total = 0;
    for (int i = 0; i < 2000000; ++i) {
        const double u = (std::floor(U(rng) * 4294967296.0) + 0.5) * 0x1p-32;  // the uniforms of the step
        e_log = std::fmax(e_log, ulp_err(hefk::f64::log(u), std::log(u)));
        const double x = std::exp((U(rng) - 0.5) * 60.0);                     // 1e-13 .. 1e13
        e_log = std::fmax(e_log, ulp_err(hefk::f64::log(x), std::log(x)));
        double s, c;
        hefk::f64::sincos2pi(u, &s, &c);
        // reference: sin/cos of the exactly reduced argument in long double
        const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)u;
        e_sin = std::fmax(e_sin, std::fabs((long double)s - std::sin(ang)) / 0x1p-53);
        e_cos = std::fmax(e_cos, std::fabs((long double)c - std::cos(ang)) / 0x1p-53);
        const double xe = -U(rng) * 50.0;
        e_exp = std::fmax(e_exp, ulp_err(hefk::f64::exp(xe), std::exp(xe)));
        const double xs = x * x;
        e_sqrt = std::fmax(e_sqrt, ulp_err(hefk::f64::sqrt(xs), std::sqrt(xs)));
        e_rcp = std::fmax(e_rcp, ulp_err(hefk::f64::rcp(x), 1.0 / x));
        // distance and its reciprocal together, against the correctly rounded sqrt and 1/sqrt (long double)
        double dr, di;
        hefk::f64::dist_inv(xs, dr, di);
        e_dr = std::fmax(e_dr, ulp_err(dr, std::sqrt(xs)));
        e_di = std::fmax(e_di, ulp_err(di, (double)(1.0L / std::sqrt((long double)xs))));
        // e^x - 1 for x <= 0: uniform over [-40, 0] and log-uniform over [-1, -1e-12]
        const double xm = (i & 1) ? -U(rng) * 40.0 : -std::exp(-U(rng) * 27.6);
        e_expm1 = std::fmax(e_expm1, ulp_err(hefk::f64::expm1_neg(xm), std::expm1(xm)));
        // binary32 e^x - 1 of the triplet step (series near 0, exponential beyond): relative error
        const float xf = (float)xm;
        e_expm1f = std::fmax(e_expm1f, std::fabs((double)hefk::m::expm1_(xf) - std::expm1((double)xf)) /
                                           std::fabs(std::expm1((double)xf)));
        // the forms without zero / subnormal tests agree bitwise with the tested ones
        total += 3;
        same += hefk::f64::sqrt_pos(xs) == hefk::f64::sqrt(xs);
        same += hefk::f64::rcp_nz(x) == hefk::f64::rcp(x);
        same += hefk::f64::log_normal(u) == hefk::f64::log(u);
    }
    std::printf("log %.3f sin %.3f cos %.3f exp %.3f sqrt %.3f rcp %.3f expm1 %.3f same %.6f expm1f %.3g dist %.3f "
                "idist %.3f\n", e_log, e_sin, e_cos, e_exp, e_sqrt, e_rcp, e_expm1, (double)same / (double)total, e_expm1f,
                e_dr, e_di);
    std::printf("special %g %g %g %g %g %g\n", hefk::f64::log(0.0), hefk::f64::sqrt(0.0), hefk::f64::rcp(0.0),
                hefk::f64::exp(-800.0), hefk::f64::expm1_neg(0.0), hefk::f64::expm1_neg(-800.0));
    return 0;
}
