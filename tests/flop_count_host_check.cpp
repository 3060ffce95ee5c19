// Host build of the kernels' per-walker code on a counting binary32 type: the binary32
// floating-point operations of one walker step (noise, Euler step, trial evaluation,
// limiter, node test), counted from the source as written.  An operation counts only
// when an operand varies per walker (a position, a noise draw, or a value computed from
// them); products of trial parameters are uniform over the launch and do not count.
// Convention: add, sub, mul, div 1; fused multiply-add 2; each hardware transcendental
// (sqrt, rsq, rcp, exp2, log2, sin, cos) 1; negation, absolute value, copysign,
// compares, selects and conversions 0.  Binary64 work (ln w) is not binary32 work.
//
// stdin: trial sym noise(0 Gauss c1, 1 Gauss c2, 2 +-1) ee drift_limit(0/1) c (the Jastrow
//        coefficient theta2, which decides whether the cusp term (ee - 2c)/r12 is evaluated)
// stdout: flops transcendentals (one step at a point with r1 < r2, away from the node)
#include <cstdint>
#include <cstdio>

namespace flopcount {
long flops = 0, trans = 0;
}

struct CF {
    float v = 0.0f;
    bool var = false;
    CF() = default;
    CF(int x) : v((float)x) {}
    CF(float x) : v(x) {}
    CF(double x) : v((float)x) {}
    CF(uint32_t x) : v((float)x), var(true) {}  // random bits of the walker's stream
    static CF varying(float x)
    {
        CF c(x);
        c.var = true;
        return c;
    }
    explicit operator double() const { return v; }
};

inline CF op1(float v, bool var, int n)
{
    if (var) flopcount::flops += n;
    CF c(v);
    c.var = var;
    return c;
}
inline CF operator+(CF a, CF b) { return op1(a.v + b.v, a.var || b.var, 1); }
inline CF operator-(CF a, CF b) { return op1(a.v - b.v, a.var || b.var, 1); }
inline CF operator*(CF a, CF b) { return op1(a.v * b.v, a.var || b.var, 1); }
inline CF operator/(CF a, CF b) { return op1(a.v / b.v, a.var || b.var, 1); }
inline CF operator-(CF a) { return op1(-a.v, a.var, 0); }
inline CF& operator+=(CF& a, CF b) { return a = a + b; }
inline CF& operator-=(CF& a, CF b) { return a = a - b; }
inline CF& operator*=(CF& a, CF b) { return a = a * b; }
inline bool operator<(CF a, CF b) { return a.v < b.v; }
inline bool operator>(CF a, CF b) { return a.v > b.v; }
inline bool operator<=(CF a, CF b) { return a.v <= b.v; }
inline bool operator>=(CF a, CF b) { return a.v >= b.v; }
inline bool operator==(CF a, CF b) { return a.v == b.v; }
inline bool operator!=(CF a, CF b) { return a.v != b.v; }

inline CF transcendental(float v, bool var)
{
    if (var) {
        flopcount::flops += 1;
        flopcount::trans += 1;
    }
    CF c(v);
    c.var = var;
    return c;
}

#include <cmath>

// The binary32 elementary functions of the step, as the device builds them (hefk_device.hpp,
// namespace m): the same sequence of binary32 operations, each counted.
namespace hefk {
namespace m {
inline CF fma_(CF a, CF b, CF c) { return op1(std::fma(a.v, b.v, c.v), a.var || b.var || c.var, 2); }
inline CF negabs_(CF a) { return op1(-std::fabs(a.v), a.var, 0); }
inline CF copysign_(CF a, CF b) { return op1(std::copysign(a.v, b.v), a.var || b.var, 0); }
inline CF sqrt_(CF x) { return transcendental(std::sqrt(x.v), x.var); }                  // v_sqrt_f32
inline CF rcp_(CF x) { return transcendental(1.0f / x.v, x.var); }                        // v_rcp_f32
inline CF exp_(CF x) { return transcendental(std::exp2((x * CF(1.4426950408889634f)).v), x.var); }  // mul, v_exp_f32
inline CF expm1_(CF x)  // the series to x^7 beside the hardware exponential minus one, and a select
{
    CF q = CF((float)(1.0 / 5040.0));
    q = fma_(q, x, CF((float)(1.0 / 720.0)));
    q = fma_(q, x, CF((float)(1.0 / 120.0)));
    q = fma_(q, x, CF((float)(1.0 / 24.0)));
    q = fma_(q, x, CF((float)(1.0 / 6.0)));
    q = fma_(q, x, CF(0.5f));
    const CF series = fma_(x * x, q, x);
    const CF e = exp_(x) - CF(1.0f);
    return x.v > -0.35f ? series : e;
}
inline CF neg2log_(CF x) { return transcendental(std::log2(x.v), x.var) * CF(-1.3862943611198906f); }
inline CF logb_(CF x) { return transcendental(std::log2(x.v), x.var); }  // v_log_f32
inline void sincos2pi(CF u, CF* s, CF* c)                                  // v_sin_f32, v_cos_f32
{
    *s = transcendental(std::sin(6.2831853071795865f * u.v), u.var);
    *c = transcendental(std::cos(6.2831853071795865f * u.v), u.var);
}
inline void dist_inv(CF q, CF& r, CF& i)  // v_rsq_f32, then r = q (1/r)
{
    i = transcendental(1.0f / std::sqrt(q.v), q.var);
    r = q * i;
}
}  // namespace m
// contract-1 uniform of binary32: the float 1.m from the top 23 bits (a funnel shift), minus (1 - 2^-24)
inline CF unit32(uint32_t w, CF)
{
    const uint32_t bits = 0x3F800000u | (w >> 9);
    float f;
    __builtin_memcpy(&f, &bits, 4);
    return CF::varying(f) - CF(0.99999994039535522461f);
}
}  // namespace hefk

#include "hefk_device.hpp"

using namespace hefk;

template <int TRIAL, int NOISE>
void count(int sym, int ee, double limit, double c)
{
    TrialParams<CF> tp;
    const double th[6][5] = {{27.0 / 16, 0, 0, 0, 0}, {2.0, 0.25, 0.5, 0, 0}, {2.0, 0.3, 0.25, 0.6, 0},
                             {2.0, 0.3, 0.5, 0.5, 0}, {2.002777, 0, 0, 0.636748, 0.73351723}, {2.0, 0, 0, 0.25, 0}};
    tp.A = CF(th[TRIAL][0]);
    tp.beta = CF(th[TRIAL][1]);
    tp.c = CF(c);
    tp.a = CF(th[TRIAL][3]);
    tp.r0 = CF(th[TRIAL][4]);
    tp.Z = CF(2.0);
    tp.ee = CF((double)ee);
    tp.sym = CF((double)sym);
    const double dt = 0.0005;
    const StepConst sc = make_step_const(dt, -2.1, false, limit, false, false);
    StepScale<CF> ss;
    ss.dt = CF(dt);
    ss.sqdt = CF(std::sqrt(dt));
    ss.rad = CF(-2.0 * 0.69314718055994531 * dt);
    ss.lim2 = CF(2.0 * limit * dt);
    WalkerState<CF> w;
    const float y0[6] = {0.31f, -0.52f, 0.47f, -0.83f, 0.26f, -0.61f};
    for (int k = 0; k < 6; ++k) w.y[k] = CF::varying(y0[k]);
    w.lnw = 0.0;
    walker_reset<CF, TRIAL, false>(tp, sc, ss, w);
    Stream st;
    st.k0 = 7u;
    st.k1 = 0u;
    st.g0 = 12345u;
    st.g1 = 0u;
    NoiseGen<CF, NOISE> noise;
    Increment<CF> inc;
    noise.draw(st, 3u, ss, inc);  // a +-1 walk fetches its block here; the next step below reuses it
    walker_step<CF, TRIAL, false>(tp, sc, ss, inc, w);
    flopcount::flops = flopcount::trans = 0;
    noise.draw(st, 4u, ss, inc);
    walker_step<CF, TRIAL, false>(tp, sc, ss, inc, w);
    std::printf("%ld %ld\n", flopcount::flops, flopcount::trans);
}

template <int TRIAL>
void by_noise(int noise, int sym, int ee, double limit, double c)
{
    if (noise == 0) count<TRIAL, NOISE_G1>(sym, ee, limit, c);
    else if (noise == 1) count<TRIAL, NOISE_G2>(sym, ee, limit, c);
    else count<TRIAL, NOISE_PM1>(sym, ee, limit, c);
}

int main()
{
    int trial, sym, noise, ee, lim;
    double c;
    if (std::scanf("%d %d %d %d %d %lf", &trial, &sym, &noise, &ee, &lim, &c) != 6) return 2;
    const double limit = lim ? 1.0 : 0.0;
    switch (trial) {
        case TRIAL_EXPO: by_noise<TRIAL_EXPO>(noise, sym, ee, limit, c); break;
        case TRIAL_PADE: by_noise<TRIAL_PADE>(noise, sym, ee, limit, c); break;
        case TRIAL_TRIPLET: by_noise<TRIAL_TRIPLET>(noise, sym, ee, limit, c); break;
        case TRIAL_PZ: by_noise<TRIAL_PZ>(noise, sym, ee, limit, c); break;
        case TRIAL_TRIPLET_R0: by_noise<TRIAL_TRIPLET_R0>(noise, sym, ee, limit, c); break;
        default: by_noise<TRIAL_PZ_SUM>(noise, sym, ee, limit, c); break;
    }
    return 0;
}
