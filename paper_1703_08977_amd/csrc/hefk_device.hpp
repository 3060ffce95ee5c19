// hefk_device.hpp -- per-walker arithmetic of the generalized Feynman-Kac
// propagation: Philox4x32-10 stream, noise maps, trial functions (ln|psi|,
// sign, drift, local energy), one walker step.  Host+device code: the HIP
// kernels run it on gfx950, and a host build of the same code serves the
// CPU checks of the kernels' arithmetic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#define HD __host__ __device__ __forceinline__

#include "hefk_f64math.hpp"

namespace hefk {

enum : int { TRIAL_EXPO = 0, TRIAL_PADE = 1, TRIAL_TRIPLET = 2, TRIAL_PZ = 3, TRIAL_TRIPLET_R0 = 4, TRIAL_PZ_SUM = 5 };
// noise kinds of the kernels: Gaussian under contract 1, Gaussian under contract 2, +-1 walk
enum : int { NOISE_G1 = 0, NOISE_G2 = 1, NOISE_PM1 = 2 };
enum : uint32_t { PHASE_INIT = 0, PHASE_METROPOLIS = 1, PHASE_GAUSS = 2, PHASE_PM1 = 3 };

template <int TRIAL>
struct has_node {
    static constexpr bool value =
        (TRIAL == TRIAL_TRIPLET || TRIAL == TRIAL_PZ || TRIAL == TRIAL_TRIPLET_R0 || TRIAL == TRIAL_PZ_SUM);
};

// ---------------------------------------------------------------------------
// Elementary functions.  binary64: the lean functions of hefk_f64math.hpp
// (a few ulp over the step's arguments).  binary32: the hardware approximations
// (v_sqrt_f32, v_rsq_f32, v_rcp_f32, v_exp_f32, v_log_f32 and v_sin_f32 /
// v_cos_f32, which take their argument in revolutions), and a short series for
// e^x - 1 near zero.
// ---------------------------------------------------------------------------
namespace m {

HD double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
// -|a|: binary32 as a negated absolute value (operand modifiers of the consumer),
// binary64 as a select, which schedules better in the binary64 step
HD double negabs_(double a) { return a <= 0.0 ? a : -a; }
HD float negabs_(float a) { return -__builtin_fabsf(a); }
HD double copysign_(double a, double b) { return __builtin_copysign(a, b); }
HD float copysign_(float a, float b) { return __builtin_copysignf(a, b); }
HD float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// The step's binary64 square roots and reciprocals take arguments that are not zero
// (distances, 1 + ..., the node factor off the node, the Box-Muller radicand), and its
// logarithms uniforms of the noise: the forms without the zero and subnormal tests.
HD double sqrt_(double x) { return f64::sqrt_pos(x); }
HD double rcp_(double x) { return f64::rcp_nz(x); }
HD double exp_(double x) { return f64::exp(x); }
HD double expm1_(double x) { return f64::expm1_neg(x); }  // x <= 0
HD double neg2log_(double x) { return f64::neg2log(x); }
// the logarithm whose base the Box-Muller radius scale assumes: natural in binary64
HD double logb_(double x) { return f64::log_normal(x); }
// r = sqrt(q) and 1/r of a squared distance q > 0
HD void dist_inv(double q, double& r, double& i) { f64::dist_inv(q, r, i); }
// sin(2 pi u), cos(2 pi u) for u in (0, 1)
HD void sincos2pi(double u, double* s, double* c) { f64::sincos2pi(u, s, c); }

HD float sqrt_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return ::sqrtf(x);
#endif
}
HD float rcp_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
HD float exp_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
#else
    return ::expf(x);
#endif
}
// e^x - 1 for x <= 0 (the node factor of the triplet): for x > -0.35 the Taylor
// series to x^7 (truncation below 2e-8 relative), else e^x - 1 from the hardware
// exponential, which has no cancellation there (e^x < 0.71)
HD float expm1_(float x)
{
    float q = (float)(1.0 / 5040.0);
    q = m::fma_(q, x, (float)(1.0 / 720.0));
    q = m::fma_(q, x, (float)(1.0 / 120.0));
    q = m::fma_(q, x, (float)(1.0 / 24.0));
    q = m::fma_(q, x, (float)(1.0 / 6.0));
    q = m::fma_(q, x, 0.5f);
    const float series = m::fma_(x * x, q, x);
#if defined(__HIP_DEVICE_COMPILE__)
    const float e = __builtin_amdgcn_exp2f(x * 1.4426950408889634f);
#else
    const float e = ::exp2f(x * 1.4426950408889634f);
#endif
    return x > -0.35f ? series : e - 1.0f;
}
// -2 ln x = (-2 ln 2) log2 x: one v_log_f32 and one multiply
HD float neg2log_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_logf(x) * -1.3862943611198906f;
#else
    return -2.0f * ::logf(x);
#endif
}
// base-2 logarithm in binary32: one v_log_f32
HD float logb_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_logf(x);
#else
    return ::log2f(x);
#endif
}
HD void sincos2pi(float u, float* s, float* c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
#else
    *s = ::sinf(6.2831853071795865f * u);
    *c = ::cosf(6.2831853071795865f * u);
#endif
}
// 1/r = 1/sqrt(q) by one v_rsq_f32 and r = q / r, for a squared distance q > 0
HD void dist_inv(float q, float& r, float& i)
{
#if defined(__HIP_DEVICE_COMPILE__)
    i = __builtin_amdgcn_rsqf(q);
#else
    i = 1.0f / ::sqrtf(q);
#endif
    r = q * i;
}

}  // namespace m

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products with the round constants below, the key bumped by
// the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct Words {
    uint32_t w[4];
};

// three-input xor: one v_bitop3_b32 (truth table 0x96) on gfx950
HD uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
    return a ^ b ^ c;
#endif
}

HD Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words o;
    o.w[0] = c0;
    o.w[1] = c1;
    o.w[2] = c2;
    o.w[3] = c3;
    return o;
}

struct Stream {
    uint32_t k0, k1;  // key: the seed
    uint32_t g0, g1;  // counter words 2, 3: the global walker id
    HD Words block(uint32_t phase, uint32_t b) const { return philox(b, phase, g0, g1, k0, k1); }
    // The same stream with a key the compiler must take as unknown at each call
    // (device): the round keys are then bumped on the scalar unit per block instead of
    // being hoisted out of the step loop, where the binary64 step has no scalar
    // registers left to hold all twenty of them.
    HD Stream key_per_call() const
    {
        Stream s = *this;
#if defined(__HIP_DEVICE_COMPILE__)
        asm volatile("" : "+s"(s.k0), "+s"(s.k1));
#endif
        return s;
    }
};

// uniform (0,1) from a 32-bit word: binary64 (w + 1/2) 2^-32; binary32 from the top 23
// bits, ((w >> 9) + 1/2) 2^-23, built as the float 1.m with m = w >> 9 (one funnel shift
// of 0x7F:w by 9) minus (1 - 2^-24), exact in binary32
HD double unit32(uint32_t w, double) { return ((double)w + 0.5) * 0x1p-32; }
HD float unit32(uint32_t w, float)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const uint32_t bits = __builtin_amdgcn_alignbit(0x7Fu, w, 9u);
#else
    const uint32_t bits = 0x3F800000u | (w >> 9);
#endif
    float f;
    __builtin_memcpy(&f, &bits, 4);
    return f - 0.99999994039535522461f;  // 1 - 2^-24
}
// uniform (0,1) from a 21-bit field, exact in both precisions
template <typename R>
HD R unit21(uint32_t f)
{
    return m::fma_((R)f, (R)0x1p-21, (R)0x1p-22);  // (f + 1/2) 2^-21 with one rounding of an exact value
}

template <typename R>
HD void box_muller(R u1, R u2, R* a, R* b)
{
    const R rad = m::sqrt_(m::neg2log_(u1));
    R s, c;
    m::sincos2pi(u2, &s, &c);
    *a = rad * c;
    *b = rad * s;
}

// The six uniforms of Gaussian vector v of a phase.  Contract 1: blocks 2v, 2v+1,
// words 0..3 of the first and 0, 1 of the second, 32 bits each.
template <typename R>
HD void uniforms6_c1(const Stream& st, uint32_t phase, uint32_t v, R u[6])
{
    const Words a = st.block(phase, 2u * v);
    const Words b = st.block(phase, 2u * v + 1u);
    u[0] = unit32(a.w[0], R());
    u[1] = unit32(a.w[1], R());
    u[2] = unit32(a.w[2], R());
    u[3] = unit32(a.w[3], R());
    u[4] = unit32(b.w[0], R());
    u[5] = unit32(b.w[1], R());
}

// contract 2: one block, six 21-bit fields (the low 21 bits of each word, then the
// top 11 bits of words 0 and 1, and of words 2 and 3, joined)
template <typename R>
HD void uniforms6_c2(const Stream& st, uint32_t phase, uint32_t v, R u[6])
{
    const Words a = st.block(phase, v);
    const uint32_t m21 = 0x1FFFFFu;
    u[0] = unit21<R>(a.w[0] & m21);
    u[1] = unit21<R>(a.w[1] & m21);
    u[2] = unit21<R>(a.w[2] & m21);
    u[3] = unit21<R>(a.w[3] & m21);
    u[4] = unit21<R>((a.w[0] >> 21) | (((a.w[1] >> 21) & 0x3FFu) << 11));
    u[5] = unit21<R>((a.w[2] >> 21) | (((a.w[3] >> 21) & 0x3FFu) << 11));
}

// Gaussian 6-vector number v of a phase, contract 1: pairs (u0, u1), (u2, u3), (u4, u5)
template <typename R>
HD void gauss6_c1(const Stream& st, uint32_t phase, uint32_t v, R xi[6])
{
    R u[6];
    uniforms6_c1<R>(st, phase, v, u);
#pragma unroll
    for (int j = 0; j < 3; ++j) box_muller<R>(u[2 * j], u[2 * j + 1], &xi[2 * j], &xi[2 * j + 1]);
}

// Per-precision constants of the position update.
template <typename R>
struct StepScale {
    R dt;    // time step
    R sqdt;  // sqrt(dt): the increment of the +-1 walk
    R rad;   // Box-Muller radius with sqrt(dt) folded in: sqrt(dt) sqrt(-2 ln u) = sqrt(rad logb(u))
    R lim2;  // 2 a dt of the drift limiting (a = drift_limit; 0: none)
};
// binary32 takes the base-2 logarithm (v_log_f32), binary64 the natural one
HD StepScale<float> step_scale(double dt, double drift_limit, float)
{
    return StepScale<float>{(float)dt, (float)std::sqrt(dt), (float)(-2.0 * 0.69314718055994531 * dt),
                            (float)(2.0 * drift_limit * dt)};
}
HD StepScale<double> step_scale(double dt, double drift_limit, double)
{
    return StepScale<double>{dt, std::sqrt(dt), -2.0 * dt, 2.0 * drift_limit * dt};
}

// The increment sqrt(dt) xi of one step, as sqrt(dt) xi_k = r[k / 2] u[k]: for the
// Gaussian noise a Box-Muller radius (sqrt(dt) included) and cos / sin of the angle,
// for the +-1 walk sqrt(dt) and the signs.  Kept factored, the increment enters the
// position update as one fused multiply-add per coordinate.
template <typename R>
struct Increment {
    R r[3];
    R u[6];
};

template <typename R>
HD void increment_from_uniforms(const R u[6], R rad, Increment<R>& inc)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        inc.r[j] = m::sqrt_(m::logb_(u[2 * j]) * rad);
        m::sincos2pi(u[2 * j + 1], &inc.u[2 * j + 1], &inc.u[2 * j]);
    }
}

// +-1 walk: step k uses bits 6 (k mod 5) + j of word (k mod 20) / 5 of block k / 20
template <typename R>
HD void pm1_from_word(uint32_t word, uint32_t k, R xi[6])
{
    const uint32_t sh = 6u * (k % 5u);
#pragma unroll
    for (int j = 0; j < 6; ++j) xi[j] = ((word >> (sh + (uint32_t)j)) & 1u) ? (R)1 : (R)-1;
}

// The propagation increment of global step k for one walker.  The +-1 walk keeps
// the Philox block it is reading (one block serves 20 steps).
template <typename R, int NOISE>
struct NoiseGen {
    uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0, blk = 0xFFFFFFFFu;

    HD void draw(const Stream& st_in, uint32_t k, const StepScale<R>& ss, Increment<R>& inc)
    {
        const Stream st = (sizeof(R) == 8) ? st_in.key_per_call() : st_in;
        if (NOISE == NOISE_G1 || NOISE == NOISE_G2) {
            R u[6];
            if (NOISE == NOISE_G1)
                uniforms6_c1<R>(st, PHASE_GAUSS, k, u);
            else
                uniforms6_c2<R>(st, PHASE_GAUSS, k, u);
            increment_from_uniforms<R>(u, ss.rad, inc);
        } else {
            const uint32_t b = k / 20u;
            if (b != blk) {
                const Words ww = st.block(PHASE_PM1, b);
                w0 = ww.w[0];
                w1 = ww.w[1];
                w2 = ww.w[2];
                w3 = ww.w[3];
                blk = b;
            }
            const uint32_t wi = (k % 20u) / 5u;
            const uint32_t word = wi == 0 ? w0 : (wi == 1 ? w1 : (wi == 2 ? w2 : w3));
            pm1_from_word<R>(word, k, inc.u);
#pragma unroll
            for (int j = 0; j < 3; ++j) inc.r[j] = ss.sqdt;
        }
    }
};

// ---------------------------------------------------------------------------
// Trial functions.  psi = Phi exp(U), U = c r12 / (1 + beta r12).
// Parameters: A = theta0 (orbital exponent), beta = theta1, c = theta2,
// a = theta3 (second exponent, TRIPLET, PZ, TRIPLET_R0), r0 = theta4 (TRIPLET_R0).
// ---------------------------------------------------------------------------
template <typename R>
struct TrialParams {
    R A, beta, c, a, Z, ee, sym, r0;
};

// Pieces of the geometry every trial uses: the separation vector, the three
// distances and their inverses, and the projections R1 . D, R2 . D (the unit
// vectors are never formed: drifts are written as a R1 + b D with scalar a, b).
template <typename R>
struct Geo {
    R D[3];  // r1 - r2
    R r1, r2, r12, i1, i2, i12;
    R p1, p2;  // R1 . D, R2 . D
};

template <typename R>
HD void geometry(const R y[6], Geo<R>& g)
{
    g.D[0] = y[0] - y[3];
    g.D[1] = y[1] - y[4];
    g.D[2] = y[2] - y[5];
    m::dist_inv(y[0] * y[0] + y[1] * y[1] + y[2] * y[2], g.r1, g.i1);
    m::dist_inv(y[3] * y[3] + y[4] * y[4] + y[5] * y[5], g.r2, g.i2);
    m::dist_inv(g.D[0] * g.D[0] + g.D[1] * g.D[1] + g.D[2] * g.D[2], g.r12, g.i12);
    g.p1 = y[0] * g.D[0] + y[1] * g.D[1] + y[2] * g.D[2];
    g.p2 = y[3] * g.D[0] + y[4] * g.D[1] + y[5] * g.D[2];
}

// Jastrow pieces: u' = c / s^2 (s = 1 + beta r12) and the radial part of the local
// energy's Jastrow terms,
//   rest = -u'' - u'^2 + (ee - 2u')/r12 = [2 c beta (1/s + 2 + beta r12) - c^2 / s^2] / s^2 + (ee - 2c)/r12,
// with u'' = -2 c beta / s^3, and (ee - 2u')/r12 written without the cancellation at
// r12 -> 0 when ee = 2c (the cusp value), from 1 - 1/s^2 = beta r12 (2 + beta r12) / s^2.
template <typename R>
struct Jas {
    R up, rest;
};

template <typename R>
HD Jas<R> jastrow(const TrialParams<R>& p, const Geo<R>& g)
{
    Jas<R> j;
    const R is = m::rcp_((R)1 + p.beta * g.r12);
    const R is2 = is * is;
    j.up = p.c * is2;
    const R cusp = p.ee - (R)2 * p.c;
    j.rest = ((R)2 * p.c * p.beta * (is + (R)2 + p.beta * g.r12) - p.c * p.c * is2) * is2 +
             (cusp != (R)0 ? cusp * g.i12 : (R)0);
    return j;
}

// b1 = a1 R1 + w D, b2 = a2 R2 - w D
template <typename R>
HD void drift_from(const R y[6], const Geo<R>& g, R a1, R a2, R w, R b[6])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R wd = w * g.D[k];  // shared by both electrons
        b[k] = m::fma_(a1, y[k], wd);
        b[3 + k] = m::fma_(a2, y[3 + k], -wd);
    }
}

// Drift b = grad ln|psi|, local energy E_L = -(1/2) Lap(psi)/psi + V and the sign
// of psi (0 on the node).  V = -Z/r1 - Z/r2 + ee/r12.  With h_i = R_i / r_i and
// h12 = D / r12, the cosines are h1 . h12 = p1 / (r1 r12), h2 . h12 = p2 / (r2 r12).
//
// TRIPLET, TRIPLET_R0 and PZ combine f = e^{-A r1 - a r2} and g = e^{-A r2 - a r1};
// with d = (A - a)(r1 - r2), g / f = e^d.  They are evaluated as Phi / max(f, g):
// (t1, t2) = (1, e^d) for d <= 0 and (e^{-d}, 1) for d > 0, so no exponential can
// overflow and every ratio grad Phi / Phi, Lap Phi / Phi is unchanged.
//
// gphi2 (optional): |grad ln|Phi||^2 summed over both electrons, Phi the orbital
// part (the factor that carries the node), for the node-distance estimate.
template <typename R, int TRIAL>
HD R trial_eval(const TrialParams<R>& p, const R y[6], R b[6], R& el, R* gphi2 = nullptr)
{
    Geo<R> g;
    geometry(y, g);
    R node = (R)1;  // a value with the sign of psi (the orbital factor for the node trials)
    if (TRIAL == TRIAL_EXPO) {
        drift_from(y, g, -p.A * g.i1, -p.A * g.i2, (R)0, b);
        if (gphi2) *gphi2 = (R)2 * p.A * p.A;
        // -A^2 + (A - Z)(1/r1 + 1/r2) + ee/r12: exactly -Z^2 for A = Z, ee = 0
        el = -p.A * p.A + (p.A - p.Z) * (g.i1 + g.i2) + (p.ee != (R)0 ? p.ee * g.i12 : (R)0);
    } else if (TRIAL == TRIAL_PADE) {
        // grad_i Phi / Phi = -A h_i;  cross term: -A u' (h1 - h2) . h12
        const Jas<R> j = jastrow(p, g);
        drift_from(y, g, -p.A * g.i1, -p.A * g.i2, j.up * g.i12, b);
        if (gphi2) *gphi2 = (R)2 * p.A * p.A;
        const R w = (g.p1 * g.i1 - g.p2 * g.i2) * g.i12;  // (h1 - h2) . h12
        el = -p.A * p.A + (p.A - p.Z) * (g.i1 + g.i2) + p.A * j.up * w + j.rest;
    } else if (TRIAL == TRIAL_TRIPLET || TRIAL == TRIAL_TRIPLET_R0) {
        const Jas<R> j = jastrow(p, g);
        const R d = (p.A - p.a) * (g.r1 - g.r2);
        const bool lo = d <= (R)0;
        R g1, g2, lsum, D;  // lsum = Lap_1 Phi / Phi + Lap_2 Phi / Phi
        if (TRIAL == TRIAL_TRIPLET) {
            // Phi / max(f, g) = t1 - t2 = D:
            //   g1 = (-A t1 + a t2) / D, g2 = (-a t1 + A t2) / D,
            //   Lap_1 Phi / Phi = [t1 (A^2 - 2A/r1) - t2 (a^2 - 2a/r1)] / D (roles exchanged for Lap_2),
            //   summed: [t1 (A^2 + a^2 - 2A/r1 - 2a/r2) - t2 (A^2 + a^2 - 2a/r1 - 2A/r2)] / D
            const R em = m::expm1_(m::negabs_(d));  // e^{-|d|} - 1, accurate near the node
            const R e = (R)1 + em;
            const R t1 = lo ? (R)1 : e;
            const R t2 = lo ? e : (R)1;
            D = lo ? -em : em;  // t1 - t2 without cancellation
            const R iD = m::rcp_(D);
            g1 = (-p.A * t1 + p.a * t2) * iD;
            g2 = (-p.a * t1 + p.A * t2) * iD;
            const R q = p.A * p.A + p.a * p.a;
            lsum = (t1 * (q - (R)2 * p.A * g.i1 - (R)2 * p.a * g.i2) - t2 * (q - (R)2 * p.a * g.i1 - (R)2 * p.A * g.i2)) * iD;
        } else {
            // Phi / max(f, g) = (r0 - r1) t1 - (r0 - r2) t2 = D; with u(r) = (r0 - r) e^{-A r}:
            //   u'/e^{-A r} = -(1 + A (r0 - r)),  Lap u / e^{-A r} = A (2 + A (r0 - r)) - 2 (1 + A (r0 - r)) / r;
            //   the two Laplacian ratios summed by their t1 and t2 terms
            const R e = m::exp_(m::negabs_(d));  // e^{-|d|}
            const R t1 = lo ? (R)1 : e;
            const R t2 = lo ? e : (R)1;
            const R q1 = p.r0 - g.r1, q2 = p.r0 - g.r2;
            D = q1 * t1 - q2 * t2;
            const R iD = m::rcp_(D);
            const R u1 = (R)1 + p.A * q1, u2 = (R)1 + p.A * q2;
            g1 = (-u1 * t1 + p.a * q2 * t2) * iD;
            g2 = (-p.a * q1 * t1 + u2 * t2) * iD;
            lsum = (t1 * (p.A * ((R)2 + p.A * q1) - (R)2 * u1 * g.i1 + q1 * (p.a * p.a - (R)2 * p.a * g.i2)) -
                    t2 * (p.A * ((R)2 + p.A * q2) - (R)2 * u2 * g.i2 + q2 * (p.a * p.a - (R)2 * p.a * g.i1))) * iD;
        }
        // grad_i Phi / Phi = g_i h_i
        drift_from(y, g, g1 * g.i1, g2 * g.i2, j.up * g.i12, b);
        if (gphi2) *gphi2 = g1 * g1 + g2 * g2;
        const R cross = (g1 * g.p1 * g.i1 - g2 * g.p2 * g.i2) * g.i12;  // g1 h1.h12 - g2 h2.h12
        el = (R)-0.5 * lsum - j.up * cross + j.rest - p.Z * (g.i1 + g.i2);
        node = D;
    } else if (TRIAL == TRIAL_PZ_SUM) {
        // Phi = (z1 + z2)(f + g) (trial function 7): with Zs = z1 + z2 and S = f + g,
        // grad_i Phi / Phi = zhat / Zs + gs_i h_i, gs_1 = -(A t1 + a t2) / (t1 + t2),
        // gs_2 = -(a t1 + A t2) / (t1 + t2); Lap_i Phi / Phi = Lap_i S / S + 2 gs_i z_i / (r_i Zs)
        const Jas<R> j = jastrow(p, g);
        const R d = (p.A - p.a) * (g.r1 - g.r2);
        const bool lo = d <= (R)0;
        const R e = m::exp_(m::negabs_(d));  // e^{-|d|}
        const R t1 = lo ? (R)1 : e;
        const R t2 = lo ? e : (R)1;
        const R iS = m::rcp_(t1 + t2);
        const R z1 = y[2], z2 = y[5];
        const R Zs = z1 + z2;
        const R iZ = m::rcp_(Zs);
        const R g1 = -(p.A * t1 + p.a * t2) * iS;
        const R g2 = -(p.a * t1 + p.A * t2) * iS;
        const R a1 = g1 * g.i1, a2 = g2 * g.i2;
        drift_from(y, g, a1, a2, j.up * g.i12, b);
        b[2] += iZ;
        b[5] += iZ;
        if (gphi2)
            *gphi2 = g1 * g1 + g2 * g2 + (R)2 * iZ * (a1 * z1 + a2 * z2 + iZ);
        // Lap_1 Phi / Phi + Lap_2 Phi / Phi, summed by the t1 and t2 terms
        const R q = p.A * p.A + p.a * p.a;
        const R lsum = (t1 * (q - (R)2 * p.A * g.i1 - (R)2 * p.a * g.i2) + t2 * (q - (R)2 * p.a * g.i1 - (R)2 * p.A * g.i2)) * iS +
                       (R)2 * iZ * (a1 * z1 + a2 * z2);
        // (grad_1 Phi / Phi - grad_2 Phi / Phi) . h12: the zhat / Zs terms cancel
        const R cr = (a1 * g.p1 - a2 * g.p2) * g.i12;
        el = (R)-0.5 * lsum - j.up * cr + j.rest - p.Z * (g.i1 + g.i2);
        node = Zs;
    } else {  // TRIAL_PZ: Phi / max(f, g) = P = z2 t1 + sym z1 t2
        const Jas<R> j = jastrow(p, g);
        const R d = (p.A - p.a) * (g.r1 - g.r2);
        const bool lo = d <= (R)0;
        const R e = m::exp_(m::negabs_(d));  // e^{-|d|}
        const R t1 = lo ? (R)1 : e;
        const R t2 = (lo ? e : (R)1) * p.sym;
        const R z1 = y[2], z2 = y[5];
        const R P = z2 * t1 + t2 * z1;
        const R iP = m::rcp_(P);
        const R k1 = p.A * z2 * t1 + t2 * p.a * z1;  // grad_1 Phi / max = -k1 h1 + t2 zhat
        const R k2 = p.a * z2 * t1 + t2 * p.A * z1;  // grad_2 Phi / max = t1 zhat - k2 h2
        const R a1 = -k1 * g.i1 * iP, a2 = -k2 * g.i2 * iP;
        const R s1 = t2 * iP, s2 = t1 * iP;
        drift_from(y, g, a1, a2, j.up * g.i12, b);
        b[2] += s1;
        b[5] += s2;
        // |a1 R1 + s1 zhat|^2 + |a2 R2 + s2 zhat|^2
        if (gphi2)
            *gphi2 = a1 * a1 * g.r1 * g.r1 + (R)2 * a1 * s1 * z1 + s1 * s1 + a2 * a2 * g.r2 * g.r2 +
                     (R)2 * a2 * s2 * z2 + s2 * s2;
        // Lap_1 Phi / Phi + Lap_2 Phi / Phi, both electrons' terms of each product combined:
        // [z2 t1 (A^2 + a^2 - 2A/r1 - 4a/r2) + t2 z1 (A^2 + a^2 - 4a/r1 - 2A/r2)] / P
        const R q = p.A * p.A + p.a * p.a;
        const R lsum = (z2 * t1 * (q - (R)2 * p.A * g.i1 - (R)4 * p.a * g.i2) +
                        t2 * z1 * (q - (R)4 * p.a * g.i1 - (R)2 * p.A * g.i2)) * iP;
        // (grad_1 Phi / Phi - grad_2 Phi / Phi) . h12
        const R cr = (a1 * g.p1 - a2 * g.p2 + (s1 - s2) * g.D[2]) * g.i12;
        el = (R)-0.5 * lsum - j.up * cr + j.rest - p.Z * (g.i1 + g.i2);
        node = P;
    }
    return node;
}

// V = -Z/r1 - Z/r2 + ee/r12 (the integrand of the plain walk)
template <typename R>
HD R potential(const TrialParams<R>& p, const R y[6])
{
    Geo<R> g;
    geometry(y, g);
    return -p.Z * (g.i1 + g.i2) + (p.ee != (R)0 ? p.ee * g.i12 : (R)0);
}

// ln|psi| (binary64; -inf on the node), for the Metropolis start.
template <int TRIAL>
HD double trial_lnpsi(const TrialParams<double>& p, const double y[6])
{
    const double r1 = f64::sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    const double r2 = f64::sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
    const double d0 = y[0] - y[3], d1 = y[1] - y[4], d2 = y[2] - y[5];
    const double r12 = f64::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double U = (TRIAL == TRIAL_EXPO || p.c == 0.0) ? 0.0 : p.c * r12 * f64::rcp_nz(1.0 + p.beta * r12);
    if (TRIAL == TRIAL_EXPO || TRIAL == TRIAL_PADE) return -p.A * (r1 + r2) + U;
    // ln max(f, g) + ln|Phi / max(f, g)|
    const double d = (p.A - p.a) * (r1 - r2);
    const bool lo = d <= 0.0;
    const double lnmax = lo ? (-p.A * r1 - p.a * r2) : (-p.A * r2 - p.a * r1);
    if (TRIAL == TRIAL_TRIPLET) {
        const double em = ::expm1(lo ? d : -d);
        return lnmax + f64::log(::fabs(em)) + U;
    }
    if (TRIAL == TRIAL_TRIPLET_R0) {
        const double e = f64::exp(lo ? d : -d);
        const double D = (p.r0 - r1) * (lo ? 1.0 : e) - (p.r0 - r2) * (lo ? e : 1.0);
        return lnmax + f64::log(::fabs(D)) + U;
    }
    const double e = f64::exp(lo ? d : -d);
    if (TRIAL == TRIAL_PZ_SUM) return lnmax + f64::log(::fabs(y[2] + y[5]) * (1.0 + e)) + U;
    const double P = y[5] * (lo ? 1.0 : e) + p.sym * y[2] * (lo ? e : 1.0);
    return lnmax + f64::log(::fabs(P)) + U;
}

// Start position of one walker (binary64): Y = init_sigma xi(phase 0, vector 0),
// then n_met Metropolis steps on |psi|^2 with a uniform box proposal of standard
// deviation sigma_m: Philox block m of phase 1 gives six 16-bit displacement fields
// (halves of words 0..2) and the accept word 3.
template <int TRIAL>
HD void init_walker(const TrialParams<double>& tp, const Stream& st, int n_met, double init_sigma,
                    double sigma_m, double y[6])
{
    double xi[6];
    gauss6_c1<double>(st, PHASE_INIT, 0u, xi);
#pragma unroll
    for (int k = 0; k < 6; ++k) y[k] = init_sigma * xi[k];
    double lp = trial_lnpsi<TRIAL>(tp, y);
    const double h = 1.7320508075688772 * sigma_m;  // sqrt(3) sigma: the box of standard deviation sigma
    // displacement h (2 v - 1), v = (f + 1/2) 2^-16, as (h 2^-16) (2 f - 65535): an exact
    // integer times an exact power-of-two multiple of h
    const double hs = h * 0x1p-16;
    for (int mstep = 0; mstep < n_met; ++mstep) {
        const Words w = st.block(PHASE_METROPOLIS, (uint32_t)mstep);
        double yt[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const uint32_t f = (w.w[k / 2] >> (16 * (k % 2))) & 0xFFFFu;
            yt[k] = m::fma_(hs, (double)((int32_t)(2u * f) - 65535), y[k]);
        }
        const double u = unit32(w.w[3], 0.0);
        const double lpt = trial_lnpsi<TRIAL>(tp, yt);
        if (f64::log_normal(u) < 2.0 * (lpt - lp)) {  // u >= 2^-33
#pragma unroll
            for (int k = 0; k < 6; ++k) y[k] = yt[k];
            lp = lpt;
        }
    }
}

// ---------------------------------------------------------------------------
// One walker: state and one step of the discretised drifted diffusion.
// ---------------------------------------------------------------------------
template <typename R>
struct WalkerState {
    R y[6];
    R b[6];     // drift grad ln|psi| at y
    R bdt;      // its factor in the next position update: dt (times the limiting factor; 0 for the plain walk)
    R el;       // local energy at y
    double eb;  // integrand at y: E_L - e_ref (limited when drift_limit > 0), or V - e_ref (plain walk)
    R gn2;      // |grad ln|Phi||^2 at y (node-touch estimate)
    R sgn;  // sign of psi at y: +-1, or 0 on the node
    double lnw;
};

struct StepConst {
    double dt, e_ref;
    int quad_right;
    // quadrature of ln w over a step: ln w -= quad_c (quad_prev eb + en); (dt/2)(eb + en)
    // for the trapezoid, dt en for the right end-point
    double quad_c, quad_prev;
    double limit_adt;  // drift_limit * dt (0: no limiting)
    int plain;         // plain Feynman-Kac walk: no drift, integrand V - e_ref
    int bridge;        // weight each step by the chance that its path missed the node
    double two_over_dt;
    double lnw_absorbed;  // -inf, held here so that the step's test reads it from a scalar register
};

inline StepConst make_step_const(double dt, double e_ref, bool quad_right, double drift_limit, bool plain,
                                 bool bridge)
{
    StepConst sc;
    sc.dt = dt;
    sc.e_ref = e_ref;
    sc.quad_right = quad_right ? 1 : 0;
    sc.quad_c = quad_right ? dt : 0.5 * dt;
    sc.quad_prev = quad_right ? 0.0 : 1.0;
    sc.limit_adt = drift_limit * dt;
    sc.plain = plain ? 1 : 0;
    sc.bridge = bridge ? 1 : 0;
    sc.two_over_dt = 2.0 / dt;
    sc.lnw_absorbed = -INFINITY;
    return sc;
}

// Drift / integrand limiting near singular points: f = 2 / (1 + sqrt(1 + 2 a dt |b|^2)),
// b -> f b, E_L - e_ref -> f (E_L - e_ref).  The limited drift is carried as the step
// factor bdt = dt f of the unlimited one: the position update takes Y + bdt b.
template <typename R>
HD double limit_drift(const StepConst& sc, const StepScale<R>& ss, const R b[6], R el, R& bdt)
{
    double e = (double)el - sc.e_ref;
    bdt = ss.dt;
    if (sc.limit_adt > 0.0) {
        R v2 = 0;
#pragma unroll
        for (int k = 0; k < 6; ++k) v2 += b[k] * b[k];
        const R f = (R)2 * m::rcp_((R)1 + m::sqrt_((R)1 + ss.lim2 * v2));
        bdt = ss.dt * f;
        e *= (double)f;
    }
    return e;
}

// Integrand at y, and the drift step factor of the next step.  EXT kernels read the
// variant flags at run time; the others are the generalized walk only.
template <typename R, bool EXT>
HD double integrand(const TrialParams<R>& tp, const StepConst& sc, const StepScale<R>& ss, const R y[6], const R b[6], R el,
                    R& bdt)
{
    if (EXT && sc.plain) {
        bdt = (R)0;  // no drift
        return (double)potential<R>(tp, y) - sc.e_ref;
    }
    return limit_drift<R>(sc, ss, b, el, bdt);
}

// ln of the chance that a Brownian bridge over one step, between points at node
// distances d = 1/sqrt(ga) and d' = 1/sqrt(gb), does not touch a flat node:
// log(1 - exp(-2 d d' / dt)), in binary64.
HD double bridge_log_survival(const StepConst& sc, double ga, double gb)
{
    const double x = sc.two_over_dt * (1.0 / ::sqrt(ga * gb));
    return ::log(-::expm1(-x));
}

template <typename R, int TRIAL, bool EXT = false>
HD void walker_reset(const TrialParams<R>& tp, const StepConst& sc, const StepScale<R>& ss, WalkerState<R>& w)
{
    const R nd = trial_eval<R, TRIAL>(tp, w.y, w.b, w.el, EXT ? &w.gn2 : nullptr);
    w.sgn = (nd > (R)0) ? (R)1 : ((nd < (R)0) ? (R)-1 : (R)0);
    w.eb = integrand<R, EXT>(tp, sc, ss, w.y, w.b, w.el, w.bdt);
}

// Y' = Y + dt b + sqrt(dt) xi, ln w updated by the quadrature in binary64.  A step
// that crosses the node absorbs the walker: it keeps Y' (where it was found across the
// node) with ln w = -inf, and takes no further steps.
template <typename R, int TRIAL, bool EXT = false>
HD void walker_step(const TrialParams<R>& tp, const StepConst& sc, const StepScale<R>& ss, const Increment<R>& inc,
                    WalkerState<R>& w)
{
    if (w.lnw == sc.lnw_absorbed) return;  // absorbed
#pragma unroll
    for (int k = 0; k < 6; ++k) w.y[k] = m::fma_(inc.r[k >> 1], inc.u[k], m::fma_(w.bdt, w.b[k], w.y[k]));
    R gt = (R)0;
    const R nd = trial_eval<R, TRIAL>(tp, w.y, w.b, w.el, EXT ? &gt : nullptr);
    const double en = integrand<R, EXT>(tp, sc, ss, w.y, w.b, w.el, w.bdt);
    double lw = m::fma_(-sc.quad_c, m::fma_(sc.quad_prev, w.eb, en), w.lnw);
    if (EXT && has_node<TRIAL>::value && sc.bridge) lw += bridge_log_survival(sc, (double)w.gn2, (double)gt);
    lw = m::fma_(0.0, (double)w.el, lw);  // NaN when E_L is not finite
    // node crossing: psi(Y') is zero, NaN or of the other sign (or the walk started on the node)
    if (has_node<TRIAL>::value && !(nd * w.sgn > (R)0)) lw = -INFINITY;
    w.lnw = lw;
    w.eb = en;
    w.gn2 = gt;
    w.sgn = m::copysign_((R)1, nd);
}

}  // namespace hefk
