/*
 * he_fk_oracle.c -- plain, slow FP64 CPU oracle for the importance-sampled
 * (generalized) Feynman-Kac propagation of two-electron (He) walkers.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no source with the HIP path: its own
 * Philox, its own trial functions, its own propagation and reductions.
 *
 * What it follows (Datta, Rejcek, Fry, "The He atom revisited"):
 *   - imaginary-time Cauchy problem and its Feynman-Kac solution, eqs. (1)-(3);
 *   - the generalized (importance-sampled) decomposition H = H0 + V_P with
 *     V0 = lambda0 + (1/2) Lap(phi)/phi (the paper prints the Laplacian term
 *     without the 1/2; with it phi is an eigenfunction of H0 and phi^2 is the
 *     stationary law of the drifted process), so V_P = E_L - lambda0;
 *   - the energy formula eq. (4) and the drifted diffusion dY = grad(phi)/phi dt + dX
 *     that follows it;
 *   - the discretised walk: 3N scaled one-dimensional walks with +/-1 steps
 *     (section "Path Integral Theory"), here also with Gaussian increments
 *     (Euler-Maruyama); the Riemann sum of the potential along the path, here
 *     with the trapezoid rule (default) or the paper's right end-point sum;
 *   - space averaging: Z(t) = mean over N_rep independent replications of
 *     exp(-sum V_P dt), kept in the log domain;
 *   - absorption of walkers that cross the trial function's node (excited
 *     states with a known node, section "Path Integral Theory", last paragraph
 *     of the discretisation discussion);
 *   - optionally the plain Feynman-Kac walk of eqs. (2)-(3) (Brownian walkers,
 *     integrand V), the non-recurrent process the generalized walk replaces, and
 *     a Brownian-bridge estimate of node touches inside a step (reflection
 *     principle), which the paper leaves to an unstated "criterion".
 *
 * Random numbers: Philox4x32-10 from its published definition (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), replacing
 * the paper's serial "Superduper" congruential generator.  The counter of a
 * block is (block index within the phase, phase, low and high 32 bits of the
 * global walker id); the key is the 64-bit seed.
 *
 * parity pins: see tests/test_oracle_pins.py (Philox vs rocRAND, finite
 * differences of ln|psi|, closed-form systems, variational energy, LSE vs
 * exact summation, resume identity, complex-step gradient vs central
 * differences).
 */
#include <complex.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OFK_TRIAL_EXPO 0    /* exp(-alpha (r1 + r2))                                 */
#define OFK_TRIAL_PADE 1    /* exp(-alpha (r1 + r2)) exp(c r12 / (1 + beta r12))     */
#define OFK_TRIAL_TRIPLET 2 /* [exp(-A r1 - a r2) - exp(-A r2 - a r1)] * Jastrow     */
#define OFK_TRIAL_PZ 3      /* [z2 exp(-A r1 - a r2) + s z1 exp(-A r2 - a r1)] * Jastrow */
#define OFK_TRIAL_TRIPLET_R0 4 /* [(r0 - r1) exp(-A r1 - a r2) - (r0 - r2) exp(-A r2 - a r1)] * Jastrow */
#define OFK_TRIAL_PZ_SUM 5  /* (z1 + z2) [exp(-A r1 - a r2) + exp(-A r2 - a r1)] * Jastrow (trial function 7) */

#define OFK_NOISE_GAUSS 0
#define OFK_NOISE_PM1 1
#define OFK_QUAD_TRAPEZOID 0
#define OFK_QUAD_RIGHT 1

#define OFK_FLAG_PLAIN 1  /* plain Feynman-Kac: no drift, integrand V - e_ref (eqs. (2)-(3)) */
#define OFK_FLAG_BRIDGE 2 /* weight each step by the chance that no node was crossed inside it */

#define OFK_PHASE_INIT 0u
#define OFK_PHASE_METROPOLIS 1u
#define OFK_PHASE_GAUSS 2u
#define OFK_PHASE_PM1 3u

typedef struct {
    int32_t trial;
    int32_t sym;          /* +1 or -1, P_z trial only */
    int32_t ee;           /* 1: the potential holds +1/r12 */
    int32_t noise;        /* OFK_NOISE_* */
    int32_t quad;         /* OFK_QUAD_* */
    int32_t contract;     /* Gaussian stream contract: 1 or 2 */
    int32_t n_metropolis; /* Metropolis sweeps of the initial ensemble */
    int32_t flags;        /* OFK_FLAG_* */
    double Z;             /* nuclear charge */
    double theta[6];      /* [0] orbital exponent, [1] Jastrow beta, [2] Jastrow c, [3] second exponent a, [4] r0 */
    double dt;
    double e_ref;         /* the trial energy lambda0 used as the shift in eq. (4) */
    double metropolis_sigma;
    double init_sigma;
    double drift_limit;   /* a >= 0: drift / integrand limiting near singular points, 0 = off */
    uint64_t seed;
} ofk_params;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10                                                            */
/* ------------------------------------------------------------------------ */

void ofk_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void block_words(const ofk_params* p, uint32_t phase, uint32_t blk, uint64_t g, uint32_t w[4])
{
    uint32_t ctr[4] = {blk, phase, (uint32_t)g, (uint32_t)(g >> 32)};
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    ofk_philox4x32_10(ctr, key, w);
}

/* 32-bit word -> uniform in (0,1): (w + 1/2) 2^-32, exact in binary64. */
double ofk_u32_to_unit(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* 21-bit field -> uniform in (0,1): (f + 1/2) 2^-21, exact in binary32 and binary64. */
double ofk_u21_to_unit(uint32_t f) { return ((double)f + 0.5) * 0x1p-21; }

/* Box-Muller: two uniforms -> two independent standard normals. */
static void box_muller(double u1, double u2, double* a, double* b)
{
    const double two_pi = 6.283185307179586476925286766559;
    double R = sqrt(-2.0 * log(u1));
    double th = two_pi * u2;
    *a = R * cos(th);
    *b = R * sin(th);
}

/*
 * Contract 1: the Gaussian 6-vector number `blk` of a phase uses Philox blocks
 * 2 blk and 2 blk + 1.  Uniform pairs (w0,w1), (w2,w3) of the first block and
 * (w0,w1) of the second give xi0..xi5 (x1 y1 z1 x2 y2 z2).  Word 2 of the
 * second block is returned as a spare uniform (the Metropolis accept test).
 */
void ofk_gauss6_c1(const ofk_params* p, uint32_t phase, uint32_t blk, uint64_t g, double xi[6], double* spare)
{
    uint32_t a[4], b[4];
    block_words(p, phase, 2u * blk, g, a);
    block_words(p, phase, 2u * blk + 1u, g, b);
    box_muller(ofk_u32_to_unit(a[0]), ofk_u32_to_unit(a[1]), &xi[0], &xi[1]);
    box_muller(ofk_u32_to_unit(a[2]), ofk_u32_to_unit(a[3]), &xi[2], &xi[3]);
    box_muller(ofk_u32_to_unit(b[0]), ofk_u32_to_unit(b[1]), &xi[4], &xi[5]);
    if (spare) *spare = ofk_u32_to_unit(b[2]);
}

/*
 * Contract 2: one Philox block per Gaussian 6-vector.  Six 21-bit fields:
 * f_j = w_j & (2^21 - 1) for j = 0..3,
 * f_4 = (w0 >> 21) | ((w1 >> 21) & 0x3FF) << 11,
 * f_5 = (w2 >> 21) | ((w3 >> 21) & 0x3FF) << 11,
 * paired (f0,f1), (f2,f3), (f4,f5) through Box-Muller.
 */
void ofk_fields21(const uint32_t w[4], uint32_t f[6])
{
    const uint32_t m21 = 0x1FFFFFu;
    f[0] = w[0] & m21;
    f[1] = w[1] & m21;
    f[2] = w[2] & m21;
    f[3] = w[3] & m21;
    f[4] = (w[0] >> 21) | (((w[1] >> 21) & 0x3FFu) << 11);
    f[5] = (w[2] >> 21) | (((w[3] >> 21) & 0x3FFu) << 11);
}

void ofk_gauss6_c2(const ofk_params* p, uint32_t phase, uint32_t blk, uint64_t g, double xi[6])
{
    uint32_t w[4], f[6];
    block_words(p, phase, blk, g, w);
    ofk_fields21(w, f);
    box_muller(ofk_u21_to_unit(f[0]), ofk_u21_to_unit(f[1]), &xi[0], &xi[1]);
    box_muller(ofk_u21_to_unit(f[2]), ofk_u21_to_unit(f[3]), &xi[2], &xi[3]);
    box_muller(ofk_u21_to_unit(f[4]), ofk_u21_to_unit(f[5]), &xi[4], &xi[5]);
}

/*
 * +/-1 walk of the paper (eps = +1 or -1 with probability 1/2 each, one per
 * coordinate per step).  Step k reads block floor(k / 20) of phase 3, word
 * floor((k mod 20) / 5), bits 6 (k mod 5) + j for coordinate j.
 */
void ofk_pm1_6(const ofk_params* p, uint64_t k, uint64_t g, double eps[6])
{
    uint32_t w[4];
    block_words(p, OFK_PHASE_PM1, (uint32_t)(k / 20u), g, w);
    uint32_t word = w[(k % 20u) / 5u];
    uint32_t sh = 6u * (uint32_t)(k % 5u);
    for (int j = 0; j < 6; ++j) eps[j] = ((word >> (sh + (uint32_t)j)) & 1u) ? 1.0 : -1.0;
}

/* ------------------------------------------------------------------------ */
/* Trial functions: ln|psi|, sign(psi), drift grad ln psi, local energy.    */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lnpsi;
    int sign;
    double b[6];
    double el;
    double V;     /* the potential */
    double gphi2; /* |grad ln|Phi||^2 of the orbital part (both electrons) */
} ofk_eval;

static int trial_has_node(const ofk_params* p)
{
    return p->trial == OFK_TRIAL_TRIPLET || p->trial == OFK_TRIAL_PZ || p->trial == OFK_TRIAL_TRIPLET_R0 ||
           p->trial == OFK_TRIAL_PZ_SUM;
}

/*
 * psi = Phi(r1vec, r2vec) * exp(U(r12)), U = c r12 / (1 + beta r12).
 * grad_i ln psi = gPhi_i + grad_i U,
 * Lap_i psi / psi = lPhi_i + 2 gPhi_i . grad_i U + Lap_i U + |grad_i U|^2,
 * E_L = -(1/2) sum_i Lap_i psi / psi + V,  V = -Z/r1 - Z/r2 (+ 1/r12).
 * gPhi_i = grad_i Phi / Phi and lPhi_i = Lap_i Phi / Phi come from the orbital
 * part of each trial by the product rule; Lap of exp(-k r) is (k^2 - 2k/r) exp(-k r).
 */
void ofk_trial_eval(const ofk_params* p, const double y[6], ofk_eval* out)
{
    const double* R1 = y;
    const double* R2 = y + 3;
    double r1 = sqrt(R1[0] * R1[0] + R1[1] * R1[1] + R1[2] * R1[2]);
    double r2 = sqrt(R2[0] * R2[0] + R2[1] * R2[1] + R2[2] * R2[2]);
    double d12[3] = {R1[0] - R2[0], R1[1] - R2[1], R1[2] - R2[2]};
    double r12 = sqrt(d12[0] * d12[0] + d12[1] * d12[1] + d12[2] * d12[2]);
    double h1[3], h2[3], h12[3]; /* unit vectors */
    for (int k = 0; k < 3; ++k) {
        h1[k] = R1[k] / r1;
        h2[k] = R2[k] / r2;
        h12[k] = d12[k] / r12;
    }

    double gP1[3], gP2[3], lP1, lP2, lnPhi;
    int sign = 1;
    const double A = p->theta[0];
    const double a = p->theta[3];

    if (p->trial == OFK_TRIAL_EXPO || p->trial == OFK_TRIAL_PADE) {
        for (int k = 0; k < 3; ++k) {
            gP1[k] = -A * h1[k];
            gP2[k] = -A * h2[k];
        }
        lP1 = A * A - 2.0 * A / r1;
        lP2 = A * A - 2.0 * A / r2;
        lnPhi = -A * (r1 + r2);
    } else if (p->trial == OFK_TRIAL_TRIPLET) {
        /* Phi = f - g, f = exp(-A r1 - a r2), g = exp(-A r2 - a r1) = f q,
           q = exp(d), d = (A - a)(r1 - r2); Phi = f D with D = 1 - q = -expm1(d). */
        double d = (A - a) * (r1 - r2);
        double q = exp(d);
        double D = -expm1(d);
        double g1 = (-A + a * q) / D;
        double g2 = (-a + A * q) / D;
        for (int k = 0; k < 3; ++k) {
            gP1[k] = g1 * h1[k];
            gP2[k] = g2 * h2[k];
        }
        lP1 = ((A * A - 2.0 * A / r1) - q * (a * a - 2.0 * a / r1)) / D;
        lP2 = ((a * a - 2.0 * a / r2) - q * (A * A - 2.0 * A / r2)) / D;
        lnPhi = -A * r1 - a * r2 + log(fabs(D));
        sign = (D > 0.0) ? 1 : ((D < 0.0) ? -1 : 0);
    } else if (p->trial == OFK_TRIAL_TRIPLET_R0) {
        /* Phi = F(1,2) - F(2,1), F(1,2) = (r0 - r1) exp(-A r1 - a r2) (trial functions 3-5 of
           the paper).  For u(r) = (r0 - r) exp(-A r): u' = -(1 + A (r0 - r)) exp(-A r),
           Lap u = [A (2 + A (r0 - r)) - 2 (1 + A (r0 - r)) / r] exp(-A r).  Written per
           f = exp(-A r1 - a r2) with q = exp((A - a)(r1 - r2)) = g / f. */
        double r0 = p->theta[4];
        double q = exp((A - a) * (r1 - r2));
        double p1 = r0 - r1, p2 = r0 - r2;
        double D = p1 - p2 * q;
        double g1 = (-(1.0 + A * p1) + a * p2 * q) / D;
        double g2 = (-a * p1 + (1.0 + A * p2) * q) / D;
        for (int k = 0; k < 3; ++k) {
            gP1[k] = g1 * h1[k];
            gP2[k] = g2 * h2[k];
        }
        lP1 = ((A * (2.0 + A * p1) - 2.0 * (1.0 + A * p1) / r1) - p2 * q * (a * a - 2.0 * a / r1)) / D;
        lP2 = (p1 * (a * a - 2.0 * a / r2) - q * (A * (2.0 + A * p2) - 2.0 * (1.0 + A * p2) / r2)) / D;
        lnPhi = -A * r1 - a * r2 + log(fabs(D));
        sign = (D > 0.0) ? 1 : ((D < 0.0) ? -1 : 0);
    } else if (p->trial == OFK_TRIAL_PZ_SUM) {
        /* Phi = Zs S, Zs = z1 + z2 (a linear function: Lap Zs = 0, grad_i Zs = zhat), S = f + g,
           f = exp(-A r1 - a r2), g = exp(-A r2 - a r1) = f q, q = exp((A - a)(r1 - r2)).
           grad_i Phi / Phi = zhat / Zs + grad_i S / S,
           Lap_i Phi / Phi = Lap_i S / S + 2 zhat . grad_i S / (Zs S). */
        double Zs = R1[2] + R2[2];
        double q = exp((A - a) * (r1 - r2));
        double Sn = 1.0 + q; /* S / f */
        double gs1 = -(A + a * q) / Sn, gs2 = -(a + A * q) / Sn; /* grad_i S / S = gs_i h_i */
        for (int k = 0; k < 3; ++k) {
            double zh = (k == 2) ? 1.0 : 0.0;
            gP1[k] = zh / Zs + gs1 * h1[k];
            gP2[k] = zh / Zs + gs2 * h2[k];
        }
        double lS1 = ((A * A - 2.0 * A / r1) + q * (a * a - 2.0 * a / r1)) / Sn;
        double lS2 = ((a * a - 2.0 * a / r2) + q * (A * A - 2.0 * A / r2)) / Sn;
        lP1 = lS1 + 2.0 * gs1 * h1[2] / Zs;
        lP2 = lS2 + 2.0 * gs2 * h2[2] / Zs;
        lnPhi = log(fabs(Zs)) - A * r1 - a * r2 + log(Sn);
        sign = (Zs > 0.0) ? 1 : ((Zs < 0.0) ? -1 : 0);
    } else { /* OFK_TRIAL_PZ */
        /* Phi = z2 f + s z1 g, g = f rho, rho = exp((A - a)(r1 - r2)); Phi = f P,
           P = z2 + s z1 rho.  grad z1 = zhat for electron 1 (likewise z2).
           Lap_1 (z1 exp(-a r1)) = z1 (a^2 - 4a/r1) exp(-a r1). */
        double s = (double)p->sym;
        double z1 = R1[2], z2 = R2[2];
        double rho = exp((A - a) * (r1 - r2));
        double P = z2 + s * z1 * rho;
        double sr = s * rho;
        for (int k = 0; k < 3; ++k) {
            double zh = (k == 2) ? 1.0 : 0.0;
            gP1[k] = (-A * z2 * h1[k] + sr * (zh - a * z1 * h1[k])) / P;
            gP2[k] = ((zh - a * z2 * h2[k]) - sr * A * z1 * h2[k]) / P;
        }
        lP1 = (z2 * (A * A - 2.0 * A / r1) + sr * z1 * (a * a - 4.0 * a / r1)) / P;
        lP2 = (z2 * (a * a - 4.0 * a / r2) + sr * z1 * (A * A - 2.0 * A / r2)) / P;
        lnPhi = -A * r1 - a * r2 + log(fabs(P));
        sign = (P > 0.0) ? 1 : ((P < 0.0) ? -1 : 0);
    }

    /* Jastrow factor exp(c r12 / (1 + beta r12)); absent for the plain exponential. */
    double c = (p->trial == OFK_TRIAL_EXPO) ? 0.0 : p->theta[2];
    double beta = p->theta[1];
    double U = 0.0, up = 0.0, upp = 0.0;
    if (c != 0.0) {
        double s = 1.0 + beta * r12;
        U = c * r12 / s;
        up = c / (s * s);
        upp = -2.0 * c * beta / (s * s * s);
    }
    double gU1[3], gU2[3];
    for (int k = 0; k < 3; ++k) {
        gU1[k] = up * h12[k];
        gU2[k] = -up * h12[k];
    }
    double lapU = (c != 0.0) ? (upp + 2.0 * up / r12) : 0.0;

    double cross = 0.0;
    for (int k = 0; k < 3; ++k) cross += gP1[k] * gU1[k] + gP2[k] * gU2[k];
    double lap_total = lP1 + lP2 + 2.0 * cross + 2.0 * (lapU + up * up);
    double V = -p->Z / r1 - p->Z / r2 + (p->ee ? 1.0 / r12 : 0.0);

    out->lnpsi = lnPhi + U;
    out->sign = sign;
    for (int k = 0; k < 3; ++k) {
        out->b[k] = gP1[k] + gU1[k];
        out->b[3 + k] = gP2[k] + gU2[k];
    }
    out->el = -0.5 * lap_total + V;
    out->V = V;
    double g2 = 0.0;
    for (int k = 0; k < 3; ++k) g2 += gP1[k] * gP1[k] + gP2[k] * gP2[k];
    out->gphi2 = g2;
}

/* ln|psi| only (used by the Metropolis accept test); -inf on the node. */
static double trial_lnpsi(const ofk_params* p, const double y[6])
{
    ofk_eval e;
    ofk_trial_eval(p, y, &e);
    if (trial_has_node(p) && e.sign == 0) return -INFINITY;
    return e.lnpsi;
}

/* ------------------------------------------------------------------------ */
/* Initial ensemble: Y0 ~ |psi|^2 by Metropolis, per walker.                 */
/* ------------------------------------------------------------------------ */

/* Walker g: Y = init_sigma * xi(phase 0, vector 0) (Gaussian, contract 1); then
   n_metropolis steps with a uniform box proposal, symmetric about Y:
   block m of phase 1 gives six 16-bit fields f_j (low and high halves of words
   0, 1, 2) and the accept uniform u = (w3 + 1/2) 2^-32;
   Y'_j = Y_j + h (2 (f_j + 1/2) 2^-16 - 1), h = sqrt(3) metropolis_sigma (the
   box of standard deviation metropolis_sigma); accepted iff
   ln u < 2 (ln|psi(Y')| - ln|psi(Y)|). */
void ofk_init_walker(const ofk_params* p, uint64_t g, double y[6])
{
    double xi[6];
    ofk_gauss6_c1(p, OFK_PHASE_INIT, 0u, g, xi, NULL);
    for (int j = 0; j < 6; ++j) y[j] = p->init_sigma * xi[j];
    double lp = trial_lnpsi(p, y);
    const double h = sqrt(3.0) * p->metropolis_sigma;
    for (int m = 0; m < p->n_metropolis; ++m) {
        uint32_t w[4];
        block_words(p, OFK_PHASE_METROPOLIS, (uint32_t)m, g, w);
        double yt[6];
        for (int j = 0; j < 6; ++j) {
            uint32_t f = (w[j / 2] >> (16 * (j % 2))) & 0xFFFFu;
            double v = ((double)f + 0.5) * 0x1p-16;
            yt[j] = y[j] + h * (2.0 * v - 1.0);
        }
        double u = ofk_u32_to_unit(w[3]);
        double lpt = trial_lnpsi(p, yt);
        if (log(u) < 2.0 * (lpt - lp)) {
            memcpy(y, yt, sizeof(double) * 6);
            lp = lpt;
        }
    }
}

/* ids: walker ids (n of them); x_out [n][6], el_out [n]. */
void ofk_init(const ofk_params* p, const uint64_t* ids, int64_t n, double* x_out, double* el_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double* y = x_out + 6 * i;
        ofk_init_walker(p, ids[i], y);
        ofk_eval e;
        ofk_trial_eval(p, y, &e);
        el_out[i] = e.el;
    }
}

/* ------------------------------------------------------------------------ */
/* Propagation of one walker over global steps [step0, step0 + n_steps).    */
/* ------------------------------------------------------------------------ */

static void noise6(const ofk_params* p, uint64_t k, uint64_t g, double xi[6])
{
    if (p->noise == OFK_NOISE_PM1)
        ofk_pm1_6(p, k, g, xi);
    else if (p->contract == 2)
        ofk_gauss6_c2(p, OFK_PHASE_GAUSS, (uint32_t)k, g, xi);
    else
        ofk_gauss6_c1(p, OFK_PHASE_GAUSS, (uint32_t)k, g, xi, NULL);
}

/*
 * Limiting of the drift and of the integrand near the singular points of an
 * inexact trial function (Umrigar, Nightingale, Runge, J. Chem. Phys. 99, 2865
 * (1993)): with x = a dt |b|^2 the drift b becomes f b and E_L - e_ref becomes
 * f (E_L - e_ref), f = (sqrt(1 + 2x) - 1) / x, evaluated here in the equivalent
 * form 2 / (1 + sqrt(1 + 2x)), which has no cancellation for small x.  f = 1 when
 * the limiting is off (a = 0) and f -> 1 as dt -> 0.
 */
static double limit_factor(const ofk_params* p, const double b[6])
{
    if (!(p->drift_limit > 0.0)) return 1.0;
    double v2 = 0.0;
    for (int j = 0; j < 6; ++j) v2 += b[j] * b[j];
    double x = p->drift_limit * p->dt * v2;
    return 2.0 / (1.0 + sqrt(1.0 + 2.0 * x));
}

/*
 * Node-crossing correction (flag OFK_FLAG_BRIDGE).  Both end points of a step lie
 * on the same side of the node, but the continuous path between them may still
 * have touched it.  For a Brownian bridge of variance dt per coordinate between
 * points at distances d and d' from a flat boundary, the reflection principle
 * gives the probability of a touch as exp(-2 d d' / dt).  The distance to the
 * node is taken as d = |Phi| / |grad Phi| = 1 / |grad ln|Phi|| (Phi the orbital
 * part, which carries the node; first order in the distance).  The step's weight
 * is multiplied by the survival probability 1 - exp(-2 d d' / dt), i.e.
 *   lnw += log(-expm1(-2 / (dt |grad ln Phi(Y)| |grad ln Phi(Y')|))).
 * Exact for a driftless walk at a flat node; with the drift of the generalized
 * walk it is the same first-order estimate applied between the end points.
 */
static double bridge_log_survival(const ofk_params* p, double g2a, double g2b)
{
    double x = 2.0 / (p->dt * sqrt(g2a * g2b));
    return log(-expm1(-x));
}

/*
 * State: y[6] and lnw.  lnw = -inf marks a walker absorbed at the node; a NaN
 * marks a walker whose local energy went non-finite (kept NaN from then on).
 * Per step: Y' = Y + dt b(Y) + sqrt(dt) xi_k; if the trial has a node and
 * sign psi(Y') differs from sign psi(Y) (or psi(Y') = 0) the walker is
 * absorbed: it moves to Y' (with E_L(Y')) and stays there with lnw = -inf;
 * otherwise, with the integrand e(Y) = E_L(Y) - e_ref,
 *   trapezoid: lnw -= (dt/2) [e(Y) + e(Y')],
 *   right:     lnw -=  dt    e(Y').
 * Plain Feynman-Kac (flag OFK_FLAG_PLAIN, eqs. (2)-(3) with f = 1): b = 0 (Brownian
 * walkers) and e(Y) = V(Y) - e_ref; the start ensemble and the node test still
 * come from the trial function.  The drift limiting does not apply to it.
 * ell_s / el_s (may be NULL) receive lnw and E_L at steps step0 + s*sample_every.
 * node_dmin (may be NULL; a diagnostic, no part of the method) receives the smallest
 * node-distance estimate 1/|grad ln|Phi|| over the positions the walker held while
 * alive: the start and every accepted step (not the first position across the node).
 */
void ofk_propagate_walker(const ofk_params* p, uint64_t g, double y[6], double* lnw, double* el_io,
                          int64_t step0, int64_t n_steps, int64_t sample_every,
                          double* ell_s, double* el_s, double* node_dmin)
{
    const int plain = (p->flags & OFK_FLAG_PLAIN) != 0;
    const int bridge = (p->flags & OFK_FLAG_BRIDGE) != 0;
    ofk_eval cur;
    ofk_trial_eval(p, y, &cur);
    double f = plain ? 0.0 : limit_factor(p, cur.b); /* drift scale: 0 for Brownian walkers */
    double eb = plain ? cur.V - p->e_ref : f * (cur.el - p->e_ref); /* integrand at the current position */
    double w = *lnw;
    double sqdt = sqrt(p->dt);
    int node = trial_has_node(p);
    int64_t s = 0;
    double dmin = 1.0 / sqrt(cur.gphi2);
    if (ell_s) ell_s[s] = w;
    if (el_s) el_s[s] = cur.el;
    ++s;
    for (int64_t k = 0; k < n_steps; ++k) {
        int live = !(w == -INFINITY);
        if (live) {
            double xi[6], yt[6];
            noise6(p, (uint64_t)(step0 + k), g, xi);
            for (int j = 0; j < 6; ++j) yt[j] = y[j] + (plain ? 0.0 : p->dt * (f * cur.b[j])) + sqdt * xi[j];
            ofk_eval nxt;
            ofk_trial_eval(p, yt, &nxt);
            if (node && (nxt.sign != cur.sign || nxt.sign == 0)) {
                /* absorbed: weight zero from here on; the walker stays at the first
                   position found across the node (the paper gives it none) */
                w = -INFINITY;
                memcpy(y, yt, sizeof(double) * 6);
                cur = nxt;
            } else {
                double fn = plain ? 0.0 : limit_factor(p, nxt.b);
                double ebn = plain ? nxt.V - p->e_ref : fn * (nxt.el - p->e_ref);
                if (p->quad == OFK_QUAD_RIGHT)
                    w = w - p->dt * ebn;
                else
                    w = w - (0.5 * p->dt) * (eb + ebn);
                if (bridge && node) w += bridge_log_survival(p, cur.gphi2, nxt.gphi2);
                if (!isfinite(nxt.el)) w = NAN;
                memcpy(y, yt, sizeof(double) * 6);
                cur = nxt;
                f = fn;
                eb = ebn;
                if (1.0 / sqrt(cur.gphi2) < dmin) dmin = 1.0 / sqrt(cur.gphi2);
            }
        }
        if (sample_every > 0 && (k + 1) % sample_every == 0) {
            if (ell_s) ell_s[s] = w;
            if (el_s) el_s[s] = cur.el;
            ++s;
        }
    }
    *lnw = w;
    if (el_io) *el_io = cur.el;
    if (node_dmin) *node_dmin = dmin;
}

/* Many walkers: x [n][6], lnw [n], el [n]; ell / els [n][n_samples] or NULL;
   node_dmin [n] or NULL (the diagnostic of ofk_propagate_walker). */
void ofk_propagate(const ofk_params* p, const uint64_t* ids, int64_t n, double* x, double* lnw, double* el,
                   int64_t step0, int64_t n_steps, int64_t sample_every, double* ell, double* els,
                   double* node_dmin)
{
    int64_t ns = (sample_every > 0) ? n_steps / sample_every + 1 : 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        ofk_propagate_walker(p, ids[i], x + 6 * i, lnw + i, el + i, step0, n_steps, sample_every,
                             ell ? ell + ns * i : NULL, els ? els + ns * i : NULL,
                             node_dmin ? node_dmin + i : NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Space average (log domain): per sample, the tuple                         */
/* (m, S0, S1, S2, n_alive, n_nonfinite, n_total, 0) with                    */
/* m = max finite ln w, S0 = sum e^(l-m), S1 = sum e^(l-m) E_L,              */
/* S2 = sum e^(2(l-m)); sums in walker order with Neumaier compensation.     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double s, c;
} neumaier;

static void nm_add(neumaier* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

void ofk_tuples(const double* ell, const double* els, int64_t n, int64_t ns, double* out)
{
    for (int64_t j = 0; j < ns; ++j) {
        double m = -INFINITY;
        int64_t alive = 0, bad = 0;
        for (int64_t i = 0; i < n; ++i) {
            double l = ell[i * ns + j];
            if (isnan(l) || l == INFINITY) {
                ++bad;
            } else if (l != -INFINITY) {
                ++alive;
                if (l > m) m = l;
            }
        }
        neumaier s0 = {0, 0}, s1 = {0, 0}, s2 = {0, 0};
        if (alive > 0) {
            for (int64_t i = 0; i < n; ++i) {
                double l = ell[i * ns + j];
                if (!isfinite(l)) continue;
                double e = exp(l - m);
                nm_add(&s0, e);
                nm_add(&s1, e * els[i * ns + j]);
                nm_add(&s2, e * e);
            }
        }
        double* o = out + 8 * j;
        o[0] = m;
        o[1] = s0.s + s0.c;
        o[2] = s1.s + s1.c;
        o[3] = s2.s + s2.c;
        o[4] = (double)alive;
        o[5] = (double)bad;
        o[6] = (double)n;
        o[7] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Pathwise derivative of ln w along each path with respect to the trial    */
/* parameters (alpha, beta) of the Pade-Jastrow trial, at fixed Y0 and fixed */
/* noise, by the complex-step method: the whole path is propagated in       */
/* complex arithmetic with theta_a -> theta_a + i h, and d lnw / d theta_a = */
/* Im(lnw) / h.  No branch depends on the imaginary parts, so the result is  */
/* the exact derivative of the discrete map up to O(h^2) and rounding.       */
/* ------------------------------------------------------------------------ */

typedef double complex cplx;

static void pade_eval_c(const ofk_params* p, cplx alpha, cplx beta, const cplx y[6], cplx b[6], cplx* el)
{
    const cplx* R1 = y;
    const cplx* R2 = y + 3;
    cplx r1 = csqrt(R1[0] * R1[0] + R1[1] * R1[1] + R1[2] * R1[2]);
    cplx r2 = csqrt(R2[0] * R2[0] + R2[1] * R2[1] + R2[2] * R2[2]);
    cplx d12[3] = {R1[0] - R2[0], R1[1] - R2[1], R1[2] - R2[2]};
    cplx r12 = csqrt(d12[0] * d12[0] + d12[1] * d12[1] + d12[2] * d12[2]);
    cplx h1[3], h2[3], h12[3];
    for (int k = 0; k < 3; ++k) {
        h1[k] = R1[k] / r1;
        h2[k] = R2[k] / r2;
        h12[k] = d12[k] / r12;
    }
    cplx c = (p->trial == OFK_TRIAL_EXPO) ? 0.0 : p->theta[2];
    cplx s = 1.0 + beta * r12;
    cplx up = c / (s * s);
    cplx upp = -2.0 * c * beta / (s * s * s);
    cplx lP1 = alpha * alpha - 2.0 * alpha / r1;
    cplx lP2 = alpha * alpha - 2.0 * alpha / r2;
    cplx cross = 0.0;
    for (int k = 0; k < 3; ++k) {
        cplx gP1 = -alpha * h1[k], gP2 = -alpha * h2[k];
        cplx gU1 = up * h12[k], gU2 = -up * h12[k];
        cross += gP1 * gU1 + gP2 * gU2;
        b[k] = gP1 + gU1;
        b[3 + k] = gP2 + gU2;
    }
    cplx lapU = (p->trial == OFK_TRIAL_EXPO) ? 0.0 : (upp + 2.0 * up / r12);
    cplx lap_total = lP1 + lP2 + 2.0 * cross + 2.0 * (lapU + up * up);
    cplx V = -p->Z / r1 - p->Z / r2 + (p->ee ? 1.0 / r12 : 0.0);
    *el = -0.5 * lap_total + V;
}

static cplx limit_factor_c(const ofk_params* p, const cplx b[6])
{
    if (!(p->drift_limit > 0.0)) return 1.0;
    cplx v2 = 0.0;
    for (int j = 0; j < 6; ++j) v2 += b[j] * b[j];
    cplx x = p->drift_limit * p->dt * v2;
    return 2.0 / (1.0 + csqrt(1.0 + 2.0 * x));
}

/*
 * For walker g starting at y0 (fixed), propagate n_steps from step 0 with
 * parameter direction `dir` (0: alpha, 1: beta) perturbed by i h.  Writes
 * d lnw / d theta_dir at every sample time into dell [n_samples].
 * Only the nodeless trials (EXPO, PADE) are supported.
 */
int ofk_dlnw_dtheta_walker(const ofk_params* p, uint64_t g, const double y0[6], int64_t n_steps,
                           int64_t sample_every, int dir, double* dell)
{
    if (p->trial != OFK_TRIAL_EXPO && p->trial != OFK_TRIAL_PADE) return -1;
    const double h = 1e-30;
    cplx alpha = p->theta[0] + (dir == 0 ? I * h : 0.0);
    cplx beta = p->theta[1] + (dir == 1 ? I * h : 0.0);
    cplx y[6], b[6], el;
    for (int j = 0; j < 6; ++j) y[j] = y0[j];
    pade_eval_c(p, alpha, beta, y, b, &el);
    cplx f = limit_factor_c(p, b);
    cplx eb = f * (el - p->e_ref);
    cplx w = 0.0;
    double sqdt = sqrt(p->dt);
    int64_t s = 0;
    dell[s++] = 0.0;
    for (int64_t k = 0; k < n_steps; ++k) {
        double xi[6];
        noise6(p, (uint64_t)k, g, xi);
        cplx yt[6], bt[6], elt;
        for (int j = 0; j < 6; ++j) yt[j] = y[j] + p->dt * (f * b[j]) + sqdt * xi[j];
        pade_eval_c(p, alpha, beta, yt, bt, &elt);
        cplx fn = limit_factor_c(p, bt);
        cplx ebn = fn * (elt - p->e_ref);
        if (p->quad == OFK_QUAD_RIGHT)
            w = w - p->dt * ebn;
        else
            w = w - (0.5 * p->dt) * (eb + ebn);
        for (int j = 0; j < 6; ++j) {
            y[j] = yt[j];
            b[j] = bt[j];
        }
        el = elt;
        f = fn;
        eb = ebn;
        if (sample_every > 0 && (k + 1) % sample_every == 0) dell[s++] = cimag(w) / h;
    }
    return 0;
}

/* d ln|psi(y0)| / d theta_dir for the nodeless trials (score of the start law). */
double ofk_dlnpsi_dtheta(const ofk_params* p, const double y[6], int dir)
{
    double r1 = sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    double r2 = sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
    double dx = y[0] - y[3], dy = y[1] - y[4], dz = y[2] - y[5];
    double r12 = sqrt(dx * dx + dy * dy + dz * dz);
    if (dir == 0) return -(r1 + r2);
    if (p->trial == OFK_TRIAL_EXPO) return 0.0;
    double s = 1.0 + p->theta[1] * r12;
    return -p->theta[2] * r12 * r12 / (s * s);
}

void ofk_dlnw_dtheta(const ofk_params* p, const uint64_t* ids, int64_t n, const double* y0, int64_t n_steps,
                     int64_t sample_every, int dir, double* dell, int* status)
{
    int64_t ns = n_steps / sample_every + 1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < n; ++i)
        bad |= (ofk_dlnw_dtheta_walker(p, ids[i], y0 + 6 * i, n_steps, sample_every, dir, dell + ns * i) != 0);
    *status = bad ? -1 : 0;
}

/* Number of OpenMP threads the oracle runs with (reported by the benchmark). */
int ofk_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from here on (timing runs). */
void ofk_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* The propagation noise of step k for many walkers: out [n][6]. */
void ofk_noise_bulk(const ofk_params* p, uint64_t k, const uint64_t* ids, int64_t n, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) noise6(p, k, ids[i], out + 6 * i);
}
