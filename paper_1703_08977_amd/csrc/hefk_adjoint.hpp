// hefk_adjoint.hpp -- reverse-mode (adjoint) pathwise derivative of the log
// space average with respect to the trial parameters theta = (alpha, beta) of
// the nodeless trials exp(-alpha (r1 + r2)) [exp(c r12 / (1 + beta r12))].
//
// Forward map of one walker at fixed start Y_0 and fixed noise xi_k:
//   Y_{k+1} = Y_k + dt b(Y_k; theta) + sqrt(dt) xi_k,
//   ln w_k  = -(dt/2) sum_{j<k} (e_j + e_{j+1})   (trapezoid)  or  -dt sum_{1<=j<=k} e_j  (right),
//   e_j = E_L(Y_j; theta) - e_ref.
// Objective J = sum_s g_s L_s, L_s = ln((1/N) sum_i w_i(t_s)), so
// dJ/d lnw_{i,s} = g_s p_{i,s}, p_{i,s} = exp(lnw_{i,s} - m_s) / S0_s.  With
// A_j the total weight of e_j in J for this walker, the adjoint of Y obeys
//   lambda_K = A_K grad e(Y_K),
//   lambda_j = lambda_{j+1} + grad_Y F_j,   F_j = dt lambda_{j+1} . b(Y_j) + A_j e(Y_j),
// and dJ/dtheta = sum_j d_theta F_j (lambda_{K+1} = 0).  One reverse-mode
// pass through the trial evaluation gives grad_Y F and d_theta F together.
#pragma once

#include "hefk_device.hpp"

namespace hefk {

// grad_Y and d(alpha, beta) of F = V . b(Y) + A e(Y), V = dt lambda (6-vector).
template <int TRIAL>
HD void vjp_trial(const TrialParams<double>& p, const double y[6], const double V[6], double A, double gy[6],
                  double gth[2])
{
    const double al = p.A;
    // forward intermediates
    const double R1[3] = {y[0], y[1], y[2]};
    const double R2[3] = {y[3], y[4], y[5]};
    const double D[3] = {y[0] - y[3], y[1] - y[4], y[2] - y[5]};
    double r1, r2, r12, i1, i2, i12;
    m::dist_inv(R1[0] * R1[0] + R1[1] * R1[1] + R1[2] * R1[2], r1, i1);
    m::dist_inv(R2[0] * R2[0] + R2[1] * R2[1] + R2[2] * R2[2], r2, i2);
    m::dist_inv(D[0] * D[0] + D[1] * D[1] + D[2] * D[2], r12, i12);
    double h1[3], h2[3], h12[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        h1[k] = R1[k] * i1;
        h2[k] = R2[k] * i2;
        h12[k] = D[k] * i12;
    }
    double up = 0.0, is = 0.0;
    if (TRIAL == TRIAL_PADE) {
        is = m::rcp_(1.0 + p.beta * r12);
        up = p.c * is * is;
    }
    double w = 0.0, vh = 0.0, dvh12 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        w += (h1[k] - h2[k]) * h12[k];
        vh += V[k] * h1[k] + V[3 + k] * h2[k];
        dvh12 += (V[k] - V[3 + k]) * h12[k];
    }

    // adjoints of the intermediates
    double bh1[3], bh2[3], bh12[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        bh1[k] = -al * V[k] + A * al * up * h12[k];
        bh2[k] = -al * V[3 + k] - A * al * up * h12[k];
        bh12[k] = up * (V[k] - V[3 + k]) + A * al * up * (h1[k] - h2[k]);
    }
    double bi1 = A * (al - p.Z);
    double bi2 = bi1;
    double bi12 = A * (p.ee - 2.0 * up);
    double balpha = -vh + A * (-2.0 * al + i1 + i2 + up * w);
    double bbeta = 0.0;
    double br12 = 0.0;
    if (TRIAL == TRIAL_PADE) {
        const double bup = dvh12 + A * (al * w - 2.0 * up - 2.0 * i12);
        const double bupp = -A;
        // up = c is^2, upp = -2 c beta is^3
        const double bis = bup * 2.0 * p.c * is + bupp * (-6.0 * p.c * p.beta * is * is);
        bbeta += bupp * (-2.0 * p.c * is * is * is);
        // is = 1 / s, s = 1 + beta r12
        const double bs = -bis * is * is;
        br12 += bs * p.beta;
        bbeta += bs * r12;
    }
    // geometry: h = R / r, i = 1 / r, r = |R|
    double bD[3];
    double dot12 = 0.0, dot1 = 0.0, dot2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        bD[k] = bh12[k] * i12;
        dot12 += bh12[k] * D[k];
        dot1 += bh1[k] * R1[k];
        dot2 += bh2[k] * R2[k];
    }
    bi12 += dot12;
    bi1 += dot1;
    bi2 += dot2;
    br12 += -bi12 * i12 * i12;
    const double br1 = -bi1 * i1 * i1;
    const double br2 = -bi2 * i2 * i2;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        bD[k] += br12 * h12[k];
        gy[k] = bh1[k] * i1 + br1 * h1[k] + bD[k];
        gy[3 + k] = bh2[k] * i2 + br2 * h2[k] - bD[k];
    }
    gth[0] = balpha;
    gth[1] = bbeta;
}

// d ln|psi(Y)| / d(alpha, beta) for the start-law score term.
template <int TRIAL>
HD void dlnpsi_dtheta(const TrialParams<double>& p, const double y[6], double out[2])
{
    const double r1 = ::sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    const double r2 = ::sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
    out[0] = -(r1 + r2);
    out[1] = 0.0;
    if (TRIAL == TRIAL_PADE) {
        const double d0 = y[0] - y[3], d1 = y[1] - y[4], d2 = y[2] - y[5];
        const double r12 = ::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        const double s = 1.0 + p.beta * r12;
        out[1] = -p.c * r12 * r12 / (s * s);
    }
}

// Weight A_j of e_j = E_L(Y_j) - e_ref in J for one walker, given the running
// sum P of g_s p_{i,s} over samples after step j and H = g_s p_{i,s} of a
// sample at step j (0 if none).
HD double adjoint_weight(int j, double P, double H, double dt, bool right)
{
    if (right) return j == 0 ? 0.0 : -dt * (P + H);
    return j == 0 ? -0.5 * dt * P : -dt * (P + 0.5 * H);
}

}  // namespace hefk
