// hefk_sweep.hpp -- the per-walker reverse sweep of the pathwise gradient
// (host + device).  The tape accessor holds the checkpoints (state every
// ckpt_every steps) and a scratch tape for one segment; the sample view gives
// m_s, S0_s of each sample row and the objective weights g_s.  Two sweeps:
// walker_reverse recomputes each segment from its checkpoint; with a checkpoint
// at every step the stored trajectory is the tape, and walker_reverse_direct
// reads it without recomputing.  Both apply reverse_step in the same order, so
// they give the same bits.
#pragma once

#include "hefk_adjoint.hpp"

namespace hefk {

// Reverse step j of the adjoint recursion, at the position y_j (ln w_j is read, through
// lnw_at(), only when j is a sampling step): accumulates dJ/dtheta and the running
// weight sums.
template <int TRIAL, class Samples, class LnW>
HD void reverse_step(const TrialParams<double>& tp, double dt, bool right, int j, int sample_every, const double y[6],
                     const LnW& lnw_at, const Samples& sv, double lam[6], double gth[2], double& P, double& Q)
{
    double H = 0.0;
    if (j % sample_every == 0) {
        const double lnw = lnw_at();
        // dJ/d ln w_j: g_s p_is + 2 g2_s q_is, with the walker's shares
        // p_is = w / sum w of L_s and q_is = w^2 / sum w^2 of L2_s
        const int s = j / sample_every;
        const double e = ::exp(lnw - sv.m(s));
        H = sv.gs(s) * e / sv.s0(s);
        const double g2 = sv.g2s(s);
        if (g2 != 0.0) {
            const double q = g2 * (e * e) / sv.s2(s);
            H += 2.0 * q;
            Q += q;
        }
    }
    const double A = adjoint_weight(j, P, H, dt, right);
    double V[6], gy[6], gt[2];
#pragma unroll
    for (int k = 0; k < 6; ++k) V[k] = dt * lam[k];
    vjp_trial<TRIAL>(tp, y, V, A, gy, gt);
#pragma unroll
    for (int k = 0; k < 6; ++k) lam[k] += gy[k];
    gth[0] += gt[0];
    gth[1] += gt[1];
    P += H;
}

template <int TRIAL, int NOISE, class Samples, class Tape>
HD void walker_reverse(const TrialParams<double>& tp, const StepConst& sc, const StepScale<double>& ss, const Stream& st,
                       int n_steps, int sample_every, int ckpt_every, const Samples& sv, Tape& tape, double gth[2],
                       double* p_total, double* q_total)
{
    const bool right = sc.quad_right != 0;
    const double dt = ss.dt;
    const int n_seg = n_steps / ckpt_every;
    double lam[6] = {0, 0, 0, 0, 0, 0};
    double P = 0.0, Q = 0.0;
    for (int seg = n_seg - 1; seg >= 0; --seg) {
        const int k0 = seg * ckpt_every;
        // recompute the segment from its checkpoint (same arithmetic as the forward kernel)
        WalkerState<double> w;
        tape.load_ckpt(seg, w.y, w.lnw);
        walker_reset<double, TRIAL>(tp, sc, ss, w);
        // the tape holds every step's position, and ln w only where the reverse pass reads
        // it: at the sampling steps
        tape.put(0, w.y);
        if (k0 % sample_every == 0) tape.put_lnw(0, w.lnw);
        NoiseGen<double, NOISE> noise;
        for (int k = 0; k < ckpt_every; ++k) {
            Increment<double> inc;
            noise.draw(st, (uint32_t)(k0 + k), ss, inc);
            walker_step<double, TRIAL>(tp, sc, ss, inc, w);
            tape.put(k + 1, w.y);
            if ((k0 + k + 1) % sample_every == 0) tape.put_lnw(k + 1, w.lnw);
        }
        // reverse over the steps of the segment (step k0 belongs to the segment below, except k0 = 0)
        const int j_lo = (seg == 0) ? 0 : k0 + 1;
        for (int j = k0 + ckpt_every; j >= j_lo; --j) {
            double y[6];
            tape.get(j - k0, y);
            reverse_step<TRIAL>(tp, dt, right, j, sample_every, y, [&] { return tape.get_lnw(j - k0); }, sv, lam, gth,
                                P, Q);
        }
    }
    *p_total = P;  // sum_s (g_s p_is + 2 g2_s q_is)
    *q_total = Q;  // sum_s g2_s q_is
}

// The sweep over a trajectory stored at every step (checkpoints with ckpt_every = 1):
// the positions of step j - 1 are read while step j is computed.
template <int TRIAL, class Samples, class Tape>
HD void walker_reverse_direct(const TrialParams<double>& tp, const StepConst& sc, const StepScale<double>& ss,
                              int n_steps, int sample_every, const Samples& sv, const Tape& tape, double gth[2],
                              double* p_total, double* q_total)
{
    const bool right = sc.quad_right != 0;
    const double dt = ss.dt;
    double lam[6] = {0, 0, 0, 0, 0, 0};
    double P = 0.0, Q = 0.0;
    double yn[6];
    tape.load_pos(n_steps, yn);
    for (int j = n_steps; j >= 0; --j) {
        double y[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) y[k] = yn[k];
        if (j > 0) tape.load_pos(j - 1, yn);
        reverse_step<TRIAL>(tp, dt, right, j, sample_every, y, [&] { return tape.load_lnw(j); }, sv, lam, gth, P, Q);
    }
    *p_total = P;
    *q_total = Q;
}

}  // namespace hefk
