// Host build of the gradient's per-walker reverse sweep (hefk_sweep.hpp) for
// CPU checks against the oracle's complex-step derivative.  ckpt_every = 1 runs
// the sweep that reads the stored trajectory instead of recomputing segments.
//
// stdin line 1: trial ee quad contract n_met Z t0 t1 t2 t3 dt e_ref metropolis_sigma init_sigma seed
//               n_steps sample_every ckpt_every
// line 2: n_samples, then n_samples quintuples (m_s S0_s S2_s g_s g2_s)
// line 3: n id_0 ... id_{n-1}
// stdout per walker: dJ/dalpha dJ/dbeta P Q (P = sum_s g_s p_is + 2 g2_s q_is, Q = sum_s g2_s q_is)
#include <cstdio>
#include <vector>

#include "hefk_sweep.hpp"

using namespace hefk;

struct HostTape {
    std::vector<double> ck, tp;  // [n_ckpt][7], [ckpt_every + 1][7]
    void load_ckpt(int c, double y[6], double& lnw) const
    {
        for (int k = 0; k < 6; ++k) y[k] = ck[7 * c + k];
        lnw = ck[7 * c + 6];
    }
    void put(int s, const double y[6])
    {
        for (int k = 0; k < 6; ++k) tp[7 * s + k] = y[k];
    }
    void put_lnw(int s, double lnw) { tp[7 * s + 6] = lnw; }
    void get(int s, double y[6]) const
    {
        for (int k = 0; k < 6; ++k) y[k] = tp[7 * s + k];
    }
    double get_lnw(int s) const { return tp[7 * s + 6]; }
    // the checkpoints as the stored trajectory (ckpt_every = 1)
    void load_pos(int c, double y[6]) const
    {
        for (int k = 0; k < 6; ++k) y[k] = ck[7 * c + k];
    }
    double load_lnw(int c) const { return ck[7 * c + 6]; }
};

struct HostSamples {
    std::vector<double> m_, s0_, s2_, g_, g2_;
    double m(int s) const { return m_[s]; }
    double s0(int s) const { return s0_[s]; }
    double s2(int s) const { return s2_[s]; }
    double gs(int s) const { return g_[s]; }
    double g2s(int s) const { return g2_[s]; }
};

template <int TRIAL, int NOISE>
void one(const TrialParams<double>& tp, const StepConst& sc, int n_met, double msig, double isig,
         unsigned long long seed, unsigned long long g, int n_steps, int se, int ce, const HostSamples& hs)
{
    Stream st;
    st.k0 = (uint32_t)seed;
    st.k1 = (uint32_t)(seed >> 32);
    st.g0 = (uint32_t)g;
    st.g1 = (uint32_t)(g >> 32);
    WalkerState<double> w;
    init_walker<TRIAL>(tp, st, n_met, isig, msig, w.y);
    w.lnw = 0.0;
    const StepScale<double> ss = step_scale(sc.dt, 0.0, 0.0);
    walker_reset<double, TRIAL>(tp, sc, ss, w);
    HostTape tape;
    tape.ck.assign(7 * (n_steps / ce + 1), 0.0);
    tape.tp.assign(7 * (ce + 1), 0.0);
    auto save = [&](int c) {
        for (int k = 0; k < 6; ++k) tape.ck[7 * c + k] = w.y[k];
        tape.ck[7 * c + 6] = w.lnw;
    };
    save(0);
    NoiseGen<double, NOISE> noise;
    for (int k = 0; k < n_steps; ++k) {
        Increment<double> inc;
        noise.draw(st, (uint32_t)k, ss, inc);
        walker_step<double, TRIAL>(tp, sc, ss, inc, w);
        if ((k + 1) % ce == 0) save((k + 1) / ce);
    }
    double gth[2] = {0, 0}, P = 0, Q = 0;
    if (ce == 1)
        walker_reverse_direct<TRIAL>(tp, sc, ss, n_steps, se, hs, tape, gth, &P, &Q);
    else
        walker_reverse<TRIAL, NOISE>(tp, sc, ss, st, n_steps, se, ce, hs, tape, gth, &P, &Q);
    std::printf("%.17g %.17g %.17g %.17g\n", gth[0], gth[1], P, Q);
}

int main()
{
    int trial, ee, quad, contract, n_met, n_steps, se, ce;
    double Z, th[4], dt, e_ref, msig, isig;
    unsigned long long seed;
    if (std::scanf("%d %d %d %d %d %lf %lf %lf %lf %lf %lf %lf %lf %lf %llu %d %d %d", &trial, &ee, &quad, &contract,
                   &n_met, &Z, &th[0], &th[1], &th[2], &th[3], &dt, &e_ref, &msig, &isig, &seed, &n_steps, &se,
                   &ce) != 18)
        return 2;
    int ns;
    if (std::scanf("%d", &ns) != 1) return 2;
    HostSamples hs;
    for (int s = 0; s < ns; ++s) {
        double a, b, c, d, e;
        if (std::scanf("%lf %lf %lf %lf %lf", &a, &b, &c, &d, &e) != 5) return 2;
        hs.m_.push_back(a);
        hs.s0_.push_back(b);
        hs.s2_.push_back(c);
        hs.g_.push_back(d);
        hs.g2_.push_back(e);
    }
    TrialParams<double> tp{th[0], th[1], th[2], th[3], Z, (double)ee, 1.0, 0.0};
    const StepConst sc = make_step_const(dt, e_ref, quad != 0, 0.0, false, false);
    long n;
    if (std::scanf("%ld", &n) != 1) return 2;
    for (long i = 0; i < n; ++i) {
        unsigned long long g;
        if (std::scanf("%llu", &g) != 1) return 2;
        if (trial == TRIAL_EXPO) {
            if (contract == 2) one<TRIAL_EXPO, NOISE_G2>(tp, sc, n_met, msig, isig, seed, g, n_steps, se, ce, hs);
            else one<TRIAL_EXPO, NOISE_G1>(tp, sc, n_met, msig, isig, seed, g, n_steps, se, ce, hs);
        } else {
            if (contract == 2) one<TRIAL_PADE, NOISE_G2>(tp, sc, n_met, msig, isig, seed, g, n_steps, se, ce, hs);
            else one<TRIAL_PADE, NOISE_G1>(tp, sc, n_met, msig, isig, seed, g, n_steps, se, ce, hs);
        }
    }
    return 0;
}
