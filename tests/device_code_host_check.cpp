// Host build of the kernels' per-walker arithmetic (hefk_device.hpp) for CPU
// checks against the oracle: same start (Metropolis), same noise, same step,
// same sampling as the propagate kernel, one walker at a time.
//
// stdin, line 1: trial sym ee noise contract quad precision n_met flags Z t0 t1 t2 t3 t4
//                dt e_ref metropolis_sigma init_sigma drift_limit seed n_steps sample_every
// line 2:        n id_0 ... id_{n-1}
// stdout, per walker one line: x0[6] x[6] lnw el ell[ns] els[ns]
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hefk_device.hpp"

using namespace hefk;

struct Cfg {
    int trial, sym, ee, noise, contract, quad, precision, n_met, flags;
    double Z, th[5], dt, e_ref, msig, isig, limit;
    unsigned long long seed;
    long n_steps, sample_every;
};

template <typename R>
TrialParams<R> tparams(const Cfg& c)
{
    TrialParams<R> t;
    t.A = (R)c.th[0];
    t.beta = (R)c.th[1];
    t.c = (R)c.th[2];
    t.a = (R)c.th[3];
    t.Z = (R)c.Z;
    t.ee = (R)c.ee;
    t.sym = (R)(c.trial == TRIAL_PZ ? c.sym : 1);
    t.r0 = (R)c.th[4];
    return t;
}

template <typename R, int TRIAL, int NOISE, bool EXT>
void run_walker(const Cfg& c, unsigned long long g)
{
    Stream st;
    st.k0 = (uint32_t)c.seed;
    st.k1 = (uint32_t)(c.seed >> 32);
    st.g0 = (uint32_t)g;
    st.g1 = (uint32_t)(g >> 32);
    const TrialParams<double> tpd = tparams<double>(c);
    const TrialParams<R> tp = tparams<R>(c);
    double y0[6];
    init_walker<TRIAL>(tpd, st, c.n_met, c.isig, c.msig, y0);
    WalkerState<R> w;
    for (int k = 0; k < 6; ++k) w.y[k] = (R)y0[k];
    w.lnw = 0.0;
    const StepConst sc =
        make_step_const(c.dt, c.e_ref, c.quad == 1, c.limit, (c.flags & 1) != 0, (c.flags & 2) != 0);
    const StepScale<R> ss = step_scale(c.dt, c.limit, R());
    walker_reset<R, TRIAL, EXT>(tp, sc, ss, w);
    std::vector<double> ell, els;
    ell.push_back(w.lnw);
    els.push_back((double)w.el);
    NoiseGen<R, NOISE> noise;
    for (long k = 0; k < c.n_steps; ++k) {
        Increment<R> inc;
        noise.draw(st, (uint32_t)k, ss, inc);
        walker_step<R, TRIAL, EXT>(tp, sc, ss, inc, w);
        if ((k + 1) % c.sample_every == 0) {
            ell.push_back(w.lnw);
            els.push_back((double)w.el);
        }
    }
    for (int k = 0; k < 6; ++k) std::printf("%.17g ", y0[k]);
    for (int k = 0; k < 6; ++k) std::printf("%.17g ", (double)w.y[k]);
    std::printf("%.17g %.17g", w.lnw, (double)w.el);
    for (double v : ell) std::printf(" %.17g", v);
    for (double v : els) std::printf(" %.17g", v);
    std::printf("\n");
}

template <typename R, int TRIAL, bool EXT>
void dispatch_noise_x(const Cfg& c, unsigned long long g)
{
    const int nk = c.noise == 1 ? NOISE_PM1 : (c.contract == 2 ? NOISE_G2 : NOISE_G1);
    if (nk == NOISE_G1) run_walker<R, TRIAL, NOISE_G1, EXT>(c, g);
    else if (nk == NOISE_G2) run_walker<R, TRIAL, NOISE_G2, EXT>(c, g);
    else run_walker<R, TRIAL, NOISE_PM1, EXT>(c, g);
}

template <typename R, int TRIAL>
void dispatch_noise(const Cfg& c, unsigned long long g)
{
    if (c.flags) dispatch_noise_x<R, TRIAL, true>(c, g);
    else dispatch_noise_x<R, TRIAL, false>(c, g);
}

template <typename R>
void dispatch(const Cfg& c, unsigned long long g)
{
    switch (c.trial) {
        case TRIAL_EXPO: dispatch_noise<R, TRIAL_EXPO>(c, g); break;
        case TRIAL_PADE: dispatch_noise<R, TRIAL_PADE>(c, g); break;
        case TRIAL_TRIPLET: dispatch_noise<R, TRIAL_TRIPLET>(c, g); break;
        case TRIAL_TRIPLET_R0: dispatch_noise<R, TRIAL_TRIPLET_R0>(c, g); break;
        case TRIAL_PZ_SUM: dispatch_noise<R, TRIAL_PZ_SUM>(c, g); break;
        default: dispatch_noise<R, TRIAL_PZ>(c, g); break;
    }
}

int main()
{
    Cfg c;
    if (std::scanf("%d %d %d %d %d %d %d %d %d %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %lf %llu %ld %ld", &c.trial,
                   &c.sym, &c.ee, &c.noise, &c.contract, &c.quad, &c.precision, &c.n_met, &c.flags, &c.Z, &c.th[0],
                   &c.th[1], &c.th[2], &c.th[3], &c.th[4], &c.dt, &c.e_ref, &c.msig, &c.isig, &c.limit, &c.seed,
                   &c.n_steps, &c.sample_every) != 23)
        return 2;
    long n = 0;
    if (std::scanf("%ld", &n) != 1) return 2;
    for (long i = 0; i < n; ++i) {
        unsigned long long g;
        if (std::scanf("%llu", &g) != 1) return 2;
        if (c.precision == 1)
            dispatch<float>(c, g);
        else
            dispatch<double>(c, g);
    }
    return 0;
}
