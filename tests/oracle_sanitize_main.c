/*
 * Driver of the CPU oracle for sanitizer builds (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only): the oracle's C file is
 * compiled into this program and run over the 4096-walker ground state in
 * full and over ragged ensembles of every trial with a node, every noise,
 * quadrature and variant, plus the complex-step gradient and the space
 * average of partly absorbed ensembles.  Any sanitizer report aborts with a
 * nonzero status.  Test infrastructure only.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/he_fk_oracle.c"

static ofk_params base(int trial)
{
    ofk_params p;
    memset(&p, 0, sizeof(p));
    p.trial = trial;
    p.sym = 1;
    p.ee = 1;
    p.contract = 1;
    p.n_metropolis = 100;
    p.Z = 2.0;
    p.theta[0] = 2.0;
    p.theta[1] = 0.3;
    p.theta[2] = 0.25;
    p.theta[3] = 0.6;
    p.theta[4] = 0.8;
    p.dt = 0.002;
    p.e_ref = -2.1;
    p.metropolis_sigma = 0.5;
    p.init_sigma = 1.0;
    p.seed = 7;
    return p;
}

static double run(const ofk_params* p, int64_t n, int64_t n_steps, int64_t every)
{
    uint64_t* ids = malloc(sizeof(uint64_t) * n);
    double* x = malloc(sizeof(double) * 6 * n);
    double* el = malloc(sizeof(double) * n);
    double* lnw = calloc(n, sizeof(double));
    double* dmin = malloc(sizeof(double) * n);
    const int64_t ns = n_steps / every + 1;
    double* ell = malloc(sizeof(double) * n * ns);
    double* els = malloc(sizeof(double) * n * ns);
    double* rows = malloc(sizeof(double) * 8 * ns);
    for (int64_t i = 0; i < n; ++i) ids[i] = (uint64_t)i * 3 + 1;
    ofk_init(p, ids, n, x, el);
    ofk_propagate(p, ids, n, x, lnw, el, 0, n_steps, every, ell, els, dmin);
    ofk_tuples(ell, els, n, ns, rows);
    const double L = rows[8 * (ns - 1)] + log(rows[8 * (ns - 1) + 1]);
    free(ids); free(x); free(el); free(lnw); free(dmin); free(ell); free(els); free(rows);
    return L;
}

int main(void)
{
    double acc = 0.0;
    ofk_params p = base(OFK_TRIAL_EXPO);  /* the 4096-walker ground state in full */
    p.theta[0] = 27.0 / 16.0;
    p.dt = 0.01;
    p.n_metropolis = 500;
    p.seed = 42;
    acc += run(&p, 4096, 200, 5);
    const int trials[] = {OFK_TRIAL_PADE, OFK_TRIAL_TRIPLET, OFK_TRIAL_PZ, OFK_TRIAL_TRIPLET_R0, OFK_TRIAL_PZ_SUM};
    for (int t = 0; t < 5; ++t)
        for (int v = 0; v < 6; ++v) {
            p = base(trials[t]);
            if (trials[t] == OFK_TRIAL_PZ_SUM) p.theta[3] = 0.25;
            p.noise = (v & 1) ? OFK_NOISE_PM1 : OFK_NOISE_GAUSS;
            p.contract = (v == 2) ? 2 : 1;
            p.quad = (v & 2) ? OFK_QUAD_RIGHT : OFK_QUAD_TRAPEZOID;
            p.drift_limit = (v == 4) ? 1.0 : 0.0;
            if (v == 5) p.flags = OFK_FLAG_PLAIN;
            if (v == 3 && trials[t] != OFK_TRIAL_PADE) p.flags = OFK_FLAG_BRIDGE;
            acc += run(&p, 257, 400, 20);
            acc += run(&p, 1, 40, 40);
        }
    /* complex-step pathwise derivative (nodeless trials) */
    p = base(OFK_TRIAL_PADE);
    {
        const int64_t n = 33, ns = 200 / 50 + 1;
        uint64_t ids[33];
        double y0[6 * 33], el[33], out[33 * 5];
        for (int i = 0; i < n; ++i) ids[i] = (uint64_t)i;
        ofk_init(&p, ids, n, y0, el);
        for (int d = 0; d < 2; ++d) {
            int st = 0;
            ofk_dlnw_dtheta(&p, ids, n, y0, 200, 50, d, out, &st);
            if (st != 0) return 3;
            for (int64_t k = 0; k < n * ns; ++k) acc += out[k];
            acc += ofk_dlnpsi_dtheta(&p, y0, d);
        }
    }
    printf("%.17g\n", acc);
    return 0;
}
