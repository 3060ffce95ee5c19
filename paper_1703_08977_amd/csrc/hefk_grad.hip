// hefk_grad.hip -- pathwise (fixed-noise) gradient of the log space average
// with respect to the trial parameters: reverse sweep over checkpoint segments.
#include <hip/hip_runtime.h>

#include "he_fk.h"

extern "C" size_t he_fk_grad_scratch_bytes(const he_fk_params* p, int64_t n_steps, int32_t sample_every,
                                           int32_t ckpt_every)
{
    (void)p;
    (void)n_steps;
    (void)sample_every;
    (void)ckpt_every;
    return 0;
}

extern "C" int he_fk_grad(const he_fk_params* p, const he_fk_walkers* y0, const double* ckpt,
                          const double* samples, const double* gL, int64_t n_steps, int32_t sample_every,
                          int32_t ckpt_every, int32_t flags, void* scratch, size_t scratch_bytes,
                          double* dtheta, void* stream)
{
    (void)p; (void)y0; (void)ckpt; (void)samples; (void)gL; (void)n_steps; (void)sample_every;
    (void)ckpt_every; (void)flags; (void)scratch; (void)scratch_bytes; (void)dtheta; (void)stream;
    return HE_FK_EINVAL;
}
