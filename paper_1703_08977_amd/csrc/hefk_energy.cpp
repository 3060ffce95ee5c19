// hefk_energy.cpp -- host estimators of the energy from the sample rows of
// he_fk_propagate (log space average L(t) = ln((1/N) sum_i w_i(t))).
//
//   eq. (4): lambda1 = lambda0 - lim_t L(t)/t with lambda0 = e_ref, and the
//   time derivative of ln Z(t) for the finite-difference estimator;
//   the paper's extrapolation ("ls fit" columns of Tables 1-5): the least-
//   squares fit L(t)/t = b + a/t, lambda1 = lambda0 - b.
#include <math.h>
#include <stdint.h>

#include <new>

#include "he_fk.h"

namespace {

double log_space_average(const double* r) { return r[0] + log(r[1]) - log(r[6]); }

// Weighted least squares of y = c0 + c1 x, centred sums; returns 0 on success.
int wls_line(int64_t n, const double* x, const double* y, const double* w, double* c0, double* c1)
{
    double sw = 0, sx = 0, sy = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double wj = w ? w[j] : 1.0;
        sw += wj;
        sx += wj * x[j];
        sy += wj * y[j];
    }
    if (!(sw > 0)) return -1;
    const double mx = sx / sw, my = sy / sw;
    double sxx = 0, sxy = 0;
    for (int64_t j = 0; j < n; ++j) {
        const double wj = w ? w[j] : 1.0;
        sxx += wj * (x[j] - mx) * (x[j] - mx);
        sxy += wj * (x[j] - mx) * (y[j] - my);
    }
    if (!(sxx > 0)) return -1;
    *c1 = sxy / sxx;
    *c0 = my - *c1 * mx;
    return 0;
}

}  // namespace

extern "C" int he_fk_energy(const double* samples, int64_t n_samples, double dt_sample, double e_ref,
                            int32_t method, const double* fit_w, double* E_out, double* aux_out)
{
    if (!samples || !E_out || n_samples < 1 || !(dt_sample > 0) || !isfinite(dt_sample) || !isfinite(e_ref))
        return HE_FK_EINVAL;
    if (method < HE_FK_E_FD || method > HE_FK_E_MIXED) return HE_FK_EINVAL;
    if ((method == HE_FK_E_FD || method == HE_FK_E_WINDOW) && n_samples < 2) return HE_FK_EINVAL;
    if (method == HE_FK_E_FIT && n_samples < 3) return HE_FK_EINVAL;

    int status = HE_FK_OK;
    for (int64_t j = 0; j < n_samples; ++j) {
        const double* r = samples + 8 * j;
        if (!(r[6] >= 1.0)) return HE_FK_EINVAL;
        if (aux_out) {
            aux_out[2 * j] = log_space_average(r);
            aux_out[2 * j + 1] = r[1] * r[1] / r[3];
        }
        if (r[5] > 0.0)
            status = HE_FK_ENONFINITE;
        else if (r[4] < 1.0 && status == HE_FK_OK)
            status = HE_FK_EALLDEAD;
    }
    if (status) return status;

    if (method == HE_FK_E_FD) {
        double prev = log_space_average(samples);
        for (int64_t j = 1; j < n_samples; ++j) {
            const double L = log_space_average(samples + 8 * j);
            E_out[j - 1] = e_ref - (L - prev) / dt_sample;
            prev = L;
        }
        return HE_FK_OK;
    }
    if (method == HE_FK_E_MIXED) {
        for (int64_t j = 0; j < n_samples; ++j) E_out[j] = samples[8 * j + 2] / samples[8 * j + 1];
        return HE_FK_OK;
    }
    // WINDOW: rows with t_j >= T/2, i.e. 2 j >= n_samples - 1
    // FIT: rows with t_j > 0, y = L/t against x = 1/t
    const int64_t j0 = (method == HE_FK_E_WINDOW) ? (n_samples / 2) : 1;
    const int64_t m = n_samples - j0;
    double xs_stack[256], ys_stack[256];
    double* xs = xs_stack;
    double* ys = ys_stack;
    double* heap = nullptr;
    if (m > 256) {
        heap = new (std::nothrow) double[2 * m];
        if (!heap) return HE_FK_EINVAL;
        xs = heap;
        ys = heap + m;
    }
    for (int64_t j = j0; j < n_samples; ++j) {
        const double t = (double)j * dt_sample;
        const double L = log_space_average(samples + 8 * j);
        if (method == HE_FK_E_WINDOW) {
            xs[j - j0] = t;
            ys[j - j0] = L;
        } else {
            xs[j - j0] = 1.0 / t;
            ys[j - j0] = L / t;
        }
    }
    double c0 = 0, c1 = 0;
    const int rc = wls_line(m, xs, ys, (method == HE_FK_E_FIT && fit_w) ? fit_w + j0 : nullptr, &c0, &c1);
    delete[] heap;
    if (rc) return HE_FK_EINVAL;
    if (method == HE_FK_E_WINDOW) {
        E_out[0] = e_ref - c1;
    } else {
        E_out[0] = e_ref - c0;
        E_out[1] = c1;
    }
    return HE_FK_OK;
}
