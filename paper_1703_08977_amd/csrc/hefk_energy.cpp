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
// ln of the mean square weight, ln((1/N) sum w^2) = 2 m + ln S2 - ln N
double log_mean_square(const double* r) { return 2.0 * r[0] + log(r[3]) - log(r[6]); }

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
            aux_out[3 * j] = log_space_average(r);
            aux_out[3 * j + 1] = r[1] * r[1] / r[3];
            aux_out[3 * j + 2] = log_mean_square(r);
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

// ---------------------------------------------------------------------------
// Error bars from one run: the per-block partial rows of he_fk_propagate cover
// fixed, disjoint sets of walkers, so groups of blocks are independent
// sub-ensembles.  Rows merge by rescaling to the larger maximum, as on the device.
// ---------------------------------------------------------------------------
namespace {

// acc <- acc (+) r for one sample row (m, S0, S1, S2, n_alive, n_nonfinite, n_total, 0)
void merge_row(double* acc, const double* r)
{
    const double ma = acc[0], mb = r[0];
    const double m = (mb > ma) ? mb : ma;
    const double fa = (ma == -INFINITY) ? 0.0 : exp(ma - m);
    const double fb = (mb == -INFINITY) ? 0.0 : exp(mb - m);
    acc[0] = m;
    acc[1] = acc[1] * fa + r[1] * fb;
    acc[2] = acc[2] * fa + r[2] * fb;
    acc[3] = acc[3] * fa * fa + r[3] * fb * fb;
    acc[4] += r[4];
    acc[5] += r[5];
    acc[6] += r[6];
    acc[7] = 0.0;
}

void empty_rows(double* rows, int64_t n_samples)
{
    for (int64_t j = 0; j < n_samples; ++j) {
        double* r = rows + 8 * j;
        r[0] = -INFINITY;
        for (int k = 1; k < 8; ++k) r[k] = 0.0;
    }
}

// The scalar statistic of an estimator: WINDOW the window energy, FIT lambda1 = e_ref - b,
// FD the energy of the last sampling interval, MIXED the mixed estimate at the last row.
int statistic(const double* rows, int64_t n_samples, double dt_sample, double e_ref, int32_t method,
              const double* fit_w, double* tmp, double* out)
{
    const int rc = he_fk_energy(rows, n_samples, dt_sample, e_ref, method, fit_w, tmp, nullptr);
    if (rc) return rc;
    *out = (method == HE_FK_E_FD) ? tmp[n_samples - 2] : (method == HE_FK_E_MIXED) ? tmp[n_samples - 1] : tmp[0];
    return HE_FK_OK;
}

}  // namespace

extern "C" int he_fk_energy_blocks(const double* partials, int64_t n_parts, int64_t n_samples, int32_t n_groups,
                                   double dt_sample, double e_ref, int32_t method, const double* fit_w,
                                   double* est_out)
{
    if (!partials || !est_out || n_parts < 2 || n_samples < 1 || n_groups < 2) return HE_FK_EINVAL;
    if (method < HE_FK_E_FD || method > HE_FK_E_MIXED) return HE_FK_EINVAL;
    const int64_t G = n_groups < n_parts ? n_groups : n_parts;
    // group g holds blocks [g q + min(g, r), (g + 1) q + min(g + 1, r)), q = n_parts / G, r = n_parts % G
    const int64_t q = n_parts / G, rem = n_parts % G;
    double* grows = new (std::nothrow) double[(size_t)(G + 2) * (size_t)n_samples * 8 + (size_t)n_samples + G];
    if (!grows) return HE_FK_EINVAL;
    double* all = grows + (size_t)G * n_samples * 8;
    double* rest = all + (size_t)n_samples * 8;
    double* tmp = rest + (size_t)n_samples * 8;  // [n_samples]: the estimator's output
    double* reps = tmp + n_samples;              // [G]: the delete-one-group replicas
    int64_t b = 0;
    for (int64_t g = 0; g < G; ++g) {
        double* gr = grows + (size_t)g * n_samples * 8;
        empty_rows(gr, n_samples);
        const int64_t end = (g + 1) * q + ((g + 1) < rem ? (g + 1) : rem);
        for (; b < end; ++b)
            for (int64_t j = 0; j < n_samples; ++j) merge_row(gr + 8 * j, partials + ((size_t)b * n_samples + j) * 8);
    }
    empty_rows(all, n_samples);
    for (int64_t g = 0; g < G; ++g)
        for (int64_t j = 0; j < n_samples; ++j) merge_row(all + 8 * j, grows + ((size_t)g * n_samples + j) * 8);
    int rc = statistic(all, n_samples, dt_sample, e_ref, method, fit_w, tmp, &est_out[0]);
    // delete-one-group replicas: their mean, then the jackknife variance (G - 1)/G sum (x_g - mean)^2
    double sum = 0.0;
    for (int64_t g = 0; g < G && !rc; ++g) {
        empty_rows(rest, n_samples);
        for (int64_t h = 0; h < G; ++h)
            if (h != g)
                for (int64_t j = 0; j < n_samples; ++j) merge_row(rest + 8 * j, grows + ((size_t)h * n_samples + j) * 8);
        rc = statistic(rest, n_samples, dt_sample, e_ref, method, fit_w, tmp, &reps[g]);
        sum += reps[g];
    }
    if (!rc) {
        const double mean = sum / (double)G;
        double ss = 0.0;
        for (int64_t g = 0; g < G; ++g) ss += (reps[g] - mean) * (reps[g] - mean);
        est_out[1] = sqrt((double)(G - 1) / (double)G * ss);
    }
    delete[] grows;
    return rc;
}
