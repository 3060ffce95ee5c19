"""Energy estimators of the oracle (plain numpy, FP64).  TEST INFRASTRUCTURE ONLY.

Input: the per-sample space-average rows (m, S0, S1, S2, n_alive, n_nonfinite,
n_total, 0) at times t_j = j * dt_sample.

* L_j = ln( (1/N) sum_i w_ij ) = m_j + ln S0_j - ln N_j  (Z(t) of the space
  average, kept in the log domain; absorbed walkers count in N with weight 0).
* Eq. (4) with lambda0 = e_ref gives lambda1 = e_ref - lim L(t)/t, and the
  time derivative of ln Z(t) gives the finite-difference estimator
  E_fd(t_j) = e_ref - (L_j - L_{j-1}) / dt_sample.
* Window: E_win = e_ref - ordinary least-squares slope of L_j on t_j for
  t_j in [T/2, T].
* Fit (the "ls fit" columns of Tables 1-5): least squares of L_j / t_j =
  b + a / t_j over t_j > 0, optionally weighted; lambda1 = e_ref - b.
* Mixed: S1_j / S0_j (weighted mean local energy, a diagnostic).
* Effective sample size S0^2 / S2.
"""
from __future__ import annotations

import numpy as np


def log_mean_weight(samples):
    s = np.asarray(samples, dtype=np.float64)
    return s[:, 0] + np.log(s[:, 1]) - np.log(s[:, 6])


def log_mean_square_weight(samples):
    """ln((1/N) sum w^2) from the rows: 2 m + ln S2 - ln N.  With L it gives the relative
    variance of the weights, ln(<w^2> / <w>^2) = L2 - 2 L, i.e. -ln(ESS / N)."""
    s = np.asarray(samples, dtype=np.float64)
    return 2.0 * s[:, 0] + np.log(s[:, 3]) - np.log(s[:, 6])


def e_fd(samples, dt_sample, e_ref):
    L = log_mean_weight(samples)
    return e_ref - np.diff(L) / dt_sample


def e_window(samples, dt_sample, e_ref):
    L = log_mean_weight(samples)
    t = np.arange(len(L)) * dt_sample
    T = t[-1]
    sel = t >= 0.5 * T - 1e-12 * T
    tt, LL = t[sel], L[sel]
    A = np.stack([np.ones_like(tt), tt], axis=1)
    coef, *_ = np.linalg.lstsq(A, LL, rcond=None)
    return e_ref - coef[1]


def fit_b_a(t, y, w=None):
    """Weighted least squares of y = b + a / t; returns (b, a)."""
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    w = np.ones_like(t) if w is None else np.asarray(w, dtype=np.float64)
    A = np.stack([np.ones_like(t), 1.0 / t], axis=1)
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)
    return coef[0], coef[1]


def e_fit(samples, dt_sample, e_ref, w=None):
    L = log_mean_weight(samples)
    t = np.arange(len(L)) * dt_sample
    b, a = fit_b_a(t[1:], L[1:] / t[1:], None if w is None else np.asarray(w)[1:])
    return e_ref - b, a


def e_mixed(samples):
    s = np.asarray(samples, dtype=np.float64)
    return s[:, 2] / s[:, 1]


def ess(samples):
    s = np.asarray(samples, dtype=np.float64)
    return s[:, 1] ** 2 / s[:, 3]
