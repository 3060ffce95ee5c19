"""Coefficients of the binary64 polynomials in hefk_f64math.hpp.

Each function is approximated on the argument range the step gives it by a
weighted least-squares polynomial over Chebyshev points, in high precision
(mpmath, 160 digits); the coefficients are fixed one at a time, lowest order
first: a coefficient is rounded to binary64 and the remaining ones are
refitted to what is left, so the rounding of each is absorbed by the next.  Printed as C++ hexadecimal floating literals, with the largest
approximation error over a dense grid (binary64 coefficients, exact
evaluation), in units of 2^-53 (relative, absolute for cos, and relative to
the factor 1 + z R it enters for the logarithm's series).

    python paper_1703_08977_amd/csrc/f64_coeffs.py
"""
from __future__ import annotations

import mpmath as mp

mp.mp.dps = 160


def fit_rounded(f, a, b, n, weight, m=240):
    """Coefficients c_0..c_n (binary64) of f(x) ~ sum c_j x^j on [a, b], fixed lowest order first: at each
    order j the remainder f - sum_{i<j} c_i x^i is fitted on the basis x^j .. x^n by least squares over m
    Chebyshev points with the error weights weight(x, f(x)), and c_j is rounded to binary64."""
    xs = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (2 * k + 1) / (2 * m)) for k in range(m)]
    fx = [f(x) for x in xs]
    wt = [weight(x, v) for x, v in zip(xs, fx)]
    fixed = []
    for j in range(n + 1):
        r = [fx[k] - sum(mp.mpf(c) * xs[k] ** i for i, c in enumerate(fixed)) for k in range(m)]
        A = mp.matrix([[wt[k] * xs[k] ** i for i in range(j, n + 1)] for k in range(m)])
        y = mp.matrix([wt[k] * r[k] for k in range(m)])
        c = mp.lu_solve(A.T * A, A.T * y)
        fixed.append(float(c[0]))
    return fixed


def max_error(f, c, a, b, weight, n=4000):
    e = mp.mpf(0)
    for k in range(n + 1):
        x = a + (b - a) * k / n
        p = mp.mpf(0)
        for cj in reversed(c):
            p = p * x + mp.mpf(cj)
        fx = f(x)
        e = max(e, abs(p - fx) * weight(x, fx))
    return float(e / mp.mpf(2) ** -53)


def main():
    q = mp.mpf(1) / 16  # y in [0, 1/4]: w = y^2 in [0, 1/16]
    s_max = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)
    z_max = s_max ** 2
    h = mp.log(2) / 2
    relative = lambda x, fx: 1 / abs(fx)  # noqa: E731
    absolute = lambda x, fx: mp.mpf(1)  # noqa: E731
    # log m = 2 s (1 + z R(z)): an error in R counts as z dR / (1 + z R) relative to the result
    in_log = lambda z, r: z / (1 + z * r)  # noqa: E731
    specs = [
        # name, f, interval, degree, error weight, what the error is relative to
        ("SIN_PI", lambda w: mp.sin(mp.pi * mp.sqrt(w)) / mp.sqrt(w) if w else mp.pi, (mp.mpf(0), q), 6, relative,
         "relative"),
        ("COS_PI", lambda w: mp.cos(mp.pi * mp.sqrt(w)), (mp.mpf(0), q), 7, absolute, "absolute"),
        ("LOG_R", lambda z: (mp.atanh(mp.sqrt(z)) / mp.sqrt(z) - 1) / z if z else mp.mpf(1) / 3, (mp.mpf(0), z_max), 6,
         in_log, "relative to 1 + z R"),
        ("EXP", mp.exp, (-h, h), 11, relative, "relative"),
        # e^r - 1 = r + r^2 Q(r): an error in Q counts as r^2 dQ / |e^r - 1| relative to the result
        ("EXPM1_Q", lambda r: (mp.exp(r) - 1 - r) / r ** 2 if r else mp.mpf(1) / 2, (-h, h), 10,
         lambda r, v: r * r / abs(mp.expm1(r)) if r else mp.mpf(0), "relative to e^r - 1"),
    ]
    for name, f, (a, b), n, weight, what in specs:
        c = fit_rounded(f, a, b, n, weight)
        err = max_error(f, c, a, b, weight)
        print("// %s: degree %d on [%s, %s], max error %.3f x 2^-53 (%s)" %
              (name, n, mp.nstr(a, 6), mp.nstr(b, 6), err, what))
        for j, cj in enumerate(c):
            print("constexpr double k%s%d = %s;  // %.17g" % (name, j, cj.hex(), cj))


if __name__ == "__main__":
    main()
