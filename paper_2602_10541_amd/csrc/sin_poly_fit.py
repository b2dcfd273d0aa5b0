"""Coefficients of the FP64 sine polynomial in flsq_device.h (sin_f64).

On the reduced interval |r| <= pi/2, sin r = r + r^3 g(r^2) with g(t) = (sin sqrt(t) - sqrt(t)) / t^(3/2).
g is fitted on [0, (pi/2)^2] by a degree-7 polynomial in the Chebyshev sense (mpmath.chebyfit at 50
digits: interpolation at Chebyshev nodes, near the minimax polynomial), and the coefficients are
rounded to double.  Run it to print the coefficients (highest degree first) and the errors: the
fit's own error is about 3.4e-19, below the format's rounding, and the largest error of the
polynomial evaluated in double (Horner in r^2, then r + (r r^2) p) over [0, pi/2] is about 1.9e-16,
the same as the Taylor series to r^21 that it replaces with two multiply-adds fewer.
"""
import math

import mpmath as mp


def fit(deg=7, dps=50):
    mp.mp.dps = dps
    t_hi = (mp.pi / 2) ** 2

    def g(t):
        if t == 0:
            return mp.mpf(-1) / 6
        r = mp.sqrt(t)
        return (mp.sin(r) - r) / (t * r)

    coef, err = mp.chebyfit(g, [0, t_hi], deg + 1, error=True)
    return [float(c) for c in coef], float(err)


def eval_double(coef, r):
    r2 = r * r
    p = coef[0]
    for c in coef[1:]:
        p = p * r2 + c
    return r + (r * r2) * p


if __name__ == "__main__":
    coef, err = fit()
    worst = 0.0
    for i in range(20001):
        r = (math.pi / 2) * i / 20000
        worst = max(worst, abs(float(mp.mpf(eval_double(coef, r)) - mp.sin(mp.mpf(r)))))
    print("fit error", err, "double evaluation error", worst)
    for c in coef:
        print(repr(c))
