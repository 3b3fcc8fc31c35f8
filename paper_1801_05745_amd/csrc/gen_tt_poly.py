"""Generates the polynomial used by the binning kernel for tt = 2 atan(u) / pi.

For |u| <= tan(pi/8) the kernel evaluates
    (2/pi) atan(u) = u * P(u^2),   P(s) = sum_k c_k s^k,  k = 0..DEG
with Horner's rule in FP64.  The coefficients interpolate f(s) = (2/pi) atan(sqrt(s))/sqrt(s)
at Chebyshev points of s in [0, tan(pi/8)^2] at 60-digit precision and are then
rounded to binary64.  The script checks the rounded polynomial against mpmath on
a dense grid and prints the coefficients and the observed maximum relative error
of u P(u^2) (excluding the FP64 evaluation rounding, which adds a few ulp).

Run: python gen_tt_poly.py   (prints C++ source for ring.hpp)
"""

import mpmath

DEG = 9
mpmath.mp.dps = 60


def coefficients(deg=DEG):
    a = mpmath.mpf(0)
    b = mpmath.tan(mpmath.pi / 8) ** 2
    two_over_pi = 2 / mpmath.pi

    def f(s):
        if s == 0:
            return two_over_pi
        r = mpmath.sqrt(s)
        return two_over_pi * mpmath.atan(r) / r

    n = deg + 1
    nodes = [(a + b) / 2 + (b - a) / 2 * mpmath.cos(mpmath.pi * (2 * k + 1) / (2 * n)) for k in range(n)]
    # solve the Vandermonde system in high precision (interpolation at Chebyshev nodes)
    A = mpmath.matrix([[s ** j for j in range(n)] for s in nodes])
    y = mpmath.matrix([f(s) for s in nodes])
    c = mpmath.lu_solve(A, y)
    return [float(c[j]) for j in range(n)]


def max_rel_error(cs, samples=20001):
    b = float(mpmath.tan(mpmath.pi / 8))
    worst = 0.0
    for i in range(1, samples):
        u = mpmath.mpf(b) * i / (samples - 1)
        s = u * u
        p = mpmath.mpf(0)
        for ck in reversed(cs):
            p = p * s + mpmath.mpf(ck)
        approx = u * p
        exact = 2 * mpmath.atan(u) / mpmath.pi
        worst = max(worst, float(abs(approx - exact) / exact))
    return worst


if __name__ == "__main__":
    cs = coefficients()
    err = max_rel_error(cs)
    print(f"// degree {DEG} in u^2, max relative error of u*P(u^2) before FP64 rounding: {err:.3e}")
    for k, v in enumerate(cs):
        print(f"    {v!r},  // c{k}")
