"""Coefficients of the polynomial that the single-precision attenuation moments
use (moments_single in fs_point.hpp).

P(r) = sum_{j>=0} r^j / (j+3)!  (so that e^r = 1 + r + r^2/2 + r^3 P(r)) on
|r| <= ln2/2, the range left by the reduction of the exponent, approximated by
its degree-6 interpolant at the 7 Chebyshev nodes of that interval (near the
best uniform approximation; the error is printed).  Run as a script to print
the coefficients, lowest degree first, as they appear in the source.
"""
from math import factorial, log

import numpy as np

DEGREE = 6
HALF_RANGE = log(2.0) / 2.0


def p_exact(r):
    """P(r) from 30 terms of its series (exact to double rounding for |r| <= 1)."""
    r = np.asarray(r, dtype=np.float64)
    s = np.zeros_like(r)
    for j in range(30, -1, -1):
        s = s * r + 1.0 / factorial(j + 3)
    return s


def coefficients(degree: int = DEGREE, a: float = HALF_RANGE):
    """Monomial coefficients c_0..c_degree of the Chebyshev interpolant of P on [-a, a]."""
    k = np.arange(degree + 1)
    t = np.cos((2 * k + 1) * np.pi / (2 * (degree + 1)))  # Chebyshev nodes on [-1, 1]
    cheb = np.polynomial.chebyshev.Chebyshev.fit(t, p_exact(a * t), degree)
    mono = cheb.convert(kind=np.polynomial.Polynomial).coef  # in t = r / a
    return mono / a ** np.arange(degree + 1)


def horner(c, r):
    p = np.full_like(np.asarray(r, dtype=np.float64), c[-1])
    for ck in c[-2::-1]:
        p = p * r + ck
    return p


def max_rel_error(c, a: float = HALF_RANGE, n: int = 200001):
    r = np.linspace(-a * 1.0001, a * 1.0001, n)
    return float(np.max(np.abs(horner(c, r) / p_exact(r) - 1.0)))


if __name__ == "__main__":
    c = coefficients()
    for k, ck in enumerate(c):
        print(f"c{k} = {float(ck)!r}")
    print(f"max relative error on |r| <= 1.0001 ln2/2: {max_rel_error(c):.3e}")
