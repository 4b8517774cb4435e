"""The polynomial behind the single-precision attenuation moments (CPU only).

moments_single in paper_2102_01734_amd/csrc/fs_point.hpp evaluates, for every
optical step D, ex = exp(-D), e0 = 1 - ex, e1 = D - e0, e2 = D^2 - 2 e1 (the
moments of the formal solution's interpolation, Listing 1 steps 4-5) from one
polynomial P(r) = sum_j r^j/(j+3)! of the reduced argument.  Checked here: the
constants in the source are those the generator script computes, the
interpolant meets its stated error bound, and the kernel's sequence of
operations, replayed in double precision with correctly rounded FMAs, gives
moments within 1e-10 (e1, e2) and 1e-12 (ex, e0) of 40-digit values over
1e-12 <= D <= 745, the accuracy single-precision results need.
"""
import importlib.util
import math
import os
import re

import mpmath
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2102_01734_amd", "csrc")
mpmath.mp.dps = 40


def _gen():
    spec = importlib.util.spec_from_file_location("gen_moment_poly", os.path.join(CSRC, "gen_moment_poly.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _source_coefficients():
    src = open(os.path.join(CSRC, "fs_point.hpp")).read()
    body = src[src.index("void moments_single("):]
    body = body[:body.index("const double r2")]
    nums = re.findall(r"fma3\(\s*([0-9.e+-]+)\s*,\s*r\s*,\s*([0-9.e+-]+)\s*\)|fma3\(P,\s*r,\s*([0-9.e+-]+)\)", body)
    first = nums[0]
    coef = [float(first[0]), float(first[1])] + [float(n[2]) for n in nums[1:]]
    return coef[::-1]  # lowest degree first


def test_source_constants_are_the_generated_ones():
    g = _gen()
    assert _source_coefficients() == [float(c) for c in g.coefficients()]


def test_interpolant_error_bound():
    g = _gen()
    assert g.max_rel_error(g.coefficients()) < 2e-11


def _fma(a, b, c):
    return float(mpmath.mpf(a) * mpmath.mpf(b) + mpmath.mpf(c))


def _moments_single(D, c):
    """The kernel's operations in order (double precision, FMAs correctly rounded)."""
    x = max(-D, -745.0)
    n = float(np.rint(x * 1.4426950408889634))
    r = _fma(-n, 0.6931471805599453, x)
    P = _fma(c[6], r, c[5])
    for k in (4, 3, 2, 1, 0):
        P = _fma(P, r, c[k])
    r2 = r * r
    h = _fma(r, P, 0.5)
    if n == 0.0:
        u = r2 * h
        e1 = u
        e0 = D - u
        ex = 1.0 - e0
        e2 = (-2.0 * r2) * (r * P)
    else:
        ex = math.ldexp(_fma(r2, h, 1.0 + r), int(n))
        e0 = 1.0 - ex
        e1 = D - e0
        e2 = _fma(D, D, -2.0 * e1)
    return ex, e0, e1, e2


def _moments_mp(D):
    Dm = mpmath.mpf(D)
    ex = mpmath.exp(-Dm)
    e0 = -mpmath.expm1(-Dm)
    e1 = Dm - e0
    e2 = Dm * Dm - 2 * e1
    return ex, e0, e1, e2


_STEPS = sorted(set(np.concatenate([np.logspace(-12, math.log10(745.0), 61),
                                    [math.log(2) / 2 * f for f in (0.999, 1.0, 1.001)],
                                    [0.25, 1.0, 1.5, 2.0, 744.0]]).tolist()))


@pytest.mark.parametrize("D", _STEPS)
def test_moments_single_accuracy(D):
    c = [float(v) for v in _gen().coefficients()]
    got = _moments_single(D, c)
    ref = _moments_mp(D)
    for name, g, r, tol in zip(("ex", "e0", "e1", "e2"), got, ref, (1e-12, 1e-12, 1e-10, 1e-10)):
        r = float(r)
        assert abs(g - r) <= tol * abs(r) + 1e-300, (name, D, g, r)
