"""Pins of the oracle's spherical grid (CPU only).

Beyond these (closed forms given the traced geometry, coverage, symmetry and
the irradiation rule) the spherical discretisation has no independent
reference: its parity is unpinned otherwise.
"""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def grid(orc):
    return orc.SphereGrid(9, 8, 12, 1.0, 2.0)


def _dirs(orc, n_mu, n_phi):
    mu, phi, w = orc.quadrature(n_mu, n_phi)
    return [orc.direction_vector(m, p) for m, p in zip(mu, phi)], w


def test_characteristics_cover_every_voxel_and_chords_are_exact(orc, grid):
    ns, _ = _dirs(orc, 4, 8)
    for d in (0, 5, 17, 31):
        n = ns[d]
        chars = grid.rays(n)
        seen = np.zeros(grid.n_vox, bool)
        for c in chars:
            v, s, t0 = grid.segments(c, n)
            seen[v] = True
            assert np.all(s > 0)
            assert abs(s.sum() - (c[4] - c[3])) <= 1e-12 * (c[4] - c[3] + 1)
            # chord geometry: the characteristic starts on the outer sphere or on the core
            p = c[:3]
            assert abs(p @ n) < 1e-12
            x0 = p + c[3] * n
            r0 = np.linalg.norm(x0)
            assert abs(r0 - (grid.rc if c[5] == 1 else grid.ro)) < 1e-12
            # every segment midpoint lies in its voxel
            tm = c[3] + t0 + 0.5 * s
            x = p[None, :] + tm[:, None] * n[None, :]
            r = np.linalg.norm(x, axis=1)
            th = np.arccos(np.clip(x[:, 2] / r, -1, 1))
            ph = np.mod(np.arctan2(x[:, 1], x[:, 0]), 2 * np.pi)
            ir = v % grid.Nr
            it = (v // grid.Nr) % grid.Nt
            ip = v // (grid.Nr * grid.Nt)
            dr = (grid.ro - grid.rc) / grid.Nr
            assert np.all((r >= grid.rc + ir * dr - 1e-12) & (r <= grid.rc + (ir + 1) * dr + 1e-12))
            assert np.all((th >= it * np.pi / grid.Nt - 1e-12) & (th <= (it + 1) * np.pi / grid.Nt + 1e-12))
            assert np.all((ph >= ip * 2 * np.pi / grid.Np - 1e-12) & (ph <= (ip + 1) * 2 * np.pi / grid.Np + 1e-12))
        assert seen.all()


def test_constant_source_closed_form(orc, grid):
    """Constant S and chi: I at each point = S(1 - e^{-chi l}) + I_0 e^{-chi l} with l the
    distance from the characteristic's start (I_0 = outer intensity or core B)."""
    n_mu, n_phi = 4, 8
    chi0, S0, Iout, Bc = 0.8, 0.6, 0.15, 1.3
    nv = grid.n_vox
    J, _ = orc.fs_sphere(grid, n_mu, n_phi, np.full(nv, chi0), np.full(nv, S0), np.full(nv, Bc), I_out=Iout)
    ns, w = _dirs(orc, n_mu, n_phi)
    Jref = np.zeros(nv)
    for d, n in enumerate(ns):
        num = np.zeros(nv); den = np.zeros(nv)
        for c in grid.rays(n):
            v, s, t0 = grid.segments(c, n)
            l = t0 + 0.5 * s
            I0 = Bc if c[5] == 1 else Iout
            I = S0 * (-np.expm1(-chi0 * l)) + I0 * np.exp(-chi0 * l)
            np.add.at(num, v, s * I)
            np.add.at(den, v, s)
        Jref += w[d] * num / den
    np.testing.assert_allclose(J, Jref, rtol=1e-13)


def test_spherically_symmetric_input_gives_nearly_symmetric_J(orc):
    g = orc.SphereGrid(12, 10, 16, 1.0, 2.0)
    r = g.rc + (np.arange(g.Nr) + 0.5) * (g.ro - g.rc) / g.Nr
    chi_r = 3.0 / r ** 2
    S_r = 0.5 + 0.5 / r
    chi = np.tile(chi_r, g.Nt * g.Np)
    S = np.tile(S_r, g.Nt * g.Np)
    J, L = orc.fs_sphere(g, 8, 16, chi, S, np.ones(g.n_vox))
    Jr = J.reshape(g.Np, g.Nt, g.Nr)
    spread = (Jr.max(axis=(0, 1)) - Jr.min(axis=(0, 1))) / Jr.mean(axis=(0, 1))
    # discretisation-limited: the angular and ray-lattice sampling break the symmetry slightly
    assert spread.max() < 0.04
    assert np.all((L > 0) & (L < 1))


def test_irradiation_rule(orc):
    n_mu, n_phi, ro, dsrc = 4, 8, 2.0, 5.0
    # sub-source point: the light travels along -z; ties between the n_phi equal-mu
    # directions go to the lowest index, and J_inc = B there
    x = np.array([0.0, 0.0, ro])
    w = 1.0 / (n_mu * n_phi)
    got = [orc.sph_irradiation(n_mu, n_phi, d, x, ro, dsrc, 1.0) for d in range(n_mu * n_phi)]
    assert abs(got[0] * w - 1.0) < 1e-14 and all(g == 0.0 for g in got[1:])
    # the far side is not lit
    assert all(orc.sph_irradiation(n_mu, n_phi, d, -x, ro, dsrc) == 0.0 for d in range(n_mu * n_phi))
    # a point source at finite distance lights less than a hemisphere: the equator is dark
    assert all(orc.sph_irradiation(n_mu, n_phi, d, np.array([ro, 0.0, 0.0]), ro, dsrc) == 0.0
               for d in range(n_mu * n_phi))
    # inverse-square fall-off at 45 degrees from the sub-source point
    xl = ro * np.array([math.sqrt(0.5), 0.0, math.sqrt(0.5)])
    dist2 = float(np.sum((xl - np.array([0.0, 0.0, dsrc * ro])) ** 2))
    vals = [orc.sph_irradiation(n_mu, n_phi, d, xl, ro, dsrc) for d in range(n_mu * n_phi)]
    assert sum(v > 0 for v in vals) == 1
    # ... and it goes to the discrete direction closest to the light's direction
    ns, _ = _dirs(orc, n_mu, n_phi)
    u = (xl - np.array([0.0, 0.0, dsrc * ro])) / math.sqrt(dist2)
    assert int(np.argmax(vals)) == int(np.argmax([n @ u for n in ns]))
    assert abs(max(vals) * w - (ro * (dsrc - 1)) ** 2 / dist2) < 1e-14
