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


# --------------------------------------------------------------------------
# nearest-neighbour Lambda* on the spherical grid
# --------------------------------------------------------------------------
def _brute_force_sphere_stencil(orc, g, chi, n_mu, n_phi, op):
    """The stencil from its definition, one point at a time: for every
    characteristic and every point u, the formal solution of operator op with
    a unit source at that single point (ray_op) gives dI_m/dS(point u) at the
    points m = u-1 .. u+3; where u's voxel is an index neighbour of m's, it is
    added to that component of m's voxel with the voxel-average weight."""
    dirs, w = _dirs(orc, n_mu, n_phi)
    nv = g.n_vox
    out = np.zeros((27, nv))
    chi = np.asarray(chi, dtype=np.float64).ravel()
    for n3, wd in zip(dirs, w):
        num = np.zeros((27, nv))
        den = np.zeros(nv)
        for ch in g.rays(n3):
            vox, s, _ = g.segments(ch, n3)
            M = vox.size
            if M == 0:
                continue
            tau = chi[vox] * s
            np.add.at(den, vox, s)
            rt = [(v % g.Nr, (v // g.Nr) % g.Nt, v // (g.Nr * g.Nt)) for v in vox]
            for u in range(M):
                e = np.zeros(M)
                e[u] = 1.0
                I = orc.ray_op(tau, e, 0.0, op)
                for m in range(max(u - 1, 0), min(u + 4, M)):
                    dr, dt = rt[u][0] - rt[m][0], rt[u][1] - rt[m][1]
                    dp = (rt[u][2] - rt[m][2]) % g.Np
                    dp = -1 if dp == g.Np - 1 else dp
                    if abs(dr) > 1 or abs(dt) > 1 or abs(dp) > 1:
                        continue
                    num[(dp + 1) * 9 + (dt + 1) * 3 + (dr + 1), vox[m]] += s[m] * I[m]
        ok = den > 0
        out[:, ok] += wd * num[:, ok] / den[ok]
    return out.reshape(27, g.Np, g.Nt, g.Nr)


@pytest.mark.parametrize("op", ["linear", "parabolic"])
def test_sphere_stencil_equals_the_per_point_definition(orc, op):
    g = orc.SphereGrid(3, 4, 6, 1.0, 2.0)
    chi = np.random.default_rng(5).uniform(0.3, 3.0, g.n_vox)
    st = orc.lstar_stencil_sphere(g, 2, 4, chi, op)
    ref = _brute_force_sphere_stencil(orc, g, chi, 2, 4, op)
    np.testing.assert_allclose(st, ref, rtol=1e-12, atol=1e-15)


def test_sphere_linear_stencil_is_a_nonnegative_substochastic_part_holding_the_diagonal(orc):
    """Linear operator: every element is non-negative, each row sums to at
    most 1 (J of a unit source is at most 1), and the centre holds at least
    the diagonal Lambda* of the formal solution (points of the same voxel
    within the window add to it)."""
    g = orc.SphereGrid(5, 6, 8, 1.0, 2.5)
    chi = np.random.default_rng(6).uniform(0.1, 5.0, g.n_vox)
    st = orc.lstar_stencil_sphere(g, 4, 4, chi, "linear")
    _, L = orc.fs_sphere(g, 4, 4, chi, np.zeros(g.n_vox), np.zeros(g.n_vox), kind="linear")
    assert st.min() >= 0.0
    assert st.reshape(27, -1).sum(axis=0).max() <= 1.0 + 1e-12
    centre = st[13].ravel()
    assert np.all(centre >= L - 1e-14)
    assert np.mean(np.abs(centre - L) <= 1e-14 * np.maximum(L, 1e-300)) > 0.5  # mostly the diagonal itself


def test_sphere_nonlocal_ali_reaches_the_lu_fixed_point_in_fewer_steps(orc):
    from oracle import solvers as so
    g = orc.SphereGrid(4, 5, 6, 1.0, 2.5)
    rng = np.random.default_rng(7)
    chi = rng.uniform(0.5, 8.0, g.n_vox)
    eps = 10.0 ** rng.uniform(-4, -1, g.n_vox)
    prob = so.SphereProblem(g, chi, eps, 1.0, 0.0, 1.0, 2, 4)
    ref = so.direct(prob)
    L = prob.lstar_nonlocal()
    r_diag = so.ali(prob, tol=1e-12, max_iter=5000, ng=False)
    r_jac = so.ali(prob, tol=1e-12, max_iter=5000, ng=False, lstar=L, inner_jacobi=6)
    r_gs = so.ali(prob, tol=1e-12, max_iter=5000, ng=False, lstar=L, inner_gs=6)
    for r in (r_diag, r_jac, r_gs):
        assert r["converged"]
        np.testing.assert_allclose(r["J"], ref["J"], rtol=1e-9)
    print("steps diagonal", r_diag["iters"], "Jacobi", r_jac["iters"], "Gauss-Seidel", r_gs["iters"])
    assert r_jac["iters"] < r_diag["iters"] and r_gs["iters"] <= r_jac["iters"]


@pytest.mark.parametrize("shape", [(6, 4, 3), (7, 5, 4), (3, 3, 3)])
def test_sphere_os_colours_separate_every_stencil_neighbour(shape):
    """phi (axis 0) periodic, theta and r bounded."""
    from oracle import solvers as so
    Np, Nt, Nr = shape
    col = so.os_colours(shape, (True, False, False))
    for p in range(Np):
        for t in range(Nt):
            for r in range(Nr):
                for dp in (-1, 0, 1):
                    for dt in (-1, 0, 1):
                        for dr in (-1, 0, 1):
                            if not (0 <= t + dt < Nt and 0 <= r + dr < Nr):
                                continue
                            u = ((p + dp) % Np, t + dt, r + dr)
                            if u != (p, t, r):
                                assert col[u] != col[p, t, r]
