"""Pins of the oracle against closed forms, identities and brute force (CPU only).

Every check here is fixed by mathematics or by a statement of the paper, not by
the oracle itself, and together they are meant to catch a dropped term, a
wrong sign, a wrong index or a transposed operand anywhere in the oracle.
"""
import math

import mpmath
import numpy as np
import pytest

import synthetic as sy

mpmath.mp.dps = 40


def _moments_mp(D):
    D = mpmath.mpf(D)
    e0 = 1 - mpmath.exp(-D)
    e1 = mpmath.quad(lambda t: t * mpmath.exp(-(D - t)), [0, D])
    e2 = mpmath.quad(lambda t: t * t * mpmath.exp(-(D - t)), [0, D])
    return e0, e1, e2


# ---------------------------------------------------------------------------
# kernel moments and interpolation weights (Listing 1, steps 3-5)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("D", [1e-9, 1e-5, 1e-3, 0.05, 0.2, 0.2499, 0.25, 0.7, 3.0, 30.0, 700.0])
def test_moments_against_high_precision_quadrature(orc, D):
    e0, e1, e2 = orc.moments(D)
    m0, m1, m2 = _moments_mp(D)
    for got, ref in ((e0, m0), (e1, m1), (e2, m2)):
        assert abs(got - float(ref)) <= 2e-14 * abs(float(ref)) + 1e-300


def test_series_and_closed_form_agree_where_both_are_accurate(orc):
    # both branches evaluated on [0.05, 0.5]: series through D^17 vs closed form
    for D in np.linspace(0.05, 0.5, 37):
        m0, m1, m2 = _moments_mp(D)
        e1_closed = D - (-math.expm1(-D))
        e2_closed = D * D - 2.0 * e1_closed
        e0, e1, e2 = orc.moments(D)
        assert abs(e1 - e1_closed) <= 1e-12 * abs(float(m1))
        assert abs(e2 - e2_closed) <= 1e-11 * abs(float(m2))


def _segment_integral(D, Dp, f):
    """integral_0^D f(t) exp(-(D-t)) dt in high precision."""
    D = mpmath.mpf(D)
    return float(mpmath.quad(lambda t: f(t) * mpmath.exp(-(D - t)), [0, D]))


@pytest.mark.parametrize("D,Dp", [(0.01, 0.013), (0.3, 0.2), (1.0, 1.0), (2.5, 4.0), (0.1, 0.06), (7.0, 9.0)])
def test_parabolic_weights_integrate_quadratics_exactly(orc, D, Dp):
    a, b, g, lin = orc.weights(D, Dp, last=False)
    assert not lin
    for f in (lambda t: 1.0 + 0 * t, lambda t: t, lambda t: t * t, lambda t: 0.3 - 2 * t + 1.7 * t * t):
        S0, S1, S2 = f(0.0), f(D), f(D + Dp)
        got = a * S0 + b * S1 + g * S2
        ref = _segment_integral(D, Dp, f)
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)) * max(1.0, D * D)


@pytest.mark.parametrize("D", [1e-4, 0.1, 1.0, 6.0])
def test_linear_weights_integrate_lines_exactly(orc, D):
    a, b, g, lin = orc.weights(D, 0.0, last=True)
    assert lin and g == 0.0
    for f in (lambda t: 1.0 + 0 * t, lambda t: 0.4 + 3.0 * t):
        got = a * f(0.0) + b * f(D)
        ref = _segment_integral(D, 0.0, f)
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))


def test_weight_identities_and_signs(orc):
    Ds = np.logspace(-6, 4, 41)
    for D in Ds:
        e0 = -math.expm1(-D)
        for Dp in Ds:
            a, b, g, lin = orc.weights(D, Dp, last=False)
            assert abs(a + b + g - e0) <= 1e-13 * max(e0, 1e-300) + 1e-15 * D
            assert a >= 0.0 and b >= 0.0 and g <= 0.0
            assert b < 1.0


def test_fallback_rule(orc):
    # (ii) downwind step less than half the upwind step -> linear
    assert orc.weights(1.0, 0.49, False)[3]
    assert not orc.weights(1.0, 0.51, False)[3]
    # (iii) D' <= D coth(D/2) - 2, which is exactly where the parabolic beta reaches 1
    for D in (4.0, 6.0, 10.0, 40.0):
        lim = float(D * mpmath.coth(mpmath.mpf(D) / 2) - 2)
        assert abs(orc.beta_limit(D) - lim) <= 1e-13 * lim
        assert orc.weights(D, lim * (1 - 1e-9), False)[3]
        Dp = lim * (1 + 1e-6)
        a, b, g, lin = orc.weights(D, Dp, False)
        assert not lin and b < 1.0
        # beta evaluated from the parabolic formula just inside the limit would exceed 1
        e0, e1, e2 = orc.moments(D)
        Din = lim * (1 - 1e-6)
        b_par = ((D + Din) * e1 - e2) / (D * Din)
        assert b_par > 1.0
    for D in (1e-3, 0.05, 0.099, 0.1, 0.101, 0.5):
        lim = float(D * mpmath.coth(mpmath.mpf(D) / 2) - 2)
        assert abs(orc.beta_limit(D) - lim) <= 1e-12 * lim
    # last point of a ray has no downwind point
    assert orc.weights(1.0, 1.0, True)[3]
    # vacuum segment: no change of I
    assert orc.weights(0.0, 1.0, False)[:3] == (0.0, 0.0, 0.0)


def test_local_diagonal_between_zero_and_one(orc):
    """d_m = beta_m + gamma_{m-1} exp(-D_{m-1}) lies in (0,1) for any three steps."""
    Ds = np.logspace(-6, 4, 23)
    lo, hi = 1.0, 0.0
    for D0 in Ds:
        for D in Ds:
            _, _, g0, _ = orc.weights(D0, D, False)
            for Dp in Ds:
                _, b, _, _ = orc.weights(D, Dp, False)
                d = b + g0 * math.exp(-D)
                lo, hi = min(lo, d), max(hi, d)
    assert 0.0 < lo and hi < 1.0


# ---------------------------------------------------------------------------
# one characteristic: closed-form solutions of the transfer equation
# ---------------------------------------------------------------------------
def _random_taus(rng, M):
    return 10.0 ** rng.uniform(-3, 1.5, size=M)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ray_homogeneous_source(orc, seed):
    """Constant S: I = S (1 - e^-tau) + I_bc e^-tau at every point, any steps."""
    rng = np.random.default_rng(seed)
    M = 60
    tau = _random_taus(rng, M)
    S = np.full(M, 0.8)
    I_bc = 0.3
    I, _ = orc.ray(tau, S, I_bc)
    t_at = np.cumsum(tau) - 0.5 * tau  # optical depth of each midpoint
    ref = 0.8 * (-np.expm1(-t_at)) + I_bc * np.exp(-t_at)
    np.testing.assert_allclose(I, ref, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("seed", [3, 4])
def test_ray_source_linear_in_depth(orc, seed):
    """S = a + b t (t from P_1): I(t) = I1 e^-t + a(1-e^-t) + b(t-1+e^-t)."""
    rng = np.random.default_rng(seed)
    M = 50
    tau = _random_taus(rng, M)
    tmid = np.cumsum(tau) - 0.5 * tau
    t = tmid - tmid[0]
    a, b = 0.2, 0.7
    S = a + b * t
    I, _ = orc.ray(tau, S, 0.0)
    ref = I[0] * np.exp(-t) + a * (-np.expm1(-t)) + b * (t + np.expm1(-t))
    np.testing.assert_allclose(I, ref, rtol=1e-12, atol=1e-14)


def test_ray_quadratic_source_equal_steps(orc):
    """Equal steps never trigger the fallback: quadratics are integrated exactly
    except on the last segment (linear there by definition)."""
    M = 40
    for step in (0.05, 0.5, 2.0):
        tau = np.full(M, step)
        tmid = np.cumsum(tau) - 0.5 * tau
        t = tmid - tmid[0]
        c0, c1, c2 = 0.5, -0.1, 0.03
        S = c0 + c1 * t + c2 * t * t
        I, _ = orc.ray(tau, S, 0.0)
        # exact: I(t) = I1 e^-t + int_0^t S(u) e^-(t-u) du
        ref = I[0] * np.exp(-t) + c0 * (-np.expm1(-t)) + c1 * (t + np.expm1(-t)) \
            + c2 * (t * t - 2 * t + 2 * (1 - np.exp(-t)))
        np.testing.assert_allclose(I[:-1], ref[:-1], rtol=1e-11, atol=1e-13)


def test_ray_local_diagonal_is_derivative(orc):
    """d_m (parabolic) = dI_m/dS_m by finite differences of the linear map."""
    rng = np.random.default_rng(7)
    M = 30
    tau = _random_taus(rng, M)
    S = rng.uniform(0.1, 1.0, M)
    I0, d = orc.ray(tau, S, 0.4, kind="parabolic")
    for m in range(M):
        e = np.zeros(M); e[m] = 1.0
        I1, _ = orc.ray(tau, S + e, 0.4, kind="parabolic")
        assert abs((I1[m] - I0[m]) - d[m]) <= 1e-12
    # linear kind: e1/D of the upwind step (first point 1-e^{-D0})
    _, dl = orc.ray(tau, S, 0.4, kind="linear")
    assert abs(dl[0] + math.expm1(-0.5 * tau[0])) < 1e-15
    for m in range(1, M):
        D = 0.5 * (tau[m - 1] + tau[m])
        e0, e1, _ = orc.moments(D)
        assert abs(dl[m] - e1 / D) <= 1e-15


# ---------------------------------------------------------------------------
# tracker
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("Nz,n_mu,n_phi", [(9, 4, 8), (13, 8, 16), (33, 8, 16)])
def test_tracker_invariants(orc, Nz, n_mu, n_phi):
    mu, phi, _ = orc.quadrature(n_mu, n_phi)
    for d in range(mu.size):
        t = orc.box_template(Nz, mu[d], phi[d])
        n3 = orc.direction_vector(mu[d], phi[d])
        s, t0 = t["s"], t["t0"]
        # total length = Nz / |mu|, segments contiguous and positive
        assert abs(s.sum() - Nz / abs(mu[d])) <= 1e-12 * Nz / abs(mu[d])
        assert np.all(s > 0)
        np.testing.assert_allclose(t0[1:], t0[:-1] + s[:-1], rtol=1e-14, atol=0)
        # every segment midpoint lies in the voxel it is assigned to
        tm = t0 + 0.5 * s
        assert np.all(np.abs(n3[0] * tm - t["di"]) <= 0.5)
        assert np.all(np.abs(n3[1] * tm - t["dj"]) <= 0.5)
        depth = np.abs(n3[2]) * tm
        layer_from_top = t["kk"] if mu[d] < 0 else Nz - 1 - t["kk"]
        assert np.all((depth >= layer_from_top) & (depth <= layer_from_top + 1))
        # consecutive voxels share a face, edge or corner (unit steps)
        steps = np.abs(np.diff(np.stack([t["di"], t["dj"], t["kk"]]), axis=1))
        assert np.all(steps.max(axis=0) == 1)


@pytest.mark.parametrize("Nx,Ny,Nz,n_mu,n_phi", [(5, 7, 6, 4, 8), (9, 9, 9, 4, 8)])
def test_tracker_path_length_per_voxel(orc, Nx, Ny, Nz, n_mu, n_phi):
    """Summed over all rays of one direction, every voxel holds exactly 1/|mu| of path."""
    mu, phi, _ = orc.quadrature(n_mu, n_phi)
    for d in range(mu.size):
        t = orc.box_template(Nz, mu[d], phi[d])
        acc = np.zeros((Nz, Ny, Nx))
        for y0 in range(Ny):
            for x0 in range(Nx):
                np.add.at(acc, (t["kk"], (y0 + t["dj"]) % Ny, (x0 + t["di"]) % Nx), t["s"])
        np.testing.assert_allclose(acc, 1.0 / abs(mu[d]), rtol=1e-12)


def test_tracker_brute_force_rays(orc):
    """Rays traced from every inflow-face centre in absolute coordinates are the
    translates of the column-(0,0) template (voxel by voxel, lengths to 1e-13)."""
    Nz, Nx = 6, 5
    mu, phi, _ = orc.quadrature(4, 8)
    for d in (0, 3, 13, 22, 31):
        n3 = orc.direction_vector(mu[d], phi[d])
        tpl = orc.box_template(Nz, mu[d], phi[d])
        for x0 in range(Nx):
            # brute force: sample the straight line densely, find where the voxel changes
            L = Nz / abs(n3[2])
            ts = np.linspace(0.0, L, 400001)[1:-1]
            ix = np.floor(x0 + n3[0] * ts + 0.5).astype(int)
            iy = np.floor(0.0 + n3[1] * ts + 0.5).astype(int)
            dep = np.abs(n3[2]) * ts
            iz = np.floor(dep).astype(int)
            key = np.stack([ix, iy, iz])
            change = np.any(np.diff(key, axis=1) != 0, axis=0)
            starts = np.concatenate([[0], np.nonzero(change)[0] + 1])
            seq = key[:, starts]
            exp_seq = np.stack([x0 + tpl["di"], tpl["dj"],
                                tpl["kk"] if mu[d] < 0 else Nz - 1 - tpl["kk"]])
            assert seq.shape == exp_seq.shape
            np.testing.assert_array_equal(seq, exp_seq)
            lens = np.diff(np.concatenate([ts[starts], [L]]))
            np.testing.assert_allclose(lens, tpl["s"], atol=3 * L / 400000)


# ---------------------------------------------------------------------------
# formal solution on the box
# ---------------------------------------------------------------------------
def test_box_constant_source_closed_form(orc):
    """eps = 1, constant S and chi: J_v = sum_d w_d sum s_m [S(1-e^{-chi l_m}) + I_bc e^{-chi l_m}] / sum s_m
    with l_m the distance of point m from the entry point."""
    Nx, Ny, Nz, n_mu, n_phi = 6, 5, 7, 4, 8
    chi0, S0, It, Ib = 0.37, 0.6, 0.1, 1.3
    chi = np.full((Nz, Ny, Nx), chi0)
    J, _ = orc.fs_box(chi, np.full_like(chi, S0), It, Ib, n_mu, n_phi)
    mu, phi, w = orc.quadrature(n_mu, n_phi)
    Jref = np.zeros(Nz)
    for d in range(mu.size):
        t = orc.box_template(Nz, mu[d], phi[d])
        l = t["t0"] + 0.5 * t["s"]
        Ibc = It if mu[d] < 0 else Ib
        I = S0 * (-np.expm1(-chi0 * l)) + Ibc * np.exp(-chi0 * l)
        num = np.bincount(t["kk"], t["s"] * I, Nz)
        den = np.bincount(t["kk"], t["s"], Nz)
        Jref += w[d] * num / den
    np.testing.assert_allclose(J, np.broadcast_to(Jref[:, None, None], J.shape), rtol=1e-13)


def test_box_opacity_limits(orc):
    Nx, Ny, Nz = 5, 5, 5
    S = np.full((Nz, Ny, Nx), 0.7)
    Jthick, Lthick = orc.fs_box(np.full_like(S, 1e6), S, 0.0, 0.0, 4, 8, kind="parabolic")
    np.testing.assert_allclose(Jthick, 0.7, rtol=1e-5)   # chi -> infinity: J -> S
    assert np.all(Lthick > 1 - 1e-5) and np.all(Lthick < 1)
    Jthin, Lthin = orc.fs_box(np.full_like(S, 1e-9), S, 0.0, 0.0, 4, 8, kind="parabolic")
    assert np.all(np.abs(Jthin) < 1e-7) and np.all(Lthin < 1e-7) and np.all(Lthin > 0)


def test_box_xy_homogeneous_equals_layer_reduction(orc):
    """x,y-uniform fields: J does not depend on (x,y) and equals the template-ray reduction."""
    Nz = 17
    chi_k = sy.stratified_chi(Nz, 1e-3, 1e3)
    S_k = np.linspace(0.2, 1.0, Nz) ** 2
    for Nx, Ny in ((7, 7), (9, 6)):
        chi = np.broadcast_to(chi_k[:, None, None], (Nz, Ny, Nx)).copy()
        S = np.broadcast_to(S_k[:, None, None], (Nz, Ny, Nx)).copy()
        for kind in ("linear", "parabolic"):
            J, L = orc.fs_box(chi, S, 0.2, 1.0, 4, 8, kind=kind)
            J1, L1 = orc.fs_1d(chi_k, S_k, 0.2, 1.0, 4, 8, kind=kind)
            np.testing.assert_allclose(J, np.broadcast_to(J1[:, None, None], J.shape), rtol=1e-13)
            np.testing.assert_allclose(L, np.broadcast_to(L1[:, None, None], L.shape), rtol=1e-13)


def _tiny_box(seed=5):
    case = sy.random_box(7, 7, 5, 4, 8, seed=seed, dtype="f64")
    return case


def test_lstar_parabolic_is_exact_diagonal_of_lambda(orc):
    """Lambda* built in the sweep equals diag(Lambda) from unit-source formal solutions."""
    c = _tiny_box()
    chi = c.chi[0]
    prob = orc.BoxProblem(chi, c.eps[0], c.B[0], 0.0, 0.0, c.n_mu, c.n_phi, kind="parabolic")
    Lam, _ = orc.lambda_matrix(prob)
    Lst = prob.lstar()
    np.testing.assert_allclose(Lst.ravel(), np.diag(Lam), rtol=1e-12, atol=1e-15)
    assert np.all(Lst > 0) and np.all(Lst < 1)
    # linear-weight diagonal: also strictly inside (0,1)
    p2 = orc.BoxProblem(chi, c.eps[0], c.B[0], 0.0, 0.0, c.n_mu, c.n_phi, kind="linear")
    L2 = p2.lstar()
    assert np.all(L2 > 0) and np.all(L2 < 1)


def test_sampled_formal_solution_matches_full(orc):
    c = sy.random_box(8, 6, 7, 4, 8, seed=11, dtype="f64")
    chi = c.chi[0]
    S = sy.random_source(chi.shape, seed=12)
    J, L = orc.fs_box(chi, S, 0.3, 1.1, 4, 8, kind="parabolic")
    vox = np.array([0, 5, 17, 100, 200, chi.size - 1])
    Js, Ls = orc.fs_box_sampled(chi, S, 0.3, 1.1, 4, 8, vox, kind="parabolic")
    np.testing.assert_allclose(Js, J.ravel()[vox], rtol=1e-13)
    np.testing.assert_allclose(Ls, L.ravel()[vox], rtol=1e-13)


def test_lambda_linear_in_source(orc):
    c = sy.random_box(6, 6, 6, 4, 8, seed=21, dtype="f64")
    chi = c.chi[0]
    S1 = sy.random_source(chi.shape, 1)
    S2 = sy.random_source(chi.shape, 2)
    J1, _ = orc.fs_box(chi, S1, 0.0, 0.0, 4, 8)
    J2, _ = orc.fs_box(chi, S2, 0.0, 0.0, 4, 8)
    J12, _ = orc.fs_box(chi, 2.0 * S1 - 0.5 * S2, 0.0, 0.0, 4, 8)
    np.testing.assert_allclose(J12, 2.0 * J1 - 0.5 * J2, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# operator splitting and its fixed point (Sec. 2.2)
# ---------------------------------------------------------------------------
def test_solvers_reach_the_lu_fixed_point(orc):
    c = _tiny_box(seed=31)
    prob = orc.BoxProblem(c.chi[0], c.eps[0], c.B[0], c.I_bc[0, 0], c.I_bc[0, 1], c.n_mu, c.n_phi)
    ref = orc.direct(prob)
    Lam, Jbc = ref["Lam"], ref["Jbc"]
    # Jacobi ALI with the diagonal Lambda*, with and without Ng
    for ng in (False, True):
        r = orc.ali(prob, tol=1e-13, ng=ng, max_iter=4000)
        assert r["converged"]
        np.testing.assert_allclose(r["J"], ref["J"], rtol=1e-10)
    # Lambda* = 0 is plain Lambda iteration: same fixed point (eps here is not small)
    r0 = orc.ali(prob, tol=1e-13, ng=False, lstar=np.zeros(prob.shape), max_iter=20000)
    np.testing.assert_allclose(r0["J"], ref["J"], rtol=1e-9)
    # Lambda* = Lambda: a direct solution, converged after the first update (Sec. 2.2)
    rfull = orc.ali(prob, tol=1e-12, ng=False, lstar=Lam, max_iter=3, record=True)
    np.testing.assert_allclose(rfull["J"], ref["J"], rtol=1e-11)
    assert rfull["iters"] <= 2
    # BiCGStab (Sec. 4)
    rb = orc.bicgstab(prob, rtol=1e-13)
    np.testing.assert_allclose(rb["J"], ref["J"], rtol=1e-10)
    # the fixed point satisfies J = Lambda S + Lambda_bc, S = (1-eps) J + eps B
    S = ref["S"].ravel()
    np.testing.assert_allclose(Lam @ S + Jbc, ref["J"].ravel(), rtol=1e-12)


def test_ng_extrapolation_exact_for_two_mode_linear_iteration(orc):
    """A linear iteration whose error has two eigen-components is solved exactly by Ng-2."""
    rng = np.random.default_rng(0)
    n = 50
    xstar = rng.uniform(1, 2, n)
    v1, v2 = rng.standard_normal(n), rng.standard_normal(n)
    xs = [xstar + 0.3 * 0.9 ** k * v1 + 0.2 * (-0.5) ** k * v2 for k in range(4)]
    x = orc.ng_extrapolate(xs[3], xs[2], xs[1], xs[0])
    np.testing.assert_allclose(x, xstar, rtol=1e-10)


@pytest.mark.parametrize("T", [10.0, 100.0, 1000.0])
def test_lambda_iteration_amplification(orc, T):
    """Largest eigenvalue of the Lambda-iteration amplification ~ (1-eps)(1-1/T) (Sec. 2.2)."""
    eps = 1e-3
    Nz = 65
    prob = orc.Plane1DProblem(np.full(Nz, T / Nz), eps, 1.0, 0.0, 0.0, 8, 4)
    lam = orc.lambda_iteration_radius(prob, n_iter=300)
    approx = (1 - eps) * (1 - 1 / T)
    assert abs(lam - approx) <= 0.1 * approx
    assert lam < 1 - eps


def _pp_fs(orc, chi, S, Itop, Ibot, n_mu):
    """Plane-parallel reduction of the characteristic integrator: one point per layer."""
    mu, _, w = orc.quadrature(n_mu, 1)
    J = np.zeros(len(chi))
    Is = []
    for m, ww in zip(mu, w):
        if m < 0:
            I, _ = orc.ray(chi / abs(m), S, Itop)
        else:
            I, _ = orc.ray((chi / abs(m))[::-1], S[::-1], Ibot)
            I = I[::-1]
        J += ww * I
        Is.append(I)
    return J, mu, w, np.array(Is)


def _pp_solve(orc, chi, eps, Itop, Ibot, n_mu, B=1.0):
    Nz = len(chi)
    L = np.zeros((Nz, Nz))
    for j in range(Nz):
        e = np.zeros(Nz); e[j] = 1.0
        L[:, j] = _pp_fs(orc, chi, e, 0.0, 0.0, n_mu)[0]
    Jbc = _pp_fs(orc, chi, np.zeros(Nz), Itop, Ibot, n_mu)[0]
    S = np.linalg.solve(np.eye(Nz) - (1 - eps) * L, (1 - eps) * Jbc + eps * B)
    return S


def test_sqrt_eps_surface_law(orc):
    """Semi-infinite atmosphere, constant eps and B, isotropic scattering: S(0) = sqrt(eps) B.
    Checked on the plane-parallel reduction (129 layers, tau 1e-4..1e3, eps = 1e-2)."""
    chi = sy.stratified_chi(129, 1e-4, 1e3)
    S = _pp_solve(orc, chi, 1e-2, 0.0, 1.0, 8)
    assert abs(S[0] / 0.1 - 1.0) < 1e-3


def test_pure_scattering_flux_conservation(orc):
    """eps = 0: the flux H = sum w mu I is constant with depth in a slab (interior layers;
    the two boundary layers use the constant-S entry half-step)."""
    Nz = 129
    chi = sy.stratified_chi(Nz, 1e-3, 1e2)
    S = _pp_solve(orc, chi, 0.0, 0.0, 1.0, 8)
    _, mu, w, Is = _pp_fs(orc, chi, S, 0.0, 1.0, 8)
    H = (w[:, None] * mu[:, None] * Is).sum(axis=0)
    Hi = H[1:-1]
    assert abs(Hi.max() - Hi.min()) <= 1e-3 * abs(Hi).max()


def _slab_fixed_point(orc, Nz, tau_range, eps, n_mu, n_phi):
    """Fixed point of the x,y-homogeneous box (the 3D voxel operator reduced to
    its layers, orc_fs_1d) by LU: no light entering at the top, I = B = 1 at
    the bottom."""
    chi = sy.stratified_chi(Nz, *tau_range)
    prob = orc.Plane1DProblem(chi, eps, 1.0, 0.0, 1.0, n_mu, n_phi)
    return chi, orc.direct(prob)


def test_sqrt_eps_surface_law_of_the_voxel_operator_under_refinement(orc):
    """S(0) = sqrt(eps) B on the 3D voxel operator of an x,y-homogeneous box
    (8 x 16 directions, tau 1e-4..1e4, eps = 1e-2).  A shallow characteristic
    crosses each layer in several segments whose lengths depend on where the
    vertical and horizontal planes fall, so the surface error scatters by a
    few times between neighbouring resolutions; its trend falls as about
    Nz^-1.7 (measured: 1.3e-1 at 33 layers, 3.0e-2 at 65, 1.9e-3 at 129,
    5.8e-3 at 257, 1.6e-3 at 385; least-squares slope -1.65).  Pinned: a least-squares slope of
    log|error| against log Nz below -1.2, and errors below 1e-2 from 129
    layers on."""
    Ns = [33, 65, 129, 257, 385]
    errs = []
    for Nz in Ns:
        _, r = _slab_fixed_point(orc, Nz, (1e-4, 1e4), 1e-2, 8, 16)
        errs.append(abs(r["S"][0] / 0.1 - 1.0))
    slope = np.polyfit(np.log(Ns), np.log(errs), 1)[0]
    print("sqrt(eps) law errors", dict(zip(Ns, errs)), "slope", slope)
    assert slope < -1.2
    assert max(errs[2:]) < 1e-2
    assert errs[0] > 10 * min(errs[2:])


def test_pure_scattering_flux_conservation_of_the_voxel_operator(orc):
    """eps = 0 on the x,y-homogeneous box: the flux H = sum_d w mu I_v(d) from
    the voxel-averaged directional intensities (orc_fs_1d_dirs) is constant
    with depth up to the voxels' optical thickness -- the mean intensity of a
    voxel is not a face flux once the voxel is thick (H drifts by tens of
    per cent across layers of dtau ~ 1..20).  Its spread across the layers
    thinner than dtau falls roughly as dtau^2 (measured 1e-2..3e-2 for
    dtau <= 0.3, 1e-3..3e-3 for <= 0.1, 1.5e-4..4.5e-4 for <= 0.03, at 33 to
    257 layers)."""
    n_mu, n_phi = 8, 16
    mu, _, w = orc.quadrature(n_mu, n_phi)
    for Nz in (65, 129):
        chi, r = _slab_fixed_point(orc, Nz, (1e-3, 1e2), 0.0, n_mu, n_phi)
        I = orc.fs_1d_dirs(chi, r["S"], 0.0, 1.0, n_mu, n_phi)
        H = (w[:, None] * mu[:, None] * I).sum(axis=0)
        spread = {}
        for thr in (0.3, 0.03):
            Hs = H[chi <= thr]
            spread[thr] = (Hs.max() - Hs.min()) / abs(Hs).max()
        print(Nz, spread)
        assert spread[0.03] < 6e-4
        assert spread[0.3] > 5 * spread[0.03]
        assert H.min() > 0.0


def test_fs_1d_dirs_is_the_angle_split_of_fs_1d(orc):
    """sum_d w_d I_v(d) of orc_fs_1d_dirs equals J of orc_fs_1d."""
    Nz, n_mu, n_phi = 23, 6, 8
    rng = np.random.default_rng(5)
    chi = 10.0 ** rng.uniform(-2, 1, Nz)
    S = rng.uniform(0.2, 1.5, Nz)
    J, _ = orc.fs_1d(chi, S, 0.3, 1.2, n_mu, n_phi)
    _, _, w = orc.quadrature(n_mu, n_phi)
    I = orc.fs_1d_dirs(chi, S, 0.3, 1.2, n_mu, n_phi)
    np.testing.assert_allclose((w[:, None] * I).sum(axis=0), J, rtol=1e-14)


def test_fs_box_dirs_subsets_sum_to_the_full_formal_solution(orc):
    """Disjoint direction subsets (the partial angle sums of a solid-angle
    split, Sec. 4) add up to the full J and Lambda*."""
    case = sy.random_box(9, 8, 6, 4, 8, seed=7, dtype="f64")
    S = sy.random_source(case.chi.shape, seed=8)[0]
    chi = case.chi[0]
    Jf, Lf = orc.fs_box(chi, S, 0.2, 1.1, 4, 8)
    rng = np.random.default_rng(9)
    part = rng.integers(0, 3, size=32)
    Js, Ls = np.zeros_like(Jf), np.zeros_like(Lf)
    for k in range(3):
        dirs = np.flatnonzero(part == k)
        J, L = orc.fs_box_dirs(chi, S, 0.2, 1.1, 4, 8, dirs, want_lstar=True)
        Js += J
        Ls += L
    np.testing.assert_allclose(Js, Jf, rtol=1e-14)
    np.testing.assert_allclose(Ls, Lf, rtol=1e-14)
