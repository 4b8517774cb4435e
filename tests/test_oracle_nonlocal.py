"""Pins of the oracle's nearest-neighbour Lambda* and of the ALI that uses it.

The stencil is computed per characteristic from the derivatives dI_m/dS of
the recurrence (oracle.lstar_stencil); these tests hold it against the plain
definition -- the elements Lambda_op[v][u] of the operator matrix, built
column by column from formal solutions of unit sources -- on grids whose
periods are longer than a characteristic's horizontal reach (so that no
characteristic wraps back into a neighbourhood), and against the diagonal
Lambda* and the direct (LU) fixed point.
"""
import numpy as np
import pytest

import oracle
import synthetic as sy
from oracle import solvers as so


def _columns(chi, n_mu, n_phi, op):
    N = chi.size
    Lam = np.zeros((N, N))
    for u in range(N):
        e = np.zeros(N)
        e[u] = 1.0
        Lam[:, u] = oracle.fs_box_op(chi, e.reshape(chi.shape), 0.0, 0.0, n_mu, n_phi, op).ravel()
    return Lam


@pytest.mark.parametrize("op", ["linear", "parabolic"])
@pytest.mark.parametrize("shape", [(11, 11, 2, 4, 8), (13, 12, 3, 2, 4)])
def test_stencil_equals_operator_elements(op, shape):
    Nx, Ny, Nz, n_mu, n_phi = shape
    case = sy.random_box(Nx, Ny, Nz, n_mu, n_phi, seed=3, dtype="f64")
    chi = case.chi[0]
    st = oracle.lstar_stencil(chi, n_mu, n_phi, op)
    Lam = _columns(chi, n_mu, n_phi, op)
    M = oracle.stencil_matrix(st).toarray()
    pattern = oracle.stencil_matrix(np.ones_like(st)).toarray() != 0
    np.testing.assert_allclose(M[pattern], Lam[pattern], rtol=1e-13, atol=1e-16)
    # no stencil element outside the 27-point neighbourhood
    assert np.all(M[~pattern] == 0)


@pytest.mark.parametrize("op", ["linear", "parabolic"])
def test_stencil_centre_is_the_diagonal_lstar(op):
    case = sy.random_box(9, 8, 6, 4, 8, seed=5, dtype="f64")
    chi = case.chi[0]
    st = oracle.lstar_stencil(chi, 4, 8, op)
    _, L = oracle.fs_box(chi, np.zeros_like(chi), 0.0, 0.0, 4, 8, kind=op)
    assert np.array_equal(st[13], L)


def test_parabolic_operator_is_the_formal_solution():
    case = sy.random_box(9, 8, 6, 4, 8, seed=6, dtype="f64")
    S = sy.random_source(case.chi.shape, seed=7)[0]
    J0, _ = oracle.fs_box(case.chi[0], S, 0.3, 0.7, 4, 8)
    J1 = oracle.fs_box_op(case.chi[0], S, 0.3, 0.7, 4, 8, "parabolic")
    # same per-point arithmetic; directions are summed in another order (per thread)
    np.testing.assert_allclose(J1, J0, rtol=1e-14)


def test_linear_operator_stencil_is_a_nonnegative_part_of_a_substochastic_row():
    """Linear-interpolation weights are non-negative, and Lambda_lin applied to
    S = 1 with no incoming radiation is at most 1: every stencil row is a
    non-negative part of that row."""
    case = sy.random_box(12, 11, 7, 4, 8, seed=8, dtype="f64")
    chi = case.chi[0]
    st = oracle.lstar_stencil(chi, 4, 8, "linear")
    row1 = oracle.fs_box_op(chi, np.ones_like(chi), 0.0, 0.0, 4, 8, "linear")
    assert st.min() >= 0.0
    assert np.all(st.sum(axis=0) <= row1 * (1 + 1e-13))
    assert row1.max() <= 1.0 + 1e-13


def test_no_elements_beyond_the_top_and_bottom_layers():
    case = sy.random_box(9, 9, 5, 4, 8, seed=9, dtype="f64")
    st = oracle.lstar_stencil(case.chi[0], 4, 8, "parabolic")
    for c in range(27):
        dz = c // 9 - 1
        if dz == -1:
            assert np.all(st[c][0] == 0)
        if dz == 1:
            assert np.all(st[c][-1] == 0)


def test_linear_ray_operator_matches_hand_recurrence():
    """One characteristic of the linear-interpolation operator against the
    recurrence written out: I_0 = I_bc e^-D0 + (1 - e^-D0) S_0 with D0 = tau_0/2,
    then I_m = I_{m-1} e^-D + (e0 - e1/D) S_{m-1} + (e1/D) S_m."""
    tau = np.array([0.3, 2.0, 0.01, 5.0, 0.7])
    S = np.array([1.0, 0.5, 2.0, 0.1, 1.5])
    I = oracle.ray_op(tau, S, 0.4, "linear")
    ref = np.zeros(5)
    D0 = tau[0] / 2
    ref[0] = 0.4 * np.exp(-D0) + (1 - np.exp(-D0)) * S[0]
    for m in range(1, 5):
        D = 0.5 * (tau[m - 1] + tau[m])
        e0 = 1 - np.exp(-D)
        e1 = D - e0
        ref[m] = ref[m - 1] * np.exp(-D) + (e0 - e1 / D) * S[m - 1] + (e1 / D) * S[m]
    np.testing.assert_allclose(I, ref, rtol=1e-12)


@pytest.mark.parametrize("op", ["linear", "parabolic"])
def test_nonlocal_ali_reaches_the_lu_fixed_point_in_fewer_steps(op):
    """Lambda* changes only the path: the non-local ALI (exact OS solve, and
    Jacobi sweeps) ends at the direct solution, in fewer steps than the
    diagonal one."""
    case = sy.random_box(7, 7, 5, 4, 8, seed=41, dtype="f64", eps_dex=(-4, -1))
    prob = so.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8, kind=op)
    ref = so.direct(prob)
    L = prob.lstar_nonlocal()
    r_diag = so.ali(prob, tol=1e-12, max_iter=5000, ng=False)
    r_nl = so.ali(prob, tol=1e-12, max_iter=5000, ng=False, lstar=L)
    r_jac = so.ali(prob, tol=1e-12, max_iter=5000, ng=False, lstar=L, inner_jacobi=6)
    for r in (r_diag, r_nl, r_jac):
        assert r["converged"]
        np.testing.assert_allclose(r["J"], ref["J"], rtol=1e-9)
    assert r_nl["iters"] < r_diag["iters"] and r_jac["iters"] < r_diag["iters"]


def test_many_jacobi_sweeps_equal_the_exact_os_solve():
    case = sy.random_box(7, 6, 5, 4, 8, seed=42, dtype="f64", eps_dex=(-3, 0))
    prob = so.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8)
    L = prob.lstar_nonlocal()
    a = so.ali(prob, tol=1e-30, max_iter=3, ng=False, lstar=L)
    b = so.ali(prob, tol=1e-30, max_iter=3, ng=False, lstar=L, inner_jacobi=400)
    np.testing.assert_allclose(b["J"], a["J"], rtol=1e-12)


def _os_system(Nx, Ny, Nz, n_mu, n_phi, op, seed, eps_dex=(-4, -1)):
    import scipy.sparse as sps
    case = sy.random_box(Nx, Ny, Nz, n_mu, n_phi, seed=seed, dtype="f64", eps_dex=eps_dex)
    L = oracle.stencil_matrix(oracle.lstar_stencil(case.chi[0], n_mu, n_phi, op))
    A = (sps.identity(L.shape[0], format="csr") - L @ sps.diags((1.0 - case.eps[0]).ravel())).tocsr()
    r = np.random.default_rng(seed).uniform(-1.0, 1.0, L.shape[0])
    return case, A, r


@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 4, 5), (3, 5, 4), (2, 7, 9), (5, 6, 6), (1, 3, 8), (4, 9, 3)])
def test_os_colours_separate_every_stencil_neighbour(shape):
    """No two distinct voxels that share a 27-point stencil coupling (x, y
    periodic, z not) have the same Gauss-Seidel colour; brute force over all
    voxel pairs of odd and even periods from 3 up."""
    Nz, Ny, Nx = shape
    col = so.os_colours(shape)
    assert col.min() >= 0 and col.max() < 18
    for k in range(Nz):
        for y in range(Ny):
            for x in range(Nx):
                for dz in (-1, 0, 1):
                    if not 0 <= k + dz < Nz:
                        continue
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            u = (k + dz, (y + dy) % Ny, (x + dx) % Nx)
                            if u != (k, y, x):
                                assert col[u] != col[k, y, x], (shape, (k, y, x), u)


@pytest.mark.parametrize("op", ["linear", "parabolic"])
def test_colour_gauss_seidel_is_the_sequential_sweep_in_colour_order(op):
    """The class-parallel sweep equals the textbook Gauss-Seidel sweep over
    single voxels, dense matrix, one voxel at a time in the order (colour,
    voxel index)."""
    case, A, r = _os_system(5, 4, 3, 2, 4, op, seed=61)
    shape = case.chi[0].shape
    col = so.os_colours(shape).ravel()
    Ad = A.toarray()
    order = sorted(range(r.size), key=lambda v: (col[v], v))
    x = r / np.diag(Ad)
    for sweeps in (1, 2):
        ref = x.copy()
        for _ in range(sweeps):
            for v in order:
                s = r[v]
                for u in range(r.size):
                    if u != v:
                        s -= Ad[v, u] * ref[u]
                ref[v] = s / Ad[v, v]
        got = so.gauss_seidel(A, r, x, col, sweeps)
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)


def test_gauss_seidel_converges_to_the_os_solution_faster_than_jacobi():
    """On the OS system of the linear operator's stencil (an M-matrix: the
    Stein-Rosenberg case), k Gauss-Seidel sweeps leave a smaller error than k
    Jacobi sweeps from the same start, and many sweeps reach the exact
    solution."""
    import scipy.sparse as sps
    import scipy.sparse.linalg as spla
    case, A, r = _os_system(9, 8, 6, 4, 8, "linear", seed=62, eps_dex=(-5, -2))
    exact = spla.spsolve(A.tocsc(), r)
    d = A.diagonal()
    off = (A - sps.diags(d)).tocsr()
    col = so.os_colours(case.chi[0].shape)
    x0 = r / d
    scale = np.abs(exact).max()
    errs_j, errs_g = [], []
    xj = x0.copy()
    for k in range(1, 17):
        xj = (r - off @ xj) / d
        if k in (2, 4, 8, 16):
            errs_j.append(np.abs(xj - exact).max() / scale)
            errs_g.append(np.abs(so.gauss_seidel(A, r, x0, col, k) - exact).max() / scale)
    print("Jacobi", errs_j, "Gauss-Seidel", errs_g)
    assert all(g < j for g, j in zip(errs_g, errs_j))
    np.testing.assert_allclose(so.gauss_seidel(A, r, x0, col, 400), exact, rtol=1e-11, atol=1e-13 * scale)


@pytest.mark.parametrize("op", ["linear", "parabolic"])
def test_ali_with_gauss_seidel_sweeps_reaches_the_lu_fixed_point(op):
    case = sy.random_box(7, 7, 5, 4, 8, seed=41, dtype="f64", eps_dex=(-4, -1))
    prob = so.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8, kind=op)
    ref = so.direct(prob)
    L = prob.lstar_nonlocal()
    r_jac = so.ali(prob, tol=1e-12, max_iter=5000, ng=False, lstar=L, inner_jacobi=3)
    r_gs = so.ali(prob, tol=1e-12, max_iter=5000, ng=False, lstar=L, inner_gs=3)
    for r in (r_jac, r_gs):
        assert r["converged"]
        np.testing.assert_allclose(r["J"], ref["J"], rtol=1e-9)
    print("steps Jacobi", r_jac["iters"], "Gauss-Seidel", r_gs["iters"])
    assert r_gs["iters"] <= r_jac["iters"]
