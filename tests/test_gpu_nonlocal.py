"""Parity of the nearest-neighbour Lambda* (rt_lstar_stencil) and of the ALI
that uses it (RT_F_LSTAR_NONLOCAL) with the oracle.

Tolerances: the GPU sums each element in 64-bit fixed point (units of 2^-52)
from double-precision per-point arithmetic, so on double grids the stencil
agrees with the oracle's to ~1e-13 absolute (elements are <= 1); single
grids store it in float (relative 6e-8).  The ALI keeps the stencil in the
grid precision for its Jacobi sweeps, so on double grids its iterates agree
with the oracle's (exact stencil, same number of sweeps) to rounding; the
fixed point does not depend on Lambda* at all, so converged results are held
to the LU solution at the usual tolerances.
"""
import numpy as np
import pytest

import synthetic as sy
from tests.gpu_helpers import gpu_solve, make_grid, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _grid(case, lstar="linear", prec=None, band_tiles=False):
    import paper_2102_01734_amd as rt
    return rt.Grid(case.Nx, case.Ny, case.Nz, case.n_mu, case.n_phi, prec or case.dtype, case.n_lambda,
                   lstar=lstar, band_tiles=band_tiles, nonlocal_lstar=True)


def _stencil(g, case, prec):
    torch = torch_cuda()
    st = g.lstar_stencil(to_dev(case.chi, prec))
    torch.cuda.synchronize()
    return st.double().cpu().numpy()


CASES = [  # (Nx, Ny, Nz, n_mu, n_phi, prec)
    (11, 11, 2, 4, 8, "f64"),
    (17, 13, 9, 4, 8, "f64"),
    (17, 13, 9, 4, 8, "f32"),
    (33, 33, 12, 8, 16, "f32"),
    (40, 37, 6, 4, 8, "f64"),
]


@pytest.mark.parametrize("op", ["linear", "parabolic"])
@pytest.mark.parametrize("shape", CASES)
def test_stencil_matches_oracle(orc, op, shape):
    Nx, Ny, Nz, n_mu, n_phi, prec = shape
    print(f"stencil {shape} {op}", flush=True)
    case = sy.random_box(Nx, Ny, Nz, n_mu, n_phi, seed=Nx + Nz, dtype=prec, n_lambda=2)
    g = _grid(case, lstar=op)
    st = _stencil(g, case, prec)
    g.close()
    for l in range(2):
        ref = orc.lstar_stencil(case.chi[l], n_mu, n_phi, op)
        if prec == "f64":
            np.testing.assert_allclose(st[l], ref, rtol=1e-12, atol=1e-13)
        else:
            np.testing.assert_allclose(st[l], ref, rtol=2e-7, atol=1e-12)


def test_stencil_centre_is_the_sweep_diagonal_and_band_tiles_do_not_matter():
    """Component 13 equals the Lambda* of the formal-solution sweep; the stencil
    does not depend on the tile kind of the grid (it is built per characteristic)."""
    torch = torch_cuda()
    case = sy.random_box(31, 23, 9, 4, 8, seed=31, dtype="f64")
    g = _grid(case)
    st = _stencil(g, case, "f64")
    chi = to_dev(case.chi, "f64")
    _, L = g.formal_solution(chi, torch.zeros_like(chi), None, want_lstar=True)
    torch.cuda.synchronize()
    g.close()
    np.testing.assert_allclose(st[0, 13], L.cpu().numpy()[0], rtol=1e-13, atol=1e-15)
    gb = _grid(case, band_tiles=True)
    assert gb.launch_shape()["band"]
    stb = _stencil(gb, case, "f64")
    gb.close()
    assert np.array_equal(st, stb)


def test_stencil_deterministic():
    case = sy.random_box(33, 33, 12, 8, 16, seed=33, dtype="f32")
    g = _grid(case)
    a = _stencil(g, case, "f32")
    b = _stencil(g, case, "f32")
    g.close()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,op", [((33, 33, 12, 8, 16, "f32"), "linear"), ((40, 37, 6, 4, 8, "f64"), "parabolic"),
                                      ((129, 17, 5, 4, 8, "f32"), "parabolic")])
def test_stencil_row_window_equals_per_characteristic_bitwise(monkeypatch, shape, op):
    """The row-window kernel (contributions gathered in LDS, one device add per
    target word and layer) and the per-characteristic kernel (one device add
    per contribution) add the same fixed-point integers: bitwise equal."""
    Nx, Ny, Nz, n_mu, n_phi, prec = shape
    print(f"stencil kernels {shape} {op}", flush=True)
    case = sy.random_box(Nx, Ny, Nz, n_mu, n_phi, seed=Ny, dtype=prec, n_lambda=2)
    g = _grid(case, lstar=op)
    a = _stencil(g, case, prec)
    g.close()
    monkeypatch.setenv("RT3D_STENCIL_PER_CHARACTERISTIC", "1")
    g = _grid(case, lstar=op)
    b = _stencil(g, case, prec)
    g.close()
    assert np.array_equal(a, b)


def test_stencil_full_size_properties():
    """129^3 x 2048 directions (single precision): the linear operator's stencil
    is non-negative, each row sums to at most 1, and its centre is the sweep's
    Lambda*."""
    torch = torch_cuda()
    case = sy.box_lognormal()
    print("stencil 129^3 x 2048", flush=True)
    g = _grid(case)
    chi = to_dev(case.chi, "f32")
    st = g.lstar_stencil(chi)
    _, L = g.formal_solution(chi, torch.zeros_like(chi), None, want_lstar=True)
    torch.cuda.synchronize()
    assert float(st.min()) >= 0.0
    assert float(st.double().sum(dim=1).max()) <= 1.0 + 1e-5
    np.testing.assert_allclose(st[0, 13].cpu().numpy(), L[0].cpu().numpy(), rtol=2e-5, atol=1e-7)
    g.close()


@pytest.mark.parametrize("method", ["jacobi", "gauss-seidel"])
@pytest.mark.parametrize("op", ["linear", "parabolic"])
def test_nonlocal_ali_steps_match_oracle_iterates(orc, op, method):
    """J after 1, 3 and 6 steps (Ng between steps 4 and 5), 5 Jacobi or
    Gauss-Seidel (colour order) sweeps per step, equals the oracle's non-local
    ALI with the same sweeps.  11 x 11 is odd: the last column and row take
    their own colour."""
    torch = torch_cuda()
    case = sy.random_box(11, 11, 6, 4, 8, seed=43, dtype="f64", eps_dex=(-4, -1))
    g = _grid(case, lstar=op)
    st = g.new_state(to_dev(case.chi, "f64"), to_dev(case.eps, "f64"), to_dev(case.B, "f64"),
                     to_dev(case.I_bc, "f64"))
    opts = g.opts(tol=1e-30, max_iter=1, ng_every=4, ng_start=4, os_sweeps=5, os_method=method)
    inner = dict(inner_jacobi=5) if method == "jacobi" else dict(inner_gs=5)
    prob = orc.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8, kind=op)
    L = prob.lstar_nonlocal()
    done = 0
    for n in (1, 3, 6):
        while done < n:
            g.ali_step(st, opts)
            done += 1
        torch.cuda.synchronize()
        Jg = g.state_tensors(st)["J"].cpu().numpy()[0]
        ref = orc.ali(prob, tol=1e-30, max_iter=n, ng=True, ng_start=4, ng_every=4, lstar=L, **inner)
        np.testing.assert_allclose(Jg, ref["J"], rtol=1e-10)
    g.close()


@pytest.mark.parametrize("op", ["linear", "parabolic"])
def test_nonlocal_fp64_reaches_lu_fixed_point_in_fewer_steps(orc, op):
    case = sy.random_box(7, 7, 5, 4, 8, seed=41, dtype="f64", eps_dex=(-4, -1))
    g = _grid(case, lstar=op)
    r = gpu_solve(case, tol=1e-13, max_iter=3000, lstar=op, grid=g)
    g.close()
    r0 = gpu_solve(case, tol=1e-13, max_iter=3000, lstar=op)
    prob = orc.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8, kind=op)
    ref = orc.direct(prob)
    assert r["status"] == 0 and r0["status"] == 0
    np.testing.assert_allclose(r["J"][0], ref["J"], rtol=1e-10)
    np.testing.assert_allclose(r["S"][0], ref["S"], rtol=1e-10)
    print("steps diagonal", r0["report"].iters, "non-local", r["report"].iters)
    assert r["report"].iters < r0["report"].iters


@pytest.mark.parametrize("method", ["jacobi", "gauss-seidel"])
@pytest.mark.parametrize("eps_dex", [(-2, 0), (-5, -3)])
def test_nonlocal_fp32_defect_corrected_reaches_fixed_point(orc, eps_dex, method):
    case = sy.random_box(9, 9, 8, 4, 8, seed=47, dtype="f32", eps_dex=eps_dex)
    g = _grid(case)
    r = gpu_solve(case, tol=1e-9, max_iter=3000, grid=g, os_method=method)
    g.close()
    prob = orc.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8)
    ref = orc.direct(prob)
    assert r["status"] == 0
    err = np.max(np.abs(r["J"][0] - ref["J"]) / np.abs(ref["J"]))
    print("non-local fp32", method, "fixed-point error", err, "steps", r["report"].iters)
    assert err < 1e-5


def test_nonlocal_batch_each_wavelength_reaches_its_fixed_point(orc):
    case = sy.random_box(8, 7, 6, 4, 8, seed=53, dtype="f64", n_lambda=3, eps_dex=(-3, 0))
    g = _grid(case)
    r = gpu_solve(case, tol=1e-12, max_iter=3000, grid=g)
    g.close()
    assert r["status"] == 0
    for l in range(3):
        prob = orc.BoxProblem(case.chi[l], case.eps[l], case.B[l], case.I_bc[l, 0], case.I_bc[l, 1], 4, 8)
        np.testing.assert_allclose(r["J"][l], orc.direct(prob)["J"], rtol=1e-9)


@pytest.mark.parametrize("method", ["jacobi", "gauss-seidel"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_nonlocal_graph_replay_equals_eager_bitwise(prec, method):
    torch = torch_cuda()
    case = sy.random_box(17, 13, 9, 4, 8, seed=57, dtype=prec, eps_dex=(-3, -1))
    out = []
    for use_graph in (False, True):
        g = _grid(case)
        st = g.new_state(to_dev(case.chi, prec), to_dev(case.eps, prec), to_dev(case.B, prec),
                         to_dev(case.I_bc, prec))
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            for _ in range(9):
                g.ali_step(st, g.opts(tol=1e-30, max_iter=1, use_graph=use_graph, os_sweeps=3, os_method=method),
                           stream=s)
        s.synchronize()
        out.append(g.state_tensors(st)["J"].cpu().numpy())
        g.close()
    assert np.array_equal(out[0], out[1])


def test_nonlocal_arguments():
    import paper_2102_01734_amd as rt
    case = sy.random_box(9, 9, 4, 4, 8, seed=59, dtype="f64")
    g = _grid(case)
    st = g.new_state(to_dev(case.chi, "f64"), to_dev(case.eps, "f64"), to_dev(case.B, "f64"))
    with pytest.raises(rt.RtError):
        g.ali_step(st, g.opts(os_sweeps=-1))
    o = g.opts()
    o.os_method = 7
    with pytest.raises(rt.RtError):
        g.ali_step(st, o)
    with pytest.raises(rt.RtError):
        g.lstar_stencil(to_dev(np.zeros((2, 4, 9, 9)), "f64"))   # 2 > n_lambda_max
    g.close()
    d = rt.rt3d.sphere_desc(9, 7, 8, 1.0, 2.0, 4, 4, "f64", 1)
    d.flags |= rt.rt3d.RT_F_LSTAR_NONLOCAL | rt.rt3d.RT_F_BAND_TILES   # band tiles are a box notion
    with pytest.raises(rt.RtError) as e:
        rt.rt3d.rt_create_grid(d)
    assert e.value.status == rt.rt3d.RT_E_INVALID


@pytest.mark.parametrize("op", ["linear", "parabolic"])
def test_stencil_jacobi_dominance_full_size(op):
    """Jacobi sweeps on [1 - Lambda*(1-eps)] dJ = r converge when every row is
    diagonally dominant: sum_{u != v} |L_vu| (1 - eps_u) < 1 - L_vv (1 - eps_v).
    On the 129^3 x 2048 workload (eps down to 1e-6): the linear operator's
    stencil (non-negative, rows summing to at most 1) satisfies it everywhere;
    for the parabolic one (negative weights) the largest ratio is printed and
    must stay below 1 as well."""
    torch = torch_cuda()
    case = sy.box_lognormal()
    print(f"stencil dominance 129^3 x 2048 {op}", flush=True)
    g = _grid(case, lstar=op)
    chi = to_dev(case.chi, "f32")
    st = g.lstar_stencil(chi)[0].double()              # (27, Nz, Ny, Nx)
    torch.cuda.synchronize()
    g.close()
    om = 1.0 - to_dev(case.eps, "f64")[0]              # (Nz, Ny, Nx)
    Nz = om.shape[0]
    off = torch.zeros_like(om)
    for c in range(27):
        if c == 13:
            continue
        dz, dy, dx = c // 9 - 1, (c // 3) % 3 - 1, c % 3 - 1
        # (1 - eps) of the neighbour u = v + (dx, dy, dz); no neighbour beyond the top/bottom layer
        omu = torch.roll(om, shifts=(-dy, -dx), dims=(1, 2))
        omu = torch.roll(omu, shifts=-dz, dims=0)
        if dz == 1:
            omu[Nz - 1] = 0.0
        elif dz == -1:
            omu[0] = 0.0
        off += st[c].abs() * omu
    den = 1.0 - st[13] * om
    ratio = float((off / den).max())
    print(f"  max_v sum_u!=v |L_vu|(1-eps_u) / (1 - L_vv(1-eps_v)) = {ratio:.6f}")
    assert ratio < 1.0
