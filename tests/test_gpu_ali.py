"""Parity of the HIP operator-splitting iteration (rt_ali_step / rt_solve) with the oracle.

The fixed point is unique (eps > 0 or open boundaries), so the GPU result is
compared with the oracle's fixed point (LU on tiny boxes, the layer reduction
for x,y-uniform slabs); single steps are compared with the oracle's ALI
iterates, which also pins the Ng schedule.
"""
import numpy as np
import pytest

import synthetic as sy
from tests.gpu_helpers import gpu_solve, make_grid, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _lu(orc, case, l=0, kind="linear"):
    prob = orc.BoxProblem(case.chi[l], case.eps[l], case.B[l], case.I_bc[l, 0], case.I_bc[l, 1],
                          case.n_mu, case.n_phi, kind=kind)
    return orc.direct(prob)


@pytest.mark.parametrize("kind", ["linear", "parabolic"])
def test_solve_fp64_tiny_box_reaches_lu_fixed_point(orc, kind):
    print(f"solve fp64 tiny {kind}", flush=True)
    case = sy.random_box(7, 7, 5, 4, 8, seed=41, dtype="f64")
    r = gpu_solve(case, tol=1e-13, max_iter=3000, lstar=kind)
    ref = _lu(orc, case)
    assert r["status"] == 0
    np.testing.assert_allclose(r["J"][0], ref["J"], rtol=1e-10)
    np.testing.assert_allclose(r["S"][0], ref["S"], rtol=1e-10)


def test_ali_steps_match_oracle_iterates(orc):
    """J after 1, 3 and 6 steps (Ng applied between steps 4 and 5) equals the oracle's iterates."""
    case = sy.random_box(9, 8, 6, 4, 8, seed=43, dtype="f64", eps_dex=(-4, -1))
    torch = torch_cuda()
    g = make_grid(case)
    st = g.new_state(to_dev(case.chi, "f64"), to_dev(case.eps, "f64"), to_dev(case.B, "f64"),
                     to_dev(case.I_bc, "f64"))
    opts = g.opts(tol=1e-30, max_iter=1, ng_every=4, ng_start=4)
    prob = orc.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8)
    done = 0
    for n in (1, 3, 6):
        while done < n:
            g.ali_step(st, opts)
            done += 1
        torch.cuda.synchronize()
        Jg = g.state_tensors(st)["J"].cpu().numpy()[0]
        ref = orc.ali(prob, tol=1e-30, max_iter=n, ng=True, ng_start=4, ng_every=4)
        np.testing.assert_allclose(Jg, ref["J"], rtol=1e-11)
    rel = g.state_tensors(st)["rel_change"].cpu().numpy()
    assert rel[0] > 0
    g.close()


def test_solve_fp64_stratified_slab(orc):
    """The 33^3 stratified slab (eps = 1e-2, 8x16 directions, FP64, Ng-ALI to
    max|dJ/J| < 1e-8): same fixed point and same number of steps as the oracle's
    Ng-ALI on the layer reduction."""
    case = sy.box_stratified()
    r = gpu_solve(case, tol=1e-8, max_iter=2000)
    prob = orc.Plane1DProblem(case.chi[0, :, 0, 0], case.eps[0, :, 0, 0], 1.0, 0.0, 1.0, case.n_mu, case.n_phi)
    ref = orc.ali(prob, tol=1e-8, ng=True)
    exact = orc.direct(prob)
    Jg = r["J"][0]
    assert r["status"] == 0
    assert abs(r["report"].iters - ref["iters"]) <= 1
    np.testing.assert_allclose(Jg, np.broadcast_to(ref["J"][:, None, None], Jg.shape), rtol=1e-9)
    # tighter solve reaches the exact (LU) fixed point
    r2 = gpu_solve(case, tol=1e-13, max_iter=4000)
    np.testing.assert_allclose(r2["J"][0], np.broadcast_to(exact["J"][:, None, None], Jg.shape), rtol=1e-10)


@pytest.mark.parametrize("eps_dex", [(-2, 0), (-4, -2)])
def test_solve_fp32_defect_corrected_reaches_fixed_point(orc, eps_dex):
    """Single-precision formal solutions with double anchors: converged J within
    1e-5 (max relative) of the oracle's fixed point."""
    print(f"solve fp32 {eps_dex}", flush=True)
    case = sy.random_box(9, 9, 8, 4, 8, seed=47, dtype="f32", eps_dex=eps_dex)
    r = gpu_solve(case, tol=1e-9, max_iter=3000)
    ref = _lu(orc, case)
    assert r["status"] == 0
    err = np.max(np.abs(r["J"][0] - ref["J"]) / np.abs(ref["J"]))
    print("fp32 fixed-point error", err, "steps", r["report"].iters, "fs64", r["report"].n_fs64)
    assert err < 1e-5


def test_solve_batch_each_wavelength_matches(orc):
    case = sy.random_box(8, 7, 6, 4, 8, seed=53, dtype="f64", n_lambda=3, eps_dex=(-3, 0))
    r = gpu_solve(case, tol=1e-12, max_iter=3000)
    for l in range(3):
        ref = _lu(orc, case, l)
        np.testing.assert_allclose(r["J"][l], ref["J"], rtol=1e-9)


def test_not_converged_then_resume(orc):
    import paper_2102_01734_amd as rt
    torch = torch_cuda()
    case = sy.random_box(8, 8, 6, 4, 8, seed=59, dtype="f64", eps_dex=(-4, -3))
    g = make_grid(case)
    st = g.new_state(to_dev(case.chi, "f64"), to_dev(case.eps, "f64"), to_dev(case.B, "f64"),
                     to_dev(case.I_bc, "f64"))
    status, rep = g.solve(st, g.opts(tol=1e-12, max_iter=3))
    assert status == rt.rt3d.RT_E_NOT_CONVERGED and rep.iters == 3
    status, rep = g.solve(st, g.opts(tol=1e-12, max_iter=3000))
    torch.cuda.synchronize()
    assert status == 0
    ref = _lu(orc, case)
    np.testing.assert_allclose(g.state_tensors(st)["J"].cpu().numpy()[0], ref["J"], rtol=1e-9)
    g.close()


def test_non_finite_input_is_reported():
    import paper_2102_01734_amd as rt
    case = sy.random_box(6, 6, 5, 4, 8, seed=61, dtype="f64")
    case.chi[0, 2, 3, 3] = np.nan
    g = make_grid(case)
    st = g.new_state(to_dev(case.chi, "f64"), to_dev(case.eps, "f64"), to_dev(case.B, "f64"),
                     to_dev(case.I_bc, "f64"))
    with pytest.raises(rt.RtError) as e:
        g.solve(st, g.opts(tol=1e-10, max_iter=50))
    assert e.value.status == rt.rt3d.RT_E_NUMERIC
    g.close()


def test_invalid_state_and_options():
    import ctypes

    import paper_2102_01734_amd as rt
    case = sy.random_box(6, 6, 5, 4, 8, seed=62, dtype="f64")
    g = make_grid(case)
    st = g.new_state(to_dev(case.chi, "f64"), to_dev(case.eps, "f64"), to_dev(case.B, "f64"))
    bad = g.opts(tol=0.0)
    with pytest.raises(rt.RtError):
        g.solve(st, bad)
    st.n_lambda = 2
    with pytest.raises(rt.RtError):
        g.ali_step(st, g.opts())
    st.n_lambda = 1
    st.struct_size = ctypes.sizeof(rt.RtState) + 8
    with pytest.raises(rt.RtError):
        g.ali_step(st, g.opts())
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replay_equals_eager_bitwise(prec):
    """Plain steps replayed from a captured HIP graph give bitwise the eager iterates
    (several replays, with host synchronisation between them)."""
    torch = torch_cuda()
    case = sy.random_box(11, 9, 7, 4, 8, seed=71, dtype=prec, n_lambda=2, eps_dex=(-3, -1))
    outs = []
    for use_graph in (False, True):
        g = make_grid(case)
        st = g.new_state(to_dev(case.chi, prec), to_dev(case.eps, prec), to_dev(case.B, prec),
                         to_dev(case.I_bc, prec))
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            status, rep = g.solve(st, g.opts(tol=1e-11, max_iter=400, use_graph=use_graph), stream=stream)
        stream.synchronize()
        outs.append((status, rep.iters, g.state_tensors(st)["J"].cpu().numpy().copy()))
        g.close()
    assert outs[0][0] == outs[1][0] == 0
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][2], outs[1][2])


def test_batched_wavelengths_converge_independently(orc):
    """A batch with very different opacity scales and eps: every wavelength reaches
    its own fixed point; converged ones drop out of later steps."""
    case = sy.random_box(8, 8, 6, 4, 8, seed=73, dtype="f64", n_lambda=4)
    scale = np.array([1e-2, 1.0, 30.0, 3e2])
    case.chi = case.chi * scale[:, None, None, None]
    case.eps[:] = np.array([0.5, 0.1, 0.03, 0.01])[:, None, None, None]
    r = gpu_solve(case, tol=1e-12, max_iter=3000)
    assert r["status"] == 0 and r["report"].n_converged == 4
    for l in range(4):
        ref = _lu(orc, case, l)
        np.testing.assert_allclose(r["J"][l], ref["J"], rtol=1e-9)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_pure_scattering_slab_reaches_fixed_point(orc, prec):
    """eps = 0 (pure scattering) on a stratified slab (tau 1e-4..1e2) lit from its
    thin top: the solve converges to the layer reduction's direct solution
    (single precision: within 1e-5 through the double anchors).  The error of an
    iteration stopped at relative change tol is about tol / (1 - rho), rho the
    contraction of the accelerated iteration, close to 1 here: stopped at 1e-11
    the double-precision error measured 1.2e-9 to 1.6e-9 (at 1e-10, 7e-9 to 1.3e-8
    depending on where the Ng steps fall), so 1e-8 keeps a margin of six."""
    import dataclasses
    case = sy.box_stratified(N=9, Nz=33, eps=0.0, dtype=prec, tau_max=1e2)
    case = dataclasses.replace(case, I_bc=np.array([[1.0, 0.0]]))
    r = gpu_solve(case, tol=1e-11, max_iter=4000)
    prob = orc.Plane1DProblem(case.chi[0, :, 0, 0], case.eps[0, :, 0, 0], 1.0, 1.0, 0.0, case.n_mu, case.n_phi)
    exact = orc.direct(prob)
    Jg = r["J"][0]
    err = np.max(np.abs(Jg - exact["J"][:, None, None]) / exact["J"][:, None, None])
    print(f"pure scattering {prec}: status {r['status']}, steps {r['report'].iters}, error {err:.2e}")
    assert r["status"] == 0
    assert err < (1e-5 if prec == "f32" else 1e-8)


@pytest.mark.parametrize("band", [False, True])
def test_anchor_shape_changes_only_the_summation_order(orc, band):
    """A fixed launch shape (whole-layer or row-band tiles) for the
    double-precision anchors of a single precision grid: the solve reaches the
    same fixed point; double-precision grids and uncompiled shapes are refused."""
    import paper_2102_01734_amd as rt
    case = sy.random_box(9, 9, 8, 4, 8, seed=47, dtype="f32", eps_dex=(-4, -2))
    g = make_grid(case)
    g.set_anchor_shape(1024, 1, band=band)
    with pytest.raises(rt.RtError):
        g.set_anchor_shape(100, 3)      # not compiled
    with pytest.raises(rt.RtError):
        g.set_anchor_shape(1024, 4)     # 81 rays cannot fill 4 ray slots per thread
    r = gpu_solve(case, tol=1e-9, max_iter=3000, grid=g)
    g.close()
    ref = _lu(orc, case)
    assert r["status"] == 0
    assert np.max(np.abs(r["J"][0] - ref["J"]) / np.abs(ref["J"])) < 1e-5
    g64 = make_grid(sy.random_box(9, 9, 8, 4, 8, seed=47, dtype="f64"))
    with pytest.raises(rt.RtError):
        g64.set_anchor_shape(1024, 1)
    g64.close()


def test_profiled_graph_steps_report_sweep_times_and_equal_unprofiled():
    """With the measurement hooks on, captured ALI steps carry event nodes
    around their sweep: every replay's sweep time is reported, and the
    iterates equal those of unprofiled graph replays bitwise."""
    import paper_2102_01734_amd as rt
    torch = torch_cuda()
    case = sy.random_box(21, 17, 9, 4, 8, seed=77, dtype="f32", eps_dex=(-3, -1))
    out = []
    for prof in (False, True):
        g = make_grid(case)
        st = g.new_state(to_dev(case.chi, "f32"), to_dev(case.eps, "f32"), to_dev(case.B, "f32"),
                         to_dev(case.I_bc, "f32"))
        s = torch.cuda.Stream()
        rt.rt_profile_enable(g.handle, prof)
        opts = g.opts(tol=1e-30, max_iter=1, use_graph=True)
        with torch.cuda.stream(s):
            for _ in range(2):  # Lambda* + anchor step, first graph capture
                g.ali_step(st, opts, stream=s)
        s.synchronize()
        rt.rt_profile_read(g.handle)
        with torch.cuda.stream(s):
            for _ in range(7):
                g.ali_step(st, opts, stream=s)
        s.synchronize()
        ms, n, pts = rt.rt_profile_read(g.handle)
        if prof:
            # seven plain steps: seven sweeps timed (Ng is applied before a step's sweep)
            assert n == 7 and ms > 0.0 and pts > 0
        else:
            assert n == 0
        out.append(g.state_tensors(st)["J"].cpu().numpy())
        g.close()
    assert np.array_equal(out[0], out[1])
