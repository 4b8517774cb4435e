"""Parity of the spherical formal solution and ALI (SphereGrid) with the oracle.

Tolerances as for the box: double-precision grids take the same steps and
fallback decisions as the oracle and differ by rounding only (1e-12);
single-precision grids run the recurrence in float and keep the geometry
(path lengths, averaging weights) in float (2e-5).
"""
import numpy as np
import pytest

import synthetic as sy
from tests.gpu_helpers import gpu_fs, gpu_solve, make_grid, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _oracle_fs(orc, case, S, kind):
    g = orc.SphereGrid(case.Nr, case.Nt, case.Np, case.r_core, case.r_out)
    Js, Ls = [], []
    for l in range(case.n_lambda):
        I_out, I_core, J_sub = case.I_bc[l]
        J, L = orc.fs_sphere(g, case.n_mu, case.n_phi, case.chi[l], S[l], np.full(case.n_vox, I_core),
                             I_out=I_out, dsrc=case.source_distance, B_sub=J_sub, kind=kind)
        Js.append(J.reshape(case.chi.shape[1:])); Ls.append(L.reshape(case.chi.shape[1:]))
    return np.array(Js), np.array(Ls)


SHAPES = [  # (Nr, Nt, Np, n_mu, n_phi, source distance)
    (9, 8, 12, 4, 8, 5.0),
    (6, 7, 5, 2, 4, 0.0),
    (12, 10, 16, 8, 16, 3.0),
    (1, 1, 1, 2, 2, 5.0),
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["linear", "parabolic"])
def test_sphere_fs_fp64_matches_oracle(orc, shape, kind):
    Nr, Nt, Np, n_mu, n_phi, dsrc = shape
    print(f"sphere fs fp64 {shape} {kind}", flush=True)
    case = sy.random_sphere(Nr, Nt, Np, n_mu, n_phi, seed=Nr * 13 + Np, dtype="f64", source_distance=dsrc)
    S = sy.random_source(case.chi.shape, seed=31)
    J, L = gpu_fs(case, S, lstar=kind)
    Jo, Lo = _oracle_fs(orc, case, S, kind)
    np.testing.assert_allclose(J, Jo, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(L, Lo, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("shape", SHAPES[:3])
def test_sphere_fs_fp32_matches_oracle(orc, shape):
    Nr, Nt, Np, n_mu, n_phi, dsrc = shape
    print(f"sphere fs fp32 {shape}", flush=True)
    case = sy.random_sphere(Nr, Nt, Np, n_mu, n_phi, seed=Nr + 7 * Np, dtype="f32", source_distance=dsrc)
    S = sy.random_source(case.chi.shape, seed=32, dtype="f32")
    J, L = gpu_fs(case, S)
    Jo, Lo = _oracle_fs(orc, case, S, "linear")
    np.testing.assert_allclose(J, Jo, rtol=2e-5, atol=1e-6 * np.abs(Jo).max())
    np.testing.assert_allclose(L, Lo, rtol=2e-5, atol=1e-7)


def test_sphere_opaque_and_vacuum_voxels(orc):
    case = sy.random_sphere(8, 6, 9, 4, 8, seed=41, dtype="f64")
    rng = np.random.default_rng(1)
    case.chi[rng.random(case.chi.shape) < 0.2] = 0.0
    case.chi[rng.random(case.chi.shape) < 0.1] = 1e6
    S = sy.random_source(case.chi.shape, seed=42)
    J, L = gpu_fs(case, S, lstar="parabolic")
    Jo, Lo = _oracle_fs(orc, case, S, "parabolic")
    np.testing.assert_allclose(J, Jo, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(L, Lo, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sphere_chunked_cache_and_batch(prec, monkeypatch):
    """Splitting the geometry cache into many chunks and batching wavelengths
    change nothing: batch entries are bitwise equal to single-wavelength runs,
    and chunked runs agree with the one-chunk run to the rounding of the
    chunk-wise accumulation."""
    case = sy.random_sphere(7, 6, 8, 4, 8, seed=51, dtype=prec, n_lambda=3)
    S = sy.random_source(case.chi.shape, seed=52, dtype=prec)
    J1, L1 = gpu_fs(case, S)
    monkeypatch.setenv("RT3D_SPHERE_CHUNK_VISITS", "4000")
    g = make_grid(case)
    assert g.info()["n_workgroups"] > 3          # number of cache chunks
    Jc, Lc = gpu_fs(case, S, grid=g)
    tol = 1e-14 if prec == "f64" else 2e-6
    np.testing.assert_allclose(Jc, J1, rtol=tol, atol=tol * np.abs(J1).max())
    np.testing.assert_allclose(Lc, L1, rtol=tol, atol=tol)
    for l in range(3):
        one = sy.random_sphere(7, 6, 8, 4, 8, seed=51, dtype=prec, n_lambda=3)
        one.chi, one.eps, one.B, one.I_bc = case.chi[l:l + 1], case.eps[l:l + 1], case.B[l:l + 1], case.I_bc[l:l + 1]
        Jl, Ll = gpu_fs(one, S[l:l + 1], grid=g)
        assert np.array_equal(Jl[0], Jc[l]) and np.array_equal(Ll[0], Lc[l])
    g.close()


def test_sphere_ali_fixed_point_matches_lu(orc):
    """FP64 Ng-ALI on the sphere reaches the oracle's LU fixed point."""
    case = sy.random_sphere(6, 5, 7, 4, 8, seed=61, dtype="f64")
    g = orc.SphereGrid(6, 5, 7, 1.0, 2.0)
    I_out, I_core, J_sub = case.I_bc[0]
    prob = orc.SphereProblem(g, case.chi[0].ravel(), case.eps[0].ravel(), case.B[0].ravel(), I_out, I_core,
                             4, 8, dsrc=case.source_distance, J_sub=J_sub)
    ref = orc.direct(prob)
    res = gpu_solve(case, tol=1e-13, max_iter=3000)
    assert res["status"] == 0
    np.testing.assert_allclose(res["J"][0], ref["J"], rtol=1e-10)


def test_sphere_ali_fp32_defect_correction_reaches_fixed_point(orc):
    """Single-precision sweeps with double-precision anchors converge to the
    fixed point of the float-geometry operator: within 1e-5 of the oracle's."""
    case = sy.random_sphere(6, 5, 7, 4, 8, seed=62, dtype="f32")
    g = orc.SphereGrid(6, 5, 7, 1.0, 2.0)
    I_out, I_core, J_sub = case.I_bc[0]
    prob = orc.SphereProblem(g, case.chi[0].ravel(), case.eps[0].ravel(), case.B[0].ravel(), I_out, I_core,
                             4, 8, dsrc=case.source_distance, J_sub=J_sub)
    ref = orc.direct(prob)
    res = gpu_solve(case, tol=1e-9, max_iter=3000)
    assert res["status"] == 0
    np.testing.assert_allclose(res["J"][0], ref["J"], rtol=1e-5)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sphere_graph_replay_equals_eager(prec):
    """Plain steps replayed from captured HIP graphs give bitwise the eager iterates."""
    torch = torch_cuda()
    case = sy.random_sphere(7, 6, 8, 4, 8, seed=71, dtype=prec, n_lambda=2, eps_dex=(-3, -1))
    outs = []
    for use_graph in (False, True):
        g = make_grid(case)
        st = g.new_state(to_dev(case.chi, prec), to_dev(case.eps, prec), to_dev(case.B, prec),
                         to_dev(case.I_bc, prec))
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            status, rep = g.solve(st, g.opts(tol=1e-10, max_iter=400, use_graph=use_graph), stream=stream)
        stream.synchronize()
        outs.append((status, rep.iters, g.state_tensors(st)["J"].cpu().numpy().copy()))
        g.close()
    assert outs[0][0] == outs[1][0] == 0
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][2], outs[1][2])


def test_sphere_rejects_box_only_calls():
    import paper_2102_01734_amd as rt
    case = sy.random_sphere(4, 4, 4, 2, 4, seed=81, dtype="f32")
    g = make_grid(case)
    with pytest.raises(rt.RtError):
        g.set_launch_shape(768, 22)
    for band in (False, True):
        with pytest.raises(rt.RtError) as e:
            g.set_launch_shape(768, 11, band=band)
        assert e.value.status == rt.rt3d.RT_E_UNSUPPORTED
        with pytest.raises(rt.RtError) as e:
            g.set_anchor_shape(768, 11, band=band)
        assert e.value.status == rt.rt3d.RT_E_UNSUPPORTED
    chi = to_dev(case.chi, "f32")
    with pytest.raises(rt.RtError):
        g.autotune(chi, chi)
    g.close()
    with pytest.raises(rt.RtError):
        rt.SphereGrid(4, 4, 4, 2.0, 1.0, 2, 4)


def test_sphere_radial_workload_small(orc):
    """The irradiated radial-opacity shell at reduced size: GPU J within the
    single-precision bound of the oracle's on the same S."""
    case = sy.sphere_radial(Nr=13, Nt=9, Np=17, n_mu=4, n_phi=8, n_lambda=2)
    S = np.broadcast_to(case.B, case.chi.shape).copy()
    J, L = gpu_fs(case, S)
    Jo, Lo = _oracle_fs(orc, case, S, "linear")
    np.testing.assert_allclose(J, Jo, rtol=2e-5, atol=1e-6 * np.abs(Jo).max())
    assert np.all(np.isfinite(J)) and np.all((L > 0) & (L <= 1))


def test_sphere_full_size_radial_workload(orc):
    """97 x 65 x 129 shell, 32 x 32 directions, 16 wavelengths in one batch, single
    precision, as the spherical benchmark runs it: wavelength 0 against the
    oracle at every voxel (S = B)."""
    import time
    case = sy.sphere_radial()
    S = np.broadcast_to(case.B, case.chi.shape).astype(np.float64)
    print("sphere full size: GPU", flush=True)
    t0 = time.time()
    J, L = gpu_fs(case, S)
    print(f"sphere full size: GPU done in {time.time() - t0:.1f} s; oracle", flush=True)
    g = orc.SphereGrid(case.Nr, case.Nt, case.Np, case.r_core, case.r_out)
    I_out, I_core, J_sub = case.I_bc[0]
    Jo, Lo = orc.fs_sphere(g, case.n_mu, case.n_phi, case.chi[0], S[0], np.full(case.n_vox, I_core),
                           I_out=I_out, dsrc=case.source_distance, B_sub=J_sub)
    print(f"sphere full size: oracle done at {time.time() - t0:.1f} s", flush=True)
    np.testing.assert_allclose(J[0].ravel(), Jo, rtol=2e-5, atol=1e-6 * np.abs(Jo).max())
    np.testing.assert_allclose(L[0].ravel(), Lo, rtol=2e-5, atol=1e-7)
    # at optical steps of 1e4 and more Lambda* = 1 - e^-D rounds to 1 in single precision
    assert np.all(np.isfinite(J)) and np.all((L > 0) & (L <= 1))
