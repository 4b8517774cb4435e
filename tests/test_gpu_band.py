"""Band tiles of the box sweep (RT_F_BAND_TILES, and layers too wide for a
whole-layer tile): parity with the oracle.

With band tiles a workgroup sweeps a bundle of whole ray rows and keeps only
the rows those rays reach within the current layer.  The visits, the point
arithmetic and the per-voxel averaging are those of the layer-tile sweep, so
the tolerances are the ones of test_gpu_fs: 1e-12 for double grids, 5e-6
relative for single grids; against the layer-tile sweep of the same grid the
results differ only in the summation order of J.
"""
import dataclasses

import numpy as np
import pytest

import synthetic as sy
from tests.gpu_helpers import gpu_fs, gpu_solve, make_grid, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _oracle_fs(orc, case, S, kind):
    Js, Ls = [], []
    for l in range(case.n_lambda):
        J, L = orc.fs_box(case.chi[l], S[l], case.I_bc[l, 0], case.I_bc[l, 1], case.n_mu, case.n_phi, kind=kind)
        Js.append(J); Ls.append(L)
    return np.array(Js), np.array(Ls)


SHAPES = [  # (Nx, Ny, Nz, n_mu, n_phi): several bands per direction, Nx != Ny, tiny rows
    (33, 33, 12, 8, 16),
    (31, 23, 9, 4, 8),
    (17, 13, 9, 4, 8),
    (9, 9, 8, 4, 8),
]


def _band_grid(case, **kw):
    g = make_grid(case, band_tiles=True, **kw)
    ls = g.launch_shape()
    assert ls["band"] and ls["bundles"] >= 2, ls
    return g


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["linear", "parabolic"])
def test_band_tiles_fp64_match_oracle(orc, shape, kind):
    Nx, Ny, Nz, n_mu, n_phi = shape
    print(f"band fp64 {shape} {kind}", flush=True)
    case = sy.random_box(Nx, Ny, Nz, n_mu, n_phi, seed=Nx * 3 + Nz, dtype="f64")
    S = sy.random_source(case.chi.shape, seed=13, dtype="f64")
    g = _band_grid(case, lstar=kind)
    J, L = gpu_fs(case, S, lstar=kind, grid=g)
    g.close()
    Jo, Lo = _oracle_fs(orc, case, S, kind)
    np.testing.assert_allclose(J, Jo, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(L, Lo, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("shape", SHAPES[:3])
def test_band_tiles_fp32_match_oracle(orc, shape):
    Nx, Ny, Nz, n_mu, n_phi = shape
    print(f"band fp32 {shape}", flush=True)
    case = sy.random_box(Nx, Ny, Nz, n_mu, n_phi, seed=Nx + 7 * Nz, dtype="f32")
    S = sy.random_source(case.chi.shape, seed=14, dtype="f32")
    g = _band_grid(case)
    J, L = gpu_fs(case, S, grid=g)
    g.close()
    Jo, Lo = _oracle_fs(orc, case, S, "linear")
    np.testing.assert_allclose(J, Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
    np.testing.assert_allclose(L, Lo, rtol=5e-6, atol=1e-8)


def test_band_and_layer_tiles_agree():
    """Same grid, both tile kinds: double-precision J and Lambda* agree to the
    rounding of a different summation order; a batch of wavelengths gives each
    wavelength's single result bitwise."""
    case = sy.random_box(40, 37, 6, 4, 8, seed=15, dtype="f64", n_lambda=3)
    S = sy.random_source(case.chi.shape, seed=16, dtype="f64")
    J0, L0 = gpu_fs(case, S)
    g = _band_grid(case)
    J1, L1 = gpu_fs(case, S, grid=g)
    g.close()
    np.testing.assert_allclose(J1, J0, rtol=1e-14, atol=1e-15 * np.abs(J0).max())
    np.testing.assert_allclose(L1, L0, rtol=1e-14, atol=1e-16)
    for l in range(3):
        one = dataclasses.replace(case, chi=case.chi[l:l + 1], eps=case.eps[l:l + 1], B=case.B[l:l + 1],
                                  I_bc=case.I_bc[l:l + 1])
        g = _band_grid(one)
        Jl, _ = gpu_fs(one, S[l:l + 1], grid=g)
        g.close()
        assert np.array_equal(Jl[0], J1[l])


def test_band_tiles_deterministic():
    case = sy.random_box(31, 23, 9, 4, 8, seed=17, dtype="f32")
    S = sy.random_source(case.chi.shape, seed=18, dtype="f32")
    g = _band_grid(case)
    J0, L0 = gpu_fs(case, S, grid=g)
    J1, L1 = gpu_fs(case, S, grid=g)
    g.close()
    assert np.array_equal(J0, J1) and np.array_equal(L0, L1)


@pytest.mark.parametrize("eps_dex", [(-2, 0), (-4, -2)])
def test_band_tiles_fp32_solve_reaches_fixed_point(orc, eps_dex):
    """Single-precision ALI with double anchors, every sweep on band tiles:
    converged J within 1e-5 of the oracle's LU fixed point."""
    print(f"band solve fp32 {eps_dex}", flush=True)
    case = sy.random_box(9, 9, 8, 4, 8, seed=47, dtype="f32", eps_dex=eps_dex)
    g = _band_grid(case)
    r = gpu_solve(case, tol=1e-9, max_iter=3000, grid=g)
    g.close()
    prob = orc.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1],
                          case.n_mu, case.n_phi)
    ref = orc.direct(prob)
    assert r["status"] == 0
    err = np.max(np.abs(r["J"][0] - ref["J"]) / np.abs(ref["J"]))
    print("band fp32 fixed-point error", err, "steps", r["report"].iters)
    assert err < 1e-5


BAND_TUNE = [(1024, 17), (768, 11), (768, 22), (512, 9), (512, 17)]


def test_wide_layer_uses_band_tiles_and_every_band_shape_matches_oracle(orc):
    """A 257 x 257 layer does not fit a whole-layer tile: the grid switches to
    band tiles by itself; every compiled band shape gives the oracle's J, and
    layer-tile-only shapes are refused."""
    import paper_2102_01734_amd as rt
    case = sy.random_box(257, 257, 4, 4, 8, seed=19, dtype="f32")
    S = sy.random_source(case.chi.shape, seed=20, dtype="f32")
    g = make_grid(case)
    assert g.launch_shape()["band"]
    Jo, Lo = _oracle_fs(orc, case, S, "linear")
    J, L = gpu_fs(case, S, grid=g)
    np.testing.assert_allclose(J, Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
    np.testing.assert_allclose(L, Lo, rtol=5e-6, atol=1e-8)
    for threads, rays in BAND_TUNE:
        print(f"band shape {threads} x {rays}", flush=True)
        g.set_launch_shape(threads, rays)
        ls = g.launch_shape()
        assert (ls["threads"], ls["rays"], ls["band"]) == (threads, rays, True)
        J1, _ = gpu_fs(case, S, grid=g, want_lstar=False)
        np.testing.assert_allclose(J1, Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
    with pytest.raises(rt.RtError):
        g.set_launch_shape(256, 5)    # compiled for layer tiles only
    g.close()


def test_band_autotune_keeps_results():
    case = sy.random_box(257, 257, 3, 2, 4, seed=21, dtype="f32")
    S = sy.random_source(case.chi.shape, seed=22, dtype="f32")
    g = make_grid(case)
    J0, _ = gpu_fs(case, S, grid=g, want_lstar=False)
    threads, rays = g.autotune(to_dev(case.chi, "f32"), to_dev(S, "f32"))
    ls = g.launch_shape()
    assert ls["band"] and (ls["threads"], ls["rays"]) == (threads, rays)
    J1, _ = gpu_fs(case, S, grid=g, want_lstar=False)
    g.close()
    np.testing.assert_allclose(J1, J0, rtol=2e-6, atol=1e-7 * np.abs(J0).max())


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_band_shape_on_a_layer_grid(orc, prec):
    """A grid whose layer fits a whole-layer tile can still run band tiles (the
    autotuner times both kinds): a shape compiled for both kinds is set with
    its kind named, matches the oracle, and is reproduced bitwise on a second
    grid; whole-layer tiles are refused on a grid that needs bands."""
    import paper_2102_01734_amd as rt
    case = sy.random_box(31, 23, 9, 4, 8, seed=23, dtype=prec)
    S = sy.random_source(case.chi.shape, seed=24, dtype=prec)
    Jo, _ = _oracle_fs(orc, case, S, "linear")
    tol = dict(rtol=1e-12) if prec == "f64" else dict(rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
    out = []
    for band in (False, True, True):
        g = make_grid(case)
        assert not g.launch_shape()["band"]
        g.set_launch_shape(1024, 2, band=band)
        ls = g.launch_shape()
        assert (ls["threads"], ls["rays"], ls["band"]) == (1024, 2, band)
        J, _ = gpu_fs(case, S, grid=g, want_lstar=False)
        g.close()
        np.testing.assert_allclose(J, Jo, **tol)
        out.append(J)
    assert np.array_equal(out[1], out[2])
    g = make_grid(case)
    g.set_launch_shape(1024, 2)               # unnamed kind: the grid's own (whole layers)
    assert not g.launch_shape()["band"]
    g.close()
    gb = make_grid(case, band_tiles=True)
    with pytest.raises(rt.RtError):
        gb.set_launch_shape(1024, 2, band=False)
    gb.close()


def test_band_tiles_refused_when_a_row_band_cannot_fit():
    """64 polar angles reach 45 rows per layer: 1000-voxel rows leave no band
    that fits the LDS of a CU, so the grid is refused (nothing launched)."""
    import paper_2102_01734_amd as rt
    with pytest.raises(rt.RtError) as e:
        rt.Grid(1000, 200, 2, 64, 4, "f32")
    assert e.value.status == rt.rt3d.RT_E_UNSUPPORTED


def test_band_flag_rejected_on_spherical_grids():
    import paper_2102_01734_amd as rt
    d = rt.rt3d.sphere_desc(9, 7, 8, 1.0, 2.0, 4, 4, "f64", 1)
    d.flags |= rt.rt3d.RT_F_BAND_TILES
    with pytest.raises(rt.RtError) as e:
        rt.rt3d.rt_create_grid(d)
    assert e.value.status == rt.rt3d.RT_E_INVALID


def test_fs_257_lognormal_sampled(orc):
    """The 257^3 box, 32x16 directions, single precision (band tiles), checked at
    sampled voxels computed one by one by the oracle."""
    case = sy.box_lognormal257()
    S = sy.random_source(case.chi.shape, seed=23, lo=0.2, hi=1.0, dtype="f32")
    print("fs 257^3 x 512 f32", flush=True)
    g = make_grid(case)
    assert g.launch_shape()["band"]
    J, L = gpu_fs(case, S, grid=g)
    g.close()
    rng = np.random.default_rng(24)
    n = case.n_vox
    NxNy = case.Nx * case.Ny
    vox = np.unique(np.concatenate([[0, n - 1, NxNy - 1, n - NxNy, 128 * NxNy + 128 * case.Nx + 128],
                                    rng.integers(0, n, 12)]))
    Jo, Lo = orc.fs_box_sampled(case.chi[0], S[0], case.I_bc[0, 0], case.I_bc[0, 1], case.n_mu, case.n_phi, vox)
    np.testing.assert_allclose(J[0].ravel()[vox], Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
    np.testing.assert_allclose(L[0].ravel()[vox], Lo, rtol=5e-6, atol=1e-8)
    assert np.all(np.isfinite(J)) and np.all((L > 0) & (L <= 1))
