"""Parity of the HIP formal solution (rt_formal_solution) with the oracle.

Tolerances:
* double-precision grids: the kernel and the oracle take identical optical
  steps and identical fallback decisions; they differ only in how exp and the
  weights are rounded (a few ulp per point), so J and Lambda* agree to 1e-12.
* single-precision grids: the recurrence and the J accumulation are float;
  per point the intensity picks up a relative error of a few 2^-24 and the
  attenuation damps older errors, so J stays within ~1e-6 of the double
  result; the tests allow 5e-6 relative (plus 1e-7 of max|J| absolute, for
  the faint voxels next to the unlit top boundary).
"""
import numpy as np
import pytest

import synthetic as sy
from tests.gpu_helpers import gpu_fs, make_grid, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _oracle_fs(orc, case, S, kind):
    Js, Ls = [], []
    for l in range(case.n_lambda):
        J, L = orc.fs_box(case.chi[l], S[l], case.I_bc[l, 0], case.I_bc[l, 1], case.n_mu, case.n_phi, kind=kind)
        Js.append(J); Ls.append(L)
    return np.array(Js), np.array(Ls)


SHAPES = [  # (Nx, Ny, Nz, n_mu, n_phi): ragged sizes, several workgroups, one voxel column
    (7, 5, 6, 4, 8),
    (17, 13, 9, 4, 8),
    (33, 33, 12, 8, 16),
    (9, 9, 1, 2, 4),
    (1, 1, 7, 4, 4),
    (70, 3, 5, 4, 8),
]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["linear", "parabolic"])
def test_fs_fp64_matches_oracle(orc, shape, kind):
    Nx, Ny, Nz, n_mu, n_phi = shape
    print(f"fs fp64 {shape} {kind}", flush=True)
    case = sy.random_box(Nx, Ny, Nz, n_mu, n_phi, seed=Nx * 7 + Nz, dtype="f64")
    S = sy.random_source(case.chi.shape, seed=3)
    J, L = gpu_fs(case, S, lstar=kind)
    Jo, Lo = _oracle_fs(orc, case, S, kind)
    np.testing.assert_allclose(J, Jo, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(L, Lo, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("shape", SHAPES[:4])
def test_fs_fp32_matches_oracle(orc, shape):
    Nx, Ny, Nz, n_mu, n_phi = shape
    print(f"fs fp32 {shape}", flush=True)
    case = sy.random_box(Nx, Ny, Nz, n_mu, n_phi, seed=Nx + 100 * Nz, dtype="f32")
    S = sy.random_source(case.chi.shape, seed=4, dtype="f32")
    J, L = gpu_fs(case, S)
    Jo, Lo = _oracle_fs(orc, case, S, "linear")
    print("max rel err J", float(np.max(np.abs(J - Jo) / np.abs(Jo))), "Lambda*", float(np.max(np.abs(L - Lo) / Lo)))
    np.testing.assert_allclose(J, Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
    np.testing.assert_allclose(L, Lo, rtol=5e-6, atol=1e-8)


def test_fs_vacuum_and_opaque_voxels(orc):
    """chi = 0 (vacuum: no change of I) and very opaque voxels side by side."""
    case = sy.random_box(11, 9, 8, 4, 8, seed=5, dtype="f64")
    rng = np.random.default_rng(0)
    mask = rng.random(case.chi.shape) < 0.2
    case.chi[mask] = 0.0
    case.chi[rng.random(case.chi.shape) < 0.1] = 1e6
    S = sy.random_source(case.chi.shape, seed=6)
    J, L = gpu_fs(case, S, lstar="parabolic")
    Jo, Lo = _oracle_fs(orc, case, S, "parabolic")
    np.testing.assert_allclose(J, Jo, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(L, Lo, rtol=1e-12, atol=1e-14)


def test_fs_stratified_slab_fp64(orc):
    """The 33^3 stratified slab (tau 1e-4..1e4, 8x16 directions): J equals the
    oracle's layer reduction in every column."""
    case = sy.box_stratified()
    S = np.broadcast_to(np.linspace(0.1, 1.0, case.Nz)[None, :, None, None], case.chi.shape).copy()
    J, L = gpu_fs(case, S)
    J1, L1 = orc.fs_1d(case.chi[0, :, 0, 0], S[0, :, 0, 0], 0.0, 1.0, case.n_mu, case.n_phi)
    np.testing.assert_allclose(J[0], np.broadcast_to(J1[:, None, None], J[0].shape), rtol=1e-12)
    np.testing.assert_allclose(L[0], np.broadcast_to(L1[:, None, None], L[0].shape), rtol=1e-12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fs_batch_equals_single_wavelengths_bitwise(prec):
    case = sy.random_box(13, 11, 7, 4, 8, seed=9, dtype=prec, n_lambda=3)
    S = sy.random_source(case.chi.shape, seed=10, dtype=prec)
    Jb, Lb = gpu_fs(case, S)
    for l in range(3):
        one = sy.random_box(13, 11, 7, 4, 8, seed=9, dtype=prec, n_lambda=3)
        one.chi, one.I_bc = case.chi[l:l + 1], case.I_bc[l:l + 1]
        one.eps, one.B = case.eps[l:l + 1], case.B[l:l + 1]
        J1, L1 = gpu_fs(one, S[l:l + 1])
        assert np.array_equal(J1[0], Jb[l])
        assert np.array_equal(L1[0], Lb[l])


def test_fs_deterministic():
    case = sy.random_box(33, 33, 16, 8, 16, seed=11, dtype="f32")
    S = sy.random_source(case.chi.shape, seed=12, dtype="f32")
    g = make_grid(case)
    a = gpu_fs(case, S, grid=g)
    b = gpu_fs(case, S, grid=g)
    g.close()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_fs_zero_wavelengths_and_invalid_arguments():
    import paper_2102_01734_amd as rt
    torch = torch_cuda()
    case = sy.random_box(5, 5, 5, 4, 8, seed=1, dtype="f32")
    g = make_grid(case)
    chi = to_dev(case.chi, "f32")
    J = torch.zeros_like(chi)
    rt.rt_formal_solution(g.handle, 0, chi.data_ptr(), chi.data_ptr(), None, J.data_ptr(), None, None)
    assert float(J.abs().max()) == 0.0
    with pytest.raises(rt.RtError) as e:
        rt.rt_formal_solution(g.handle, 2, chi.data_ptr(), chi.data_ptr(), None, J.data_ptr(), None, None)
    assert e.value.status == rt.rt3d.RT_E_INVALID
    with pytest.raises(rt.RtError):
        rt.rt_formal_solution(g.handle, 1, None, chi.data_ptr(), None, J.data_ptr(), None, None)
    g.close()
    with pytest.raises(rt.RtError):
        rt.Grid(5, 5, 5, 3, 8)          # odd n_mu
    with pytest.raises(rt.RtError):
        rt.Grid(0, 5, 5, 4, 8)


def test_fs_full_size_lognormal_sampled(orc):
    """129^3 box, 32x64 directions, log-normal opacity, single precision: the
    launch the benchmark times, checked at sampled voxels computed one by one
    by the oracle."""
    case = sy.box_lognormal()
    S = sy.random_source(case.chi.shape, seed=77, lo=0.2, hi=1.0, dtype="f32")
    print("fs full-size 129^3 x 2048 f32", flush=True)
    J, L = gpu_fs(case, S)
    rng = np.random.default_rng(5)
    n = case.n_vox
    vox = np.unique(np.concatenate([[0, n - 1, case.Nx * case.Ny - 1, n - case.Nx * case.Ny],
                                    rng.integers(0, n, 20)]))
    Jo, Lo = orc.fs_box_sampled(case.chi[0], S[0], case.I_bc[0, 0], case.I_bc[0, 1], case.n_mu, case.n_phi, vox)
    np.testing.assert_allclose(J[0].ravel()[vox], Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
    np.testing.assert_allclose(L[0].ravel()[vox], Lo, rtol=5e-6, atol=1e-8)
    assert np.all(np.isfinite(J)) and np.all((L > 0) & (L < 1))


def test_autotune_keeps_results(orc):
    """The shape the autotuner picks changes only the grouping of directions into
    partial sums: J agrees to single-precision rounding."""
    torch = torch_cuda()
    case = sy.random_box(40, 37, 9, 4, 8, seed=81, dtype="f32")
    S = sy.random_source(case.chi.shape, seed=82, dtype="f32")
    g = make_grid(case)
    J0, _ = gpu_fs(case, S, grid=g, want_lstar=False)
    threads, rays = g.autotune(to_dev(case.chi, "f32"), to_dev(S, "f32"))
    ls = g.launch_shape()
    assert (ls["threads"], ls["rays"]) == (threads, rays)
    if not ls["band"]:     # whole-layer tiles: the bundles hold every ray of a direction
        assert threads * rays * ls["bundles"] >= case.Nx * case.Ny
    J1, _ = gpu_fs(case, S, grid=g, want_lstar=False)
    g.close()
    np.testing.assert_allclose(J1, J0, rtol=2e-6, atol=1e-7 * np.abs(J0).max())


def test_set_launch_shape(orc):
    """A fixed compiled shape gives the same J as the default one up to the
    summation order; shapes that are not compiled or cannot hold a direction's
    rays are rejected."""
    import paper_2102_01734_amd as rt
    case = sy.random_box(40, 37, 9, 4, 8, seed=83, dtype="f32")
    S = sy.random_source(case.chi.shape, seed=84, dtype="f32")
    g = make_grid(case)
    J0, _ = gpu_fs(case, S, grid=g, want_lstar=False)
    g.set_launch_shape(768, 2)
    J1, _ = gpu_fs(case, S, grid=g, want_lstar=False)
    np.testing.assert_allclose(J1, J0, rtol=2e-6, atol=1e-7 * np.abs(J0).max())
    with pytest.raises(rt.RtError):
        g.set_launch_shape(256, 5)       # 1280 rays < 40 x 37
    with pytest.raises(rt.RtError):
        g.set_launch_shape(100, 3)       # not compiled
    g.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_largest_layer_tile(orc, prec):
    """140 x 140 = 19600 voxels per layer is the largest square layer whose
    double tile (plus one scratch word for each of the 832 threads that hold
    its rays, 24 per thread) fits the 160 KiB of LDS of a CU: it runs on
    layer tiles and matches the oracle; 141 x 141 refuses layer tiles and runs
    on band tiles (the default of both, whose layer-tile kernels of so many
    rays per thread spill registers) and matches the oracle as well."""
    import paper_2102_01734_amd as rt
    for N, band in ((140, False), (141, True)):
        case = sy.random_box(N, N, 3, 2, 4, seed=61, dtype=prec)
        S = sy.random_source(case.chi.shape, seed=62, dtype=prec)
        print(f"largest tile {prec} {N}", flush=True)
        g = make_grid(case)
        assert g.launch_shape()["band"]
        if band:
            with pytest.raises(rt.RtError):
                g.set_launch_shape(1024, 24, band=False)
        else:
            g.set_launch_shape(1024, 24, band=False)
            ls = g.launch_shape()
            assert (ls["threads"], ls["rays"], ls["band"]) == (1024, 24, False)
        J, L = gpu_fs(case, S, grid=g)
        g.close()
        Jo, Lo = _oracle_fs(orc, case, S, "linear")
        tol = 1e-12 if prec == "f64" else 5e-6
        np.testing.assert_allclose(J, Jo, rtol=tol, atol=tol * 0.02 * np.abs(Jo).max())
        np.testing.assert_allclose(L, Lo, rtol=tol, atol=tol * 0.002)


def test_batched_64_wavelengths_full_size_sampled(orc):
    """The 64-wavelength batch on the 129^3 box (32x32 directions, single
    precision) in one launch: three wavelengths checked against the oracle at
    sampled voxels, computed one by one."""
    case = sy.box_batched()
    S = sy.random_source(case.chi.shape[1:], seed=63, lo=0.2, hi=1.0, dtype="f32")
    S = np.broadcast_to(S, case.chi.shape)
    print("batched 64 x 129^3 x 1024 f32", flush=True)
    J, L = gpu_fs(case, S)
    rng = np.random.default_rng(8)
    vox = np.unique(rng.integers(0, case.n_vox, 12))
    for l in (0, 37, 63):
        Jo, Lo = orc.fs_box_sampled(case.chi[l], S[l], case.I_bc[l, 0], case.I_bc[l, 1], case.n_mu, case.n_phi, vox)
        np.testing.assert_allclose(J[l].ravel()[vox], Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
        np.testing.assert_allclose(L[l].ravel()[vox], Lo, rtol=5e-6, atol=1e-8)


@pytest.mark.parametrize("prec,shape", [("f32", (512, 3)), ("f32", (512, 17)), ("f64", (512, 3)), ("f64", (512, 17))])
def test_ray_bundle_shapes_match_single_workgroup_sweeps(orc, prec, shape):
    """Shapes that split each direction's rays into two bundles (two workgroups
    and two layer tiles per direction) give the oracle's J; against the default
    one-workgroup sweep they differ only in the summation order."""
    Nx, Ny = (40, 37) if shape[1] < 10 else (129, 129)
    case = sy.random_box(Nx, Ny, 6, 4, 8, seed=85, dtype=prec)
    S = sy.random_source(case.chi.shape, seed=86, dtype=prec)
    g = make_grid(case)
    J0, _ = gpu_fs(case, S, grid=g, want_lstar=False)
    g.set_launch_shape(*shape)
    J1, _ = gpu_fs(case, S, grid=g, want_lstar=False)
    g.close()
    tol = 1e-14 if prec == "f64" else 2e-6
    np.testing.assert_allclose(J1, J0, rtol=tol, atol=tol * np.abs(J0).max())
    Jo, _ = _oracle_fs(orc, case, S, "linear")
    np.testing.assert_allclose(J1, Jo, rtol=1e-12 if prec == "f64" else 5e-6,
                               atol=(1e-14 if prec == "f64" else 1e-7) * np.abs(Jo).max())


# Launch shapes of the single-precision sweep that the autotuner chooses among
# on the 129^3 workloads (row-band tiles; threads, rays per thread): the timed
# benchmark lines run 768 x 11 with two bundles.
TIMED_SHAPES = [(768, 11), (768, 10), (896, 10), (512, 7)]


@pytest.fixture(scope="module")
def full_size_case(orc):
    """129^3 x 2048 log-normal workload, a source field, and the oracle's J and
    Lambda* at 1028 voxels: the four x/y corners (where rays wrap round the
    period) of every layer, plus 512 random voxels."""
    case = sy.box_lognormal()
    S = sy.random_source(case.chi.shape, seed=77, lo=0.2, hi=1.0, dtype="f32")
    N = case.Nx
    k = np.arange(case.Nz)[:, None]
    corners = np.array([0, N - 1, (N - 1) * N, N * N - 1])[None, :]
    vox = (k * N * N + corners).ravel()
    rng = np.random.default_rng(5)
    vox = np.unique(np.concatenate([vox, rng.integers(0, case.n_vox, 512)]))
    print(f"oracle at {vox.size} voxels of 129^3 x 2048", flush=True)
    Jo, Lo = orc.fs_box_sampled(case.chi[0], S[0], case.I_bc[0, 0], case.I_bc[0, 1], case.n_mu, case.n_phi, vox)
    return case, S, vox, Jo, Lo


@pytest.mark.parametrize("shape", TIMED_SHAPES)
def test_fs_full_size_at_timed_shapes(full_size_case, shape):
    """The benchmark's 129^3 x 2048 single-precision launch at the band shapes
    the autotuner picks from, against the oracle at every layer's wrap corners
    and at random voxels."""
    case, S, vox, Jo, Lo = full_size_case
    print(f"fs full-size 129^3 x 2048 f32 at {shape} band", flush=True)
    g = make_grid(case)
    g.set_launch_shape(*shape, band=True)
    J, _ = gpu_fs(case, S, grid=g, want_lstar=False)   # the J-only sweep runs the set shape
    ls = g.launch_shape()
    g.close()
    assert (ls["threads"], ls["rays"], ls["band"]) == (*shape, 1)
    Jg = J[0].ravel()[vox]
    print(f"  {ls['bundles']} bundles: max rel err J {float(np.max(np.abs(Jg - Jo) / np.abs(Jo))):.2e}")
    np.testing.assert_allclose(Jg, Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
    assert np.all(np.isfinite(J))


def test_batched_64_wavelengths_at_the_timed_shape(orc):
    """The 64-wavelength batch (129^3, 32x32 directions, single precision) at
    the benchmark's launch shape (768 x 11, band tiles; J-only sweep): four
    wavelengths of very different opacity scale against the oracle at 256
    voxels each."""
    case = sy.box_batched()
    S = sy.random_source(case.chi.shape[1:], seed=63, lo=0.2, hi=1.0, dtype="f32")
    S = np.ascontiguousarray(np.broadcast_to(S, case.chi.shape))
    print("batched 64 x 129^3 x 1024 f32 at 768 x 11 band", flush=True)
    g = make_grid(case)
    g.set_launch_shape(768, 11, band=True)
    J, _ = gpu_fs(case, S, grid=g, want_lstar=False)
    g.close()
    rng = np.random.default_rng(9)
    vox = np.unique(rng.integers(0, case.n_vox, 256))
    for l in (0, 21, 42, 63):
        Jo, _ = orc.fs_box_sampled(case.chi[l], S[l], case.I_bc[l, 0], case.I_bc[l, 1], case.n_mu, case.n_phi, vox)
        Jg = J[l].ravel()[vox]
        print(f"  wavelength {l}: max rel err J {float(np.max(np.abs(Jg - Jo) / np.abs(Jo))):.2e}")
        np.testing.assert_allclose(Jg, Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())


def _compiled_shapes():
    """(threads, rays, band) of every compiled single-output sweep shape, read from the kernel source."""
    import os
    import re
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2102_01734_amd", "csrc", "fs_box.hip")).read()
    out = []
    for macro, band in (("RT_FS_SHAPES_FULL", False), ("RT_FS_SHAPES_TUNE", False),
                        ("RT_FS_SHAPES_BAND_FULL", True), ("RT_FS_SHAPES_BAND_TUNE", True)):
        text = re.search(r"#define " + macro + r"\(X\)(.*?)(?=\n#define|\nstatic const)", src, re.S).group(1)
        for lb, r, _ in re.findall(r"X\((\d+),\s*(\d+),\s*(\d+)\)", text):
            out.append((int(lb), int(r), band))
    return sorted(set(out))


@pytest.mark.gpu
@pytest.mark.parametrize("dims", [(37, 29, 3), (97, 89, 3), (160, 158, 3)])
def test_every_compiled_shape_matches_oracle(orc, dims):
    """Every compiled launch shape that can hold a direction's rays on this grid
    (single precision, J only), and the default J + Lambda* sweep, give the
    oracle's results: each kernel instantiation is run, not only the shapes the
    autotuner or the defaults pick."""
    import paper_2102_01734_amd as rt
    Nx, Ny, Nz = dims
    case = sy.random_box(Nx, Ny, Nz, 2, 4, seed=97, dtype="f32")
    S = sy.random_source(case.chi.shape, seed=98, dtype="f32")
    Jo, Lo = _oracle_fs(orc, case, S, "linear")
    g = make_grid(case)
    J, L = gpu_fs(case, S, grid=g)
    np.testing.assert_allclose(J, Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
    np.testing.assert_allclose(L, Lo, rtol=5e-6, atol=1e-8)
    ran = 0
    for threads, rays, band in _compiled_shapes():
        try:
            g.set_launch_shape(threads, rays, band=band)
        except rt.RtError:
            continue  # this grid's rays do not fit the shape (or layer tiles where bands are needed)
        print(f"shape {threads} x {rays} {'band' if band else 'layer'}", flush=True)
        J1, _ = gpu_fs(case, S, grid=g, want_lstar=False)
        np.testing.assert_allclose(J1, Jo, rtol=5e-6, atol=1e-7 * np.abs(Jo).max())
        ran += 1
    g.close()
    assert ran >= 4
