"""rt_formal_solution_noalloc (scratch in a fixed device array, no device
allocation) against rt_formal_solution on the same inputs, through the C ABI.

The two entry points run the same kernels; the no-allocation one may launch
fewer persistent workgroups (its partial sums must fit the fixed array), so
the results agree up to the summation order: 1e-12 relative in double
precision, 1e-6 in single precision (sums of a few hundred float partials).
Two calls in a row, the second on a smaller input, check that nothing left in
the shared array from the first call leaks into the second.
"""
import numpy as np
import pytest

import synthetic as sy
from tests.gpu_helpers import to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _both(g, case, prec, n_lambda, want_lstar):
    import paper_2102_01734_amd as rt
    torch = torch_cuda()
    chi = to_dev(case.chi[:n_lambda], prec)
    S = to_dev(sy.random_source(case.chi[:n_lambda].shape, seed=case.Nx + n_lambda, dtype=prec), prec)
    Ib = to_dev(case.I_bc[:n_lambda], prec)
    out = []
    for fn in (rt.rt3d.rt_formal_solution, rt.rt3d.rt_formal_solution_noalloc):
        J = torch.full_like(chi, float("nan"))
        L = torch.full_like(chi, float("nan")) if want_lstar else None
        fn(g.handle, n_lambda, chi.data_ptr(), S.data_ptr(), Ib.data_ptr(), J.data_ptr(),
           L.data_ptr() if L is not None else None, None)
        torch.cuda.synchronize()
        out.append((J.double().cpu().numpy(), L.double().cpu().numpy() if L is not None else None))
    return out


def _check(out, prec):
    (J0, L0), (J1, L1) = out
    rtol = 1e-12 if prec == "f64" else 1e-6
    assert np.all(np.isfinite(J1))
    np.testing.assert_allclose(J1, J0, rtol=rtol, atol=1e-300)
    if L0 is not None:
        assert np.all(np.isfinite(L1))
        np.testing.assert_allclose(L1, L0, rtol=rtol, atol=1e-300)


@pytest.mark.parametrize("prec,band", [("f64", False), ("f32", False), ("f32", True)])
def test_noalloc_matches_formal_solution_two_calls(prec, band):
    import paper_2102_01734_amd as rt
    big = sy.random_box(24, 20, 10, 4, 8, seed=71, dtype=prec, n_lambda=3)
    small = sy.random_box(11, 9, 6, 4, 8, seed=72, dtype=prec, n_lambda=1)
    print(f"no-alloc {prec} band={band}: 24x20x10 x3 with Lambda*, then 11x9x6 x1", flush=True)
    g1 = rt.Grid(24, 20, 10, 4, 8, prec, 3, band_tiles=band)
    _check(_both(g1, big, prec, 3, True), prec)
    g2 = rt.Grid(11, 9, 6, 4, 8, prec, 1, band_tiles=band)
    _check(_both(g2, small, prec, 1, False), prec)
    g1.close()
    g2.close()


def test_noalloc_fewer_workgroups_when_partials_do_not_fit():
    """64 x 64 x 32 voxels in double precision: a slot is 1 MB, so the fixed
    array holds far fewer slots than the grid's resident workgroups."""
    import paper_2102_01734_amd as rt
    case = sy.random_box(64, 64, 32, 4, 8, seed=73, dtype="f64")
    print("no-alloc 64x64x32 f64 (reduced workgroups)", flush=True)
    g = rt.Grid(64, 64, 32, 4, 8, "f64", 1)
    assert g.info()["n_workgroups"] * 64 * 64 * 32 * 8 > rt.rt3d.RT_NOALLOC_SCRATCH_BYTES
    _check(_both(g, case, "f64", 1, True), "f64")
    _check(_both(g, case, "f64", 1, False), "f64")
    g.close()


def test_noalloc_refuses_oversized_input_before_launching():
    import paper_2102_01734_amd as rt
    torch = torch_cuda()
    print("no-alloc refusal 129x129x129 f32", flush=True)
    g = rt.Grid(129, 129, 129, 2, 2, "f32", 1)
    chi = torch.ones((1, 129, 129, 129), dtype=torch.float32, device="cuda")
    J = torch.zeros_like(chi)
    with pytest.raises(rt.RtError) as e:
        rt.rt3d.rt_formal_solution_noalloc(g.handle, 1, chi.data_ptr(), chi.data_ptr(), None, J.data_ptr(), None,
                                           None)
    assert e.value.status == rt.rt3d.RT_E_INVALID
    torch.cuda.synchronize()
    assert float(J.abs().max()) == 0.0
    g.close()
