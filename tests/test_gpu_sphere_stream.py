"""Streamed spherical geometry cache (RT_F_HOST_CACHE, the SmallGPU mode):
chunks kept in pinned host memory and copied to the GPU for every formal
solution through two staging buffers.  The kernels, chunks and their order
are those of the device-resident cache, so every result is bitwise equal to
it; the fixed point is checked against the oracle's LU solution as well."""
import numpy as np
import pytest

import synthetic as sy
from tests.gpu_helpers import gpu_fs, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _sphere(case, host_cache, n_lambda_max=None):
    import paper_2102_01734_amd as rt
    return rt.SphereGrid(case.Nr, case.Nt, case.Np, case.r_core, case.r_out, case.n_mu, case.n_phi, case.dtype,
                         n_lambda_max or case.n_lambda, source_distance=case.source_distance, host_cache=host_cache)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_streamed_cache_equals_resident_cache_bitwise(monkeypatch, prec):
    monkeypatch.setenv("RT3D_SPHERE_CHUNK_VISITS", "4000")   # many chunks: both staging buffers cycle
    case = sy.random_sphere(7, 6, 8, 4, 8, seed=71, dtype=prec, n_lambda=3)
    S = sy.random_source(case.chi.shape, seed=72, dtype=prec)
    gd = _sphere(case, False)
    gh = _sphere(case, True)
    assert gh.info()["n_workgroups"] > 3
    cd, ch = gd.cache_bytes(), gh.cache_bytes()
    assert cd["host"] == 0 and cd["device"] > 0
    assert ch["device"] == 0 and ch["host"] == cd["device"]
    Jd, Ld = gpu_fs(case, S, grid=gd)
    Jh, Lh = gpu_fs(case, S, grid=gh)
    Jh2, Lh2 = gpu_fs(case, S, grid=gh)          # a second pass reuses the staging buffers
    gd.close()
    gh.close()
    assert np.array_equal(Jh, Jd) and np.array_equal(Lh, Ld)
    assert np.array_equal(Jh2, Jd) and np.array_equal(Lh2, Ld)


def test_streamed_cache_ali_matches_resident_cache_and_lu(monkeypatch, orc):
    """Ng-ALI on a streamed cache (eager steps) follows the resident cache's
    trajectory (graph-captured steps) bitwise and ends at the LU fixed point."""
    torch = torch_cuda()
    monkeypatch.setenv("RT3D_SPHERE_CHUNK_VISITS", "3000")
    case = sy.random_sphere(6, 5, 7, 4, 8, seed=61, dtype="f64")
    out = []
    for host in (False, True):
        g = _sphere(case, host)
        st = g.new_state(to_dev(case.chi, "f64"), to_dev(case.eps, "f64"), to_dev(case.B, "f64"),
                         to_dev(case.I_bc, "f64"))
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            status, rep = g.solve(st, g.opts(tol=1e-12, max_iter=2000, use_graph=True), stream=s)
        s.synchronize()
        assert status == 0
        out.append((g.state_tensors(st)["J"].cpu().numpy(), rep.iters))
        g.close()
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])
    grid = orc.SphereGrid(6, 5, 7, 1.0, 2.0)
    I_out, I_core, J_sub = case.I_bc[0]
    prob = orc.SphereProblem(grid, case.chi[0].ravel(), case.eps[0].ravel(), case.B[0].ravel(), I_out, I_core,
                             4, 8, dsrc=case.source_distance, J_sub=J_sub)
    ref = orc.direct(prob)
    np.testing.assert_allclose(out[1][0][0], ref["J"], rtol=1e-9)


def test_host_cache_flag_is_sphere_only():
    import paper_2102_01734_amd as rt
    g = rt.Grid(5, 5, 3, 2, 4, "f64")
    d = g.desc
    g.close()
    d.flags |= rt.rt3d.RT_F_HOST_CACHE
    with pytest.raises(rt.RtError) as e:
        rt.rt3d.rt_create_grid(d)
    assert e.value.status == rt.rt3d.RT_E_INVALID
