"""The BiCGStab outer solver (rt_solve with method "bicgstab") reaches the
oracle's LU fixed point on box and spherical grids."""
import numpy as np
import pytest

import synthetic as sy
from tests.gpu_helpers import make_grid, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _solve(case, prec, tol=1e-12, max_iter=500):
    torch = torch_cuda()
    g = make_grid(case, prec=prec)
    st = g.new_state(*(to_dev(a, prec) for a in (case.chi, case.eps, case.B, case.I_bc)))
    status, rep = g.solve(st, g.opts(tol=tol, max_iter=max_iter, method="bicgstab"))
    torch.cuda.synchronize()
    out = g.state_tensors(st)
    J, S = out["J"].cpu().numpy(), out["S"].cpu().numpy()
    g.close()
    return status, rep, J, S


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bicgstab_box_matches_lu(orc, prec):
    case = sy.random_box(7, 7, 5, 4, 8, seed=101, dtype=prec, eps_dex=(-4, -1))
    if prec == "f32":  # the boundary intensities reach a single-precision grid rounded to float
        case.I_bc = case.I_bc.astype(np.float32).astype(np.float64)
    prob = orc.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8)
    ref = orc.direct(prob)
    status, rep, J, S = _solve(case, prec)
    # every formal solution is double precision but, on single-precision grids, the Lambda* pass
    assert status == 0 and rep.iters < 60 and rep.n_fs - rep.n_fs64 == (1 if prec == "f32" else 0)
    np.testing.assert_allclose(J[0], ref["J"], rtol=1e-10)
    np.testing.assert_allclose(S[0], (1 - case.eps[0]) * J[0] + case.eps[0] * case.B[0], rtol=1e-14)


def test_bicgstab_sphere_matches_lu(orc):
    case = sy.random_sphere(6, 5, 7, 4, 8, seed=102, dtype="f64")
    g = orc.SphereGrid(6, 5, 7, 1.0, 2.0)
    I_out, I_core, J_sub = case.I_bc[0]
    prob = orc.SphereProblem(g, case.chi[0].ravel(), case.eps[0].ravel(), case.B[0].ravel(), I_out, I_core, 4, 8,
                             dsrc=case.source_distance, J_sub=J_sub)
    ref = orc.direct(prob)
    status, rep, J, _ = _solve(case, "f64")
    assert status == 0
    np.testing.assert_allclose(J[0], ref["J"], rtol=1e-10)


def test_bicgstab_batch_and_limits(orc):
    """Wavelengths of very different conditioning converge independently in one
    batch; too few iterations report not-converged with a valid state."""
    import paper_2102_01734_amd as rt
    case = sy.random_box(8, 8, 6, 4, 8, seed=103, dtype="f64", n_lambda=3)
    case.chi = case.chi * np.array([1e-2, 1.0, 1e2])[:, None, None, None]
    case.eps[:] = np.array([0.5, 1e-2, 1e-4])[:, None, None, None]
    status, rep, J, _ = _solve(case, "f64", tol=1e-12)
    assert status == 0 and rep.n_converged == 3
    for l in range(3):
        prob = orc.BoxProblem(case.chi[l], case.eps[l], case.B[l], case.I_bc[l, 0], case.I_bc[l, 1], 4, 8)
        np.testing.assert_allclose(J[l], orc.direct(prob)["J"], rtol=1e-9)
    status, rep, J2, _ = _solve(case, "f64", tol=1e-12, max_iter=2)
    assert status == rt.rt3d.RT_E_NOT_CONVERGED and np.all(np.isfinite(J2))
