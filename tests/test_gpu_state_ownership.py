"""A grid's per-state scratch (padded inputs, Ng history, double anchor,
nearest-neighbour stencil) follows the state being stepped, and grids too
large for the device are refused before anything is allocated.

* Two states stepped alternately on one grid give the iterates of two grids
  stepping one state each (Ng off, so that the restarted Ng history of a
  switch does not change the path): the stencil, padded inputs and S are
  rebuilt from the state at every switch.  With Ng on, both still reach their
  own LU fixed point (Sec. 2.2: the fixed point does not depend on the path).
* BiCGStab leaves Lambda* valid but builds no stencil; the ALI steps after it
  on a non-local grid build the stencil themselves and follow the iterates of
  a fresh grid started from the BiCGStab result.
"""
import numpy as np
import pytest

import synthetic as sy
from tests.gpu_helpers import to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _grid(case, prec, nonlocal_lstar):
    import paper_2102_01734_amd as rt
    return rt.Grid(case.Nx, case.Ny, case.Nz, case.n_mu, case.n_phi, prec, case.n_lambda,
                   nonlocal_lstar=nonlocal_lstar)


def _state(g, case, prec, J0=None):
    return g.new_state(to_dev(case.chi, prec), to_dev(case.eps, prec), to_dev(case.B, prec),
                       to_dev(case.I_bc, prec), J0=J0)


def _cases(prec):
    a = sy.random_box(13, 11, 7, 4, 8, seed=61, dtype=prec, eps_dex=(-3, -1))
    b = sy.random_box(13, 11, 7, 4, 8, seed=62, dtype=prec, eps_dex=(-3, -1))
    return a, b


@pytest.mark.parametrize("nonlocal_lstar", [False, True])
def test_two_states_alternating_equal_separate_grids(nonlocal_lstar):
    torch = torch_cuda()
    ca, cb = _cases("f64")
    print(f"alternating states, nonlocal={nonlocal_lstar}", flush=True)
    opts_kw = dict(tol=1e-30, max_iter=1, ng_every=0, os_sweeps=4)
    shared = _grid(ca, "f64", nonlocal_lstar)
    sa, sb = _state(shared, ca, "f64"), _state(shared, cb, "f64")
    for _ in range(10):
        shared.ali_step(sa, shared.opts(**opts_kw))
        shared.ali_step(sb, shared.opts(**opts_kw))
    torch.cuda.synchronize()
    out = {}
    for name, case in (("a", ca), ("b", cb)):
        g = _grid(case, "f64", nonlocal_lstar)
        st = _state(g, case, "f64")
        for _ in range(10):
            g.ali_step(st, g.opts(**opts_kw))
        torch.cuda.synchronize()
        out[name] = g.state_tensors(st)["J"].cpu().numpy()
        g.close()
    Ja = shared.state_tensors(sa)["J"].cpu().numpy()
    Jb = shared.state_tensors(sb)["J"].cpu().numpy()
    shared.close()
    np.testing.assert_allclose(Ja, out["a"], rtol=1e-10)
    np.testing.assert_allclose(Jb, out["b"], rtol=1e-10)


@pytest.mark.parametrize("prec,nonlocal_lstar", [("f64", False), ("f64", True), ("f32", True)])
def test_two_states_alternating_reach_their_fixed_points(orc, prec, nonlocal_lstar):
    """Alternating rt_solve calls of three steps each, Ng on, to convergence."""
    torch = torch_cuda()
    ca, cb = _cases(prec)
    print(f"alternating solves {prec} nonlocal={nonlocal_lstar}", flush=True)
    g = _grid(ca, prec, nonlocal_lstar)
    sa, sb = _state(g, ca, prec), _state(g, cb, prec)
    tol = 1e-12 if prec == "f64" else 1e-9
    done = {"a": False, "b": False}
    for _ in range(200):
        for name, st in (("a", sa), ("b", sb)):
            if not done[name]:
                status, _ = g.solve(st, g.opts(tol=tol, max_iter=3))
                done[name] = status == 0
        if all(done.values()):
            break
    torch.cuda.synchronize()
    assert all(done.values())
    for case, st in ((ca, sa), (cb, sb)):
        prob = orc.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8)
        ref = orc.direct(prob)["J"]
        J = g.state_tensors(st)["J"].cpu().numpy()[0]
        err = float(np.max(np.abs(J - ref) / ref))
        print(f"  fixed-point error {err:.2e}")
        assert err < (1e-9 if prec == "f64" else 1e-5)
    g.close()


def test_bicgstab_then_nonlocal_ali_builds_the_stencil():
    import paper_2102_01734_amd as rt
    torch = torch_cuda()
    case = sy.random_box(15, 13, 8, 4, 8, seed=63, dtype="f64", eps_dex=(-4, -1))
    print("BiCGStab then non-local ALI", flush=True)
    g = _grid(case, "f64", True)
    st = _state(g, case, "f64")
    status, _ = g.solve(st, g.opts(tol=1e-14, max_iter=2, method="bicgstab"))
    assert status in (rt.rt3d.RT_OK, rt.rt3d.RT_E_NOT_CONVERGED)
    torch.cuda.synchronize()
    assert st.lstar_valid == 1 and st.iter == 0
    J_start = g.state_tensors(st)["J"].clone()
    opts_kw = dict(tol=1e-30, max_iter=1, ng_every=0, os_sweeps=6)
    for _ in range(8):
        g.ali_step(st, g.opts(**opts_kw))
    torch.cuda.synchronize()
    J = g.state_tensors(st)["J"].cpu().numpy()
    g.close()
    # reference: a fresh non-local grid from the same J, building Lambda* and the stencil itself
    g2 = _grid(case, "f64", True)
    st2 = _state(g2, case, "f64", J0=J_start)
    for _ in range(8):
        g2.ali_step(st2, g2.opts(**opts_kw))
    torch.cuda.synchronize()
    J2 = g2.state_tensors(st2)["J"].cpu().numpy()
    g2.close()
    assert np.all(np.isfinite(J))
    np.testing.assert_allclose(J, J2, rtol=1e-10)


def test_oversized_grid_refused_before_allocating():
    import paper_2102_01734_amd as rt
    torch = torch_cuda()
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    desc = rt.rt3d.box_desc(129, 129, 129, 2, 2, "f64", 16384)
    with pytest.raises(rt.RtError) as e:
        rt.rt3d.rt_create_grid(desc)
    assert e.value.status == rt.rt3d.RT_E_NOMEM
    assert "GB" in str(e.value)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert abs(free1 - free0) < (64 << 20)
    # a grid that fits is still created and works
    desc.n_lambda_max = 1
    h = rt.rt3d.rt_create_grid(desc)
    rt.rt3d.rt_destroy_grid(h)
