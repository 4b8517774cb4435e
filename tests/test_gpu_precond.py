"""The learned ALI correction: bf16 matrix-core inference against a float
reference of the same weights, and the accept/reject logic inside rt_solve.

The reference forward below is written independently of the kernels (numpy,
float32 arithmetic) and rounds to bf16 exactly where the kernels store bf16:
matrix-core layer weights, every stored activation, the upsampled map.  The
remaining differences are float32 summation order and the resulting rare
bf16 rounding flips (2^-8 relative on single activations), hence 2e-2.
"""
import numpy as np
import pytest

import synthetic as sy
from paper_2102_01734_amd import precond
from tests.gpu_helpers import gpu_solve, make_grid, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def bf16(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32)


def conv3(x, W, b, stride):
    """x [Z][Y][X][Ci]; W [27][Co][Ci]; periodic in y, x; zero-padded in z."""
    Z, Y, X, _ = x.shape
    Zo, Yo, Xo = ((n + 1) // 2 for n in (Z, Y, X)) if stride == 2 else (Z, Y, X)
    xp = np.concatenate([x[:, -1:], x, x[:, :1]], axis=1)
    xp = np.concatenate([xp[:, :, -1:], xp, xp[:, :, :1]], axis=2)
    xp = np.pad(xp, ((1, 1), (0, 0), (0, 0), (0, 0)))
    out = np.zeros((Zo, Yo, Xo, W.shape[1]), np.float32)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                sl = xp[dz:dz + stride * (Zo - 1) + 1:stride, dy:dy + stride * (Yo - 1) + 1:stride,
                        dx:dx + stride * (Xo - 1) + 1:stride]
                out += sl @ W[(dz * 3 + dy) * 3 + dx].T
    return out + b


def up2(x, shape):
    for ax, (n_f, periodic) in zip((0, 1, 2), ((shape[0], False), (shape[1], True), (shape[2], True))):
        n_c = x.shape[ax]
        o = np.arange(n_f)
        i1 = (o + 1) // 2
        i1 = i1 % n_c if periodic else np.minimum(i1, n_c - 1)
        x = 0.5 * (np.take(x, o // 2, axis=ax) + np.take(x, i1, axis=ax))
    return x


def reference_forward(blob, f):
    C, convs = precond.unpack_blob(blob)
    L = len(C)
    it = iter(convs)
    relu = lambda a: np.maximum(a, 0.0)  # noqa: E731
    W, b = next(it)
    x = bf16(relu(conv3(f, W, b, 1)))
    W, b = next(it)
    h = [None] * L
    h[0] = bf16(relu(conv3(x, bf16(W), b, 1)))
    for l in range(1, L):
        W, b = next(it)
        x = bf16(relu(conv3(h[l - 1], bf16(W), b, 2)))
        W, b = next(it)
        h[l] = bf16(relu(conv3(x, bf16(W), b, 1)))
    for l in range(L - 1, 0, -1):
        u = bf16(up2(h[l], h[l - 1].shape[:3]))
        W, b = next(it)
        x = bf16(relu(conv3(u, bf16(W), b, 1)) + h[l - 1])
        W, b = next(it)
        h[l - 1] = bf16(relu(conv3(x, bf16(W), b, 1)))
    W, b = next(it)
    return (h[0] @ W[0].T + b)[..., 0]


@pytest.mark.parametrize("shape,C", [((17, 13, 9), (16, 32, 64)), ((20, 12, 7), (32, 16)), ((33, 33, 5), (16,)),
                                     ((9, 10, 11), (64, 64, 32, 16))])
def test_network_forward_matches_reference(shape, C):
    torch = torch_cuda()
    Nx, Ny, Nz = shape
    print(f"net forward {shape} {C}", flush=True)
    case = sy.random_box(Nx, Ny, Nz, 2, 4, seed=3, dtype="f32")
    g = make_grid(case)
    blob = precond.random_blob(C, seed=len(C))
    g.set_preconditioner(blob)
    rng = np.random.default_rng(1)
    f = rng.uniform(-1, 1, size=(Nz, Ny, Nx, 3)).astype(np.float32)
    out = g.precond_forward(torch.tensor(f, device="cuda"))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = reference_forward(blob, f)
    np.testing.assert_allclose(got, ref, rtol=2e-2, atol=2e-2 * np.abs(ref).max())
    g.close()


def _broken_blob():
    """A network that always proposes doubling J: every proposal must be rejected."""
    C = (16,)
    convs = [(np.zeros((t, co, ci)), np.zeros(co)) for ci, co, t in precond.conv_shapes(C)]
    convs[-1] = (np.zeros((1, 1, 16)), np.array([1e3]))
    return precond.pack_blob(C, convs)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_rejected_corrections_reproduce_the_plain_trajectory(prec):
    case = sy.random_box(12, 10, 8, 4, 8, seed=91, dtype=prec, eps_dex=(-3, -1))
    plain = gpu_solve(case, tol=1e-10, max_iter=2000)
    g = make_grid(case)
    g.set_preconditioner(_broken_blob())
    torch = torch_cuda()
    st = g.new_state(to_dev(case.chi, prec), to_dev(case.eps, prec), to_dev(case.B, prec), to_dev(case.I_bc, prec))
    status, rep = g.solve(st, g.opts(tol=1e-10, max_iter=2000, net_every=3))
    torch.cuda.synchronize()
    J = g.state_tensors(st)["J"].cpu().numpy()
    g.close()
    assert status == 0 and plain["status"] == 0
    assert rep.n_net_accept == 0 and rep.n_net_reject > 3
    # a rejected proposal costs its smoothing sweep and the sweep that judges it
    assert rep.iters == plain["report"].iters + 2 * rep.n_net_reject
    assert rep.n_ng == plain["report"].n_ng
    assert np.array_equal(J, plain["J"])


def test_random_network_keeps_the_fixed_point(orc):
    """Whatever a (random) network proposes, the solve ends at the LU fixed point."""
    case = sy.random_box(7, 7, 5, 4, 8, seed=92, dtype="f64", eps_dex=(-3, -1))
    prob = orc.BoxProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1], 4, 8)
    ref = orc.direct(prob)
    g = make_grid(case)
    g.set_preconditioner(precond.random_blob((16, 32), seed=5, scale=0.3))
    res = gpu_solve(case, tol=1e-12, max_iter=3000, grid=g)
    rep = res["report"]
    assert res["status"] == 0 and rep.n_net_accept + rep.n_net_reject == 0   # net_every defaults to 0
    torch = torch_cuda()
    st = g.new_state(to_dev(case.chi, "f64"), to_dev(case.eps, "f64"), to_dev(case.B, "f64"),
                     to_dev(case.I_bc, "f64"))
    status, rep = g.solve(st, g.opts(tol=1e-12, max_iter=3000, net_every=2))
    torch.cuda.synchronize()
    J = g.state_tensors(st)["J"].cpu().numpy()[0]
    g.close()
    assert status == 0 and rep.n_net_accept + rep.n_net_reject > 0
    np.testing.assert_allclose(J, ref["J"], rtol=1e-9)


def test_preconditioner_rejects_bad_blobs():
    import paper_2102_01734_amd as rt
    case = sy.random_box(5, 5, 5, 2, 4, seed=1, dtype="f32")
    g = make_grid(case)
    good = precond.random_blob((16,), seed=1)
    for bad in (b"XXXX" + good[4:], good[:-4], good + b"\0\0\0\0",
                precond.pack_blob((16,), [(np.full((t, co, ci), np.nan), np.zeros(co))
                                          for ci, co, t in precond.conv_shapes((16,))])):
        with pytest.raises(rt.RtError):
            g.set_preconditioner(bad)
    with pytest.raises(rt.RtError):
        g.precond_forward(to_dev(np.zeros((5, 5, 5, 3)), "f32"))     # no network set
    g.set_preconditioner(good)
    g.set_preconditioner(None)
    g.close()
    sph = rt.SphereGrid(4, 4, 4, 1.0, 2.0, 2, 4)
    with pytest.raises(rt.RtError):
        sph.set_preconditioner(good)
    sph.close()


@pytest.mark.parametrize("N", [129, 257])
def test_network_forward_full_size_is_finite_and_deterministic(N):
    """The shipped 3-level 16/32/32 network and a 4-level 16/32/64/64 one on
    N^3 feature volumes: finite outputs, bitwise equal on a second forward
    (no atomics anywhere in the network); times printed.  Parity of the
    arithmetic is held by the reference forward above on small volumes with
    every layer type."""
    import os
    torch = torch_cuda()
    blob_path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2102_01734_amd",
                             "data", "precond_box.rtun")
    nets = {"16/32/32": open(blob_path, "rb").read(), "16/32/64/64": precond.random_blob((16, 32, 64, 64), seed=4)}
    case = sy.random_box(N, N, N, 2, 4, seed=5, dtype="f32")
    g = make_grid(case)
    f = torch.rand((N, N, N, 3), device="cuda", generator=torch.Generator(device="cuda").manual_seed(3)) * 2 - 1
    for name, blob in nets.items():
        g.set_preconditioner(blob)
        a = g.precond_forward(f)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b = g.precond_forward(f)
        e1.record()
        torch.cuda.synchronize()
        print(f"net {name} forward at {N}^3: {e0.elapsed_time(e1):.2f} ms", flush=True)
        assert bool(torch.isfinite(a).all())
        assert torch.equal(a, b)
    g.close()
