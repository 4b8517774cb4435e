"""Helpers for the GPU tests: run the HIP library on numpy inputs."""
import numpy as np


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def to_dev(a, prec):
    torch = torch_cuda()
    dt = torch.float32 if prec == "f32" else torch.float64
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def make_grid(case, n_lambda_max=None, lstar="linear", prec=None, band_tiles=False):
    import paper_2102_01734_amd as rt
    if hasattr(case, "Nr"):
        return rt.SphereGrid(case.Nr, case.Nt, case.Np, case.r_core, case.r_out, case.n_mu, case.n_phi,
                             prec or case.dtype, n_lambda_max or case.n_lambda, lstar=lstar,
                             source_distance=case.source_distance)
    return rt.Grid(case.Nx, case.Ny, case.Nz, case.n_mu, case.n_phi, prec or case.dtype,
                   n_lambda_max or case.n_lambda, lstar=lstar, band_tiles=band_tiles)


def gpu_fs(case, S, lstar="linear", want_lstar=True, prec=None, grid=None, I_bc=None):
    """Formal solution of all wavelengths of `case` with source S (n_lambda, Nz, Ny, Nx)."""
    torch = torch_cuda()
    prec = prec or case.dtype
    g = grid or make_grid(case, lstar=lstar, prec=prec)
    chi = to_dev(case.chi, prec)
    St = to_dev(S, prec)
    Ib = to_dev(case.I_bc if I_bc is None else I_bc, prec)
    J, L = g.formal_solution(chi, St, Ib, want_lstar=want_lstar)
    torch.cuda.synchronize()
    out = (J.double().cpu().numpy(), L.double().cpu().numpy() if L is not None else None)
    if grid is None:
        g.close()
    return out


def gpu_solve(case, tol=1e-10, max_iter=2000, ng_every=4, ng_start=4, lstar="linear", prec=None, reanchor=0,
              grid=None, os_method="jacobi", os_sweeps=0):
    torch = torch_cuda()
    prec = prec or case.dtype
    g = grid or make_grid(case, lstar=lstar, prec=prec)
    chi, eps, B = to_dev(case.chi, prec), to_dev(case.eps, prec), to_dev(case.B, prec)
    Ib = to_dev(case.I_bc, prec)
    st = g.new_state(chi, eps, B, Ib)
    status, rep = g.solve(st, g.opts(tol=tol, max_iter=max_iter, ng_every=ng_every, ng_start=ng_start,
                                     reanchor=reanchor, os_method=os_method, os_sweeps=os_sweeps))
    torch.cuda.synchronize()
    t = g.state_tensors(st)
    res = dict(J=t["J"].cpu().numpy(), S=t["S"].cpu().numpy(), lstar=t["lstar"].double().cpu().numpy(),
               status=status, report=rep)
    if grid is None:
        g.close()
    return res
