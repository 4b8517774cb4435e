"""ctypes binding of the rt3d C ABI (include/rt3d.h).

Argument marshalling only: every computation runs in the HIP library.  The
functions carry the C names; ``Grid`` is a small convenience wrapper that
takes torch tensors (device memory) and the current torch stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librt3d.so")

RT_OK, RT_E_INVALID, RT_E_NOMEM, RT_E_HIP, RT_E_NOT_CONVERGED, RT_E_NUMERIC, RT_E_UNSUPPORTED = range(7)
RT_GEOM_BOX_PERIODIC_XY, RT_GEOM_SPHERICAL = 0, 1
RT_FP64, RT_FP32 = 0, 1
RT_F_LSTAR_PARABOLIC = 0x1
RT_F_BAND_TILES = 0x2
RT_F_LSTAR_NONLOCAL = 0x4
RT_F_HOST_CACHE = 0x8
RT_NOALLOC_SCRATCH_BYTES = 64 << 20

STATUS_NAMES = {0: "RT_OK", 1: "RT_E_INVALID", 2: "RT_E_NOMEM", 3: "RT_E_HIP", 4: "RT_E_NOT_CONVERGED",
                5: "RT_E_NUMERIC", 6: "RT_E_UNSUPPORTED"}


class RtGridDesc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("geom", ctypes.c_int32), ("n", ctypes.c_int32 * 3),
                ("h", ctypes.c_double * 3), ("n_mu", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("n_lambda_max", ctypes.c_int32), ("prec", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class RtState(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_lambda", ctypes.c_int32), ("chi", ctypes.c_void_p),
                ("eps", ctypes.c_void_p), ("B", ctypes.c_void_p), ("I_bc", ctypes.c_void_p),
                ("J", ctypes.c_void_p), ("S", ctypes.c_void_p), ("lstar", ctypes.c_void_p),
                ("lstar_valid", ctypes.c_int32), ("iter", ctypes.c_int32), ("rel_change", ctypes.c_void_p)]


class RtSolveOpts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("ng_every", ctypes.c_int32), ("ng_start", ctypes.c_int32), ("reanchor", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("method", ctypes.c_int32), ("net_every", ctypes.c_int32),
                ("os_sweeps", ctypes.c_int32), ("os_method", ctypes.c_int32)]


class RtSolveReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("n_fs", ctypes.c_int32), ("n_fs64", ctypes.c_int32),
                ("n_ng", ctypes.c_int32), ("n_converged", ctypes.c_int32), ("max_rel_change", ctypes.c_double),
                ("seconds", ctypes.c_double), ("n_net_accept", ctypes.c_int32), ("n_net_reject", ctypes.c_int32)]


class RtError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Loads librt3d.so from the package directory; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"rt3d HIP library not built: {LIB_PATH} is missing "
                          "(run python paper_2102_01734_amd/build.py)")
    # torch bundles its own HIP runtime with the same soname as the system one;
    # loading torch first makes librt3d.so bind to that single runtime (two
    # runtimes in one process do not share the device)
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    L.rt_create_grid.argtypes = [ctypes.POINTER(RtGridDesc), ctypes.POINTER(vp)]
    L.rt_destroy_grid.argtypes = [vp]
    L.rt_grid_info.argtypes = [vp, i64p, ctypes.POINTER(i32), i64p, ctypes.POINTER(i32)]
    L.rt_formal_solution.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.rt_ali_step.argtypes = [vp, ctypes.POINTER(RtState), ctypes.POINTER(RtSolveOpts), vp]
    L.rt_solve.argtypes = [vp, ctypes.POINTER(RtState), ctypes.POINTER(RtSolveOpts),
                           ctypes.POINTER(RtSolveReport), vp]
    for f in ("rt_create_grid", "rt_destroy_grid", "rt_grid_info", "rt_formal_solution", "rt_ali_step", "rt_solve"):
        getattr(L, f).restype = ctypes.c_int
    L.rt_autotune.argtypes = [vp, i32, vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32), vp]
    L.rt_autotune.restype = ctypes.c_int
    L.rt_autotune_dirs.argtypes = [vp, i32, vp, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32), vp]
    L.rt_autotune_dirs.restype = ctypes.c_int
    L.rt_set_launch_shape.argtypes = [vp, i32, i32]
    L.rt_set_anchor_shape.argtypes = [vp, i32, i32, i32]
    L.rt_set_launch_shape_tiles.argtypes = [vp, i32, i32, i32]
    L.rt_set_launch_shape_tiles.restype = ctypes.c_int
    L.rt_set_anchor_shape.restype = ctypes.c_int
    L.rt_set_launch_shape.restype = ctypes.c_int
    L.rt_launch_shape.argtypes = [vp] + [ctypes.POINTER(i32)] * 4
    L.rt_launch_shape.restype = ctypes.c_int
    L.rt_lstar_stencil.argtypes = [vp, i32, vp, vp, vp]
    L.rt_lstar_stencil.restype = ctypes.c_int
    L.rt_cache_bytes.argtypes = [vp, i64p, i64p]
    L.rt_cache_bytes.restype = ctypes.c_int
    L.rt_profile_enable.argtypes = [vp, i32]
    L.rt_profile_enable.restype = ctypes.c_int
    L.rt_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), i64p]
    L.rt_profile_read.restype = ctypes.c_int
    ip, dp = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    L.rt_box_template.argtypes = [i32, i32, i32, i32, i32, ip, ip, ip, dp, ip]
    L.rt_box_template.restype = ctypes.c_int
    L.rt_sphere_tracks.argtypes = [ctypes.POINTER(RtGridDesc), i32, dp, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_int64), dp, ctypes.POINTER(ctypes.c_int64), ip, dp]
    L.rt_sphere_tracks.restype = ctypes.c_int
    L.rt_formal_solution_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    L.rt_formal_solution_noalloc.restype = ctypes.c_int
    L.rt_formal_solution_dirs.argtypes = [vp, i32, vp, vp, vp, i32, ip, vp, vp, vp]
    L.rt_formal_solution_dirs.restype = ctypes.c_int
    L.rt_shard_directions.argtypes = [vp, i32, i32, ip, ctypes.POINTER(i32)]
    L.rt_shard_directions.restype = ctypes.c_int
    L.rt_set_preconditioner.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.rt_set_preconditioner.restype = ctypes.c_int
    L.rt_precond_forward.argtypes = [vp, vp, vp, vp]
    L.rt_precond_forward.restype = ctypes.c_int
    L.rt_last_error.restype = ctypes.c_char_p
    L.rt_last_error.argtypes = []
    L.rt_version.restype = ctypes.c_char_p
    L.rt_version.argtypes = []
    _lib = L
    return L


def _check(status: int, where: str, allow=()):
    if status != RT_OK and status not in allow:
        raise RtError(status, where, rt_last_error())
    return status


# ---------------------------------------------------------------------------
# the C entry points, same names
# ---------------------------------------------------------------------------
def rt_last_error() -> str:
    return lib().rt_last_error().decode()


def rt_version() -> str:
    return lib().rt_version().decode()


def rt_create_grid(desc: RtGridDesc) -> int:
    h = ctypes.c_void_p()
    _check(lib().rt_create_grid(ctypes.byref(desc), ctypes.byref(h)), "rt_create_grid")
    return h.value


def rt_destroy_grid(grid: int) -> None:
    _check(lib().rt_destroy_grid(ctypes.c_void_p(grid)), "rt_destroy_grid")


def rt_grid_info(grid: int):
    nv, nvis = ctypes.c_int64(), ctypes.c_int64()
    nd, nwg = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().rt_grid_info(ctypes.c_void_p(grid), ctypes.byref(nv), ctypes.byref(nd), ctypes.byref(nvis),
                              ctypes.byref(nwg)), "rt_grid_info")
    return dict(n_vox=nv.value, n_dir=nd.value, n_visits=nvis.value, n_workgroups=nwg.value)


def rt_formal_solution(grid: int, n_lambda: int, chi: int, S: int, I_bc: Optional[int], J_out: int,
                       lstar_out: Optional[int], stream: Optional[int]) -> None:
    _check(lib().rt_formal_solution(ctypes.c_void_p(grid), int(n_lambda), ctypes.c_void_p(chi), ctypes.c_void_p(S),
                                    ctypes.c_void_p(I_bc or None), ctypes.c_void_p(J_out),
                                    ctypes.c_void_p(lstar_out or None), ctypes.c_void_p(stream or None)),
           "rt_formal_solution")


def rt_formal_solution_noalloc(grid: int, n_lambda: int, chi: int, S: int, I_bc: Optional[int], J_out: int,
                               lstar_out: Optional[int], stream: Optional[int]) -> None:
    _check(lib().rt_formal_solution_noalloc(ctypes.c_void_p(grid), int(n_lambda), ctypes.c_void_p(chi),
                                            ctypes.c_void_p(S), ctypes.c_void_p(I_bc or None),
                                            ctypes.c_void_p(J_out), ctypes.c_void_p(lstar_out or None),
                                            ctypes.c_void_p(stream or None)),
           "rt_formal_solution_noalloc")


def rt_ali_step(grid: int, state: RtState, opts: RtSolveOpts, stream: Optional[int]) -> None:
    _check(lib().rt_ali_step(ctypes.c_void_p(grid), ctypes.byref(state), ctypes.byref(opts),
                             ctypes.c_void_p(stream or None)), "rt_ali_step")


def rt_solve(grid: int, state: RtState, opts: RtSolveOpts, stream: Optional[int]) -> tuple[int, RtSolveReport]:
    rep = RtSolveReport()
    st = _check(lib().rt_solve(ctypes.c_void_p(grid), ctypes.byref(state), ctypes.byref(opts), ctypes.byref(rep),
                               ctypes.c_void_p(stream or None)), "rt_solve", allow=(RT_E_NOT_CONVERGED,))
    return st, rep


def rt_autotune(grid: int, n_lambda: int, chi: int, S: int, stream: Optional[int]):
    """Times the compiled launch shapes on these fields; returns (threads, rays per thread) kept."""
    t, r = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().rt_autotune(ctypes.c_void_p(grid), int(n_lambda), ctypes.c_void_p(chi), ctypes.c_void_p(S),
                             ctypes.byref(t), ctypes.byref(r), ctypes.c_void_p(stream or None)), "rt_autotune")
    return t.value, r.value


def rt_set_anchor_shape(grid: int, threads: int, rays: int, band: int) -> None:
    _check(lib().rt_set_anchor_shape(ctypes.c_void_p(grid), int(threads), int(rays), int(band)),
           "rt_set_anchor_shape")


def rt_autotune_dirs(grid: int, n_lambda: int, chi: int, S: int, dirs, stream: Optional[int]):
    """rt_autotune over a direction subset; returns (threads, rays per thread) kept."""
    import numpy as np
    d = np.ascontiguousarray(dirs, dtype=np.int32)
    t, r = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().rt_autotune_dirs(ctypes.c_void_p(grid), int(n_lambda), ctypes.c_void_p(chi), ctypes.c_void_p(S),
                                  int(d.size), d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(t),
                                  ctypes.byref(r), ctypes.c_void_p(stream or None)), "rt_autotune_dirs")
    return t.value, r.value


def rt_set_launch_shape(grid: int, threads: int, rays: int) -> None:
    _check(lib().rt_set_launch_shape(ctypes.c_void_p(grid), int(threads), int(rays)), "rt_set_launch_shape")


def rt_set_launch_shape_tiles(grid: int, threads: int, rays: int, band: int) -> None:
    _check(lib().rt_set_launch_shape_tiles(ctypes.c_void_p(grid), int(threads), int(rays), int(band)),
           "rt_set_launch_shape_tiles")


def rt_lstar_stencil(grid: int, n_lambda: int, chi: int, out: int, stream: Optional[int]) -> None:
    _check(lib().rt_lstar_stencil(ctypes.c_void_p(grid), int(n_lambda), ctypes.c_void_p(chi), ctypes.c_void_p(out),
                                  ctypes.c_void_p(stream or None)), "rt_lstar_stencil")


def rt_cache_bytes(grid: int) -> dict:
    """Geometry-cache bytes in device memory and in pinned host memory."""
    d, h = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().rt_cache_bytes(ctypes.c_void_p(grid), ctypes.byref(d), ctypes.byref(h)), "rt_cache_bytes")
    return dict(device=d.value, host=h.value)


def rt_launch_shape(grid: int) -> dict:
    """Launch shape of the single-output sweep: threads, rays, bundles, band (bool)."""
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().rt_launch_shape(ctypes.c_void_p(grid), *[ctypes.byref(x) for x in v]), "rt_launch_shape")
    return dict(threads=v[0].value, rays=v[1].value, bundles=v[2].value, band=bool(v[3].value))


def rt_profile_enable(grid: int, enable: bool) -> None:
    _check(lib().rt_profile_enable(ctypes.c_void_p(grid), int(bool(enable))), "rt_profile_enable")


def rt_profile_read(grid: int):
    """(summed formal-solution kernel ms, launches, characteristic points) since the last read."""
    ms, n, pts = ctypes.c_double(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().rt_profile_read(ctypes.c_void_p(grid), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(pts)),
           "rt_profile_read")
    return ms.value, n.value, pts.value


def rt_box_template(Nz: int, n_mu: int, n_phi: int, d: int):
    """Host tracker output of direction d: dict of numpy arrays di, dj, kk, s."""
    import numpy as np
    M = ctypes.c_int32()
    _check(lib().rt_box_template(Nz, n_mu, n_phi, d, 0, None, None, None, None, ctypes.byref(M)), "rt_box_template")
    n = M.value
    di = np.zeros(n, np.int32); dj = np.zeros(n, np.int32); kk = np.zeros(n, np.int32); s = np.zeros(n)
    ip, dp = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    _check(lib().rt_box_template(Nz, n_mu, n_phi, d, n, di.ctypes.data_as(ip), dj.ctypes.data_as(ip),
                                 kk.ctypes.data_as(ip), s.ctypes.data_as(dp), ctypes.byref(M)), "rt_box_template")
    return dict(di=di, dj=dj, kk=kk, s=s)


def rt_formal_solution_dirs(grid: int, n_lambda: int, chi: int, S: int, I_bc: Optional[int], dirs, J_out: int,
                            lstar_out: Optional[int], stream: Optional[int]) -> None:
    import numpy as np
    d = np.ascontiguousarray(dirs, dtype=np.int32)
    _check(lib().rt_formal_solution_dirs(ctypes.c_void_p(grid), int(n_lambda), ctypes.c_void_p(chi),
                                         ctypes.c_void_p(S), ctypes.c_void_p(I_bc or None), int(d.size),
                                         d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.c_void_p(J_out),
                                         ctypes.c_void_p(lstar_out or None), ctypes.c_void_p(stream or None)),
           "rt_formal_solution_dirs")


def rt_shard_directions(grid: int, n_shards: int, shard: int):
    import numpy as np
    n = ctypes.c_int32()
    _check(lib().rt_shard_directions(ctypes.c_void_p(grid), n_shards, shard, None, ctypes.byref(n)),
           "rt_shard_directions")
    out = np.zeros(n.value, np.int32)
    _check(lib().rt_shard_directions(ctypes.c_void_p(grid), n_shards, shard,
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(n)),
           "rt_shard_directions")
    return out


def rt_set_preconditioner(grid: int, blob: Optional[bytes]) -> None:
    """Sets (bytes) or removes (None) the learned-correction network of a box grid."""
    _check(lib().rt_set_preconditioner(ctypes.c_void_p(grid), blob, len(blob) if blob else 0),
           "rt_set_preconditioner")


def rt_precond_forward(grid: int, features: int, out: int, stream: Optional[int]) -> None:
    _check(lib().rt_precond_forward(ctypes.c_void_p(grid), ctypes.c_void_p(features), ctypes.c_void_p(out),
                                    ctypes.c_void_p(stream or None)), "rt_precond_forward")


def box_desc(Nx: int, Ny: int, Nz: int, n_mu: int, n_phi: int, prec: str = "f32", n_lambda_max: int = 1,
             lstar: str = "linear", band_tiles: bool = False, nonlocal_lstar: bool = False) -> RtGridDesc:
    d = RtGridDesc()
    d.struct_size = ctypes.sizeof(RtGridDesc)
    d.geom = RT_GEOM_BOX_PERIODIC_XY
    d.n[0], d.n[1], d.n[2] = Nx, Ny, Nz
    d.n_mu, d.n_phi = n_mu, n_phi
    d.n_lambda_max = n_lambda_max
    d.prec = RT_FP32 if prec == "f32" else RT_FP64
    d.flags = ((RT_F_LSTAR_PARABOLIC if lstar == "parabolic" else 0) | (RT_F_BAND_TILES if band_tiles else 0)
               | (RT_F_LSTAR_NONLOCAL if nonlocal_lstar else 0))
    return d


def sphere_desc(Nr: int, Nt: int, Np: int, r_core: float, r_out: float, n_mu: int, n_phi: int, prec: str = "f32",
                n_lambda_max: int = 1, lstar: str = "linear", source_distance: float = 0.0,
                host_cache: bool = False, nonlocal_lstar: bool = False) -> RtGridDesc:
    d = RtGridDesc()
    d.struct_size = ctypes.sizeof(RtGridDesc)
    d.geom = RT_GEOM_SPHERICAL
    d.n[0], d.n[1], d.n[2] = Nr, Nt, Np
    d.h[0], d.h[1], d.h[2] = r_core, r_out, source_distance
    d.n_mu, d.n_phi = n_mu, n_phi
    d.n_lambda_max = n_lambda_max
    d.prec = RT_FP32 if prec == "f32" else RT_FP64
    d.flags = ((RT_F_LSTAR_PARABOLIC if lstar == "parabolic" else 0) | (RT_F_HOST_CACHE if host_cache else 0)
               | (RT_F_LSTAR_NONLOCAL if nonlocal_lstar else 0))
    return d


def rt_sphere_tracks(desc: RtGridDesc, d: int):
    """Host tracker output of direction d of a spherical grid: dict with h, chars (n, 6),
    begin (n + 1), vox, s."""
    import numpy as np
    h = ctypes.c_double()
    nc, nv = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().rt_sphere_tracks(ctypes.byref(desc), d, ctypes.byref(h), ctypes.byref(nc), ctypes.byref(nv),
                                  None, None, None, None), "rt_sphere_tracks")
    chars = np.zeros((nc.value, 6)); begin = np.zeros(nc.value + 1, np.int64)
    vox = np.zeros(nv.value, np.int32); s = np.zeros(nv.value)
    dp, ip, lp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    _check(lib().rt_sphere_tracks(ctypes.byref(desc), d, ctypes.byref(h), ctypes.byref(nc), ctypes.byref(nv),
                                  chars.ctypes.data_as(dp), begin.ctypes.data_as(lp), vox.ctypes.data_as(ip),
                                  s.ctypes.data_as(dp)), "rt_sphere_tracks")
    return dict(h=h.value, chars=chars, begin=begin, vox=vox, s=s)


# ---------------------------------------------------------------------------
# torch-facing convenience wrapper
# ---------------------------------------------------------------------------
def _stream_ptr(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


class Grid:
    """A library grid handle.  Fields are torch tensors on the GPU, shaped
    (n_lambda, Nz, Ny, Nx), of dtype float32 (prec "f32") or float64 ("f64")."""

    def __init__(self, Nx: int, Ny: int, Nz: int, n_mu: int, n_phi: int, prec: str = "f32",
                 n_lambda_max: int = 1, lstar: str = "linear", band_tiles: bool = False,
                 nonlocal_lstar: bool = False):
        d = box_desc(Nx, Ny, Nz, n_mu, n_phi, prec, n_lambda_max, lstar, band_tiles, nonlocal_lstar)
        self.desc = d
        self.shape = (Nz, Ny, Nx)
        self.nbc = 2
        self.prec = prec
        self.n_lambda_max = n_lambda_max
        self.handle = rt_create_grid(d)

    @property
    def dtype(self):
        import torch
        return torch.float32 if self.prec == "f32" else torch.float64

    def info(self):
        return rt_grid_info(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            rt_destroy_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_field(self, t, n_lambda, name, dtype=None):
        import torch
        dtype = dtype or self.dtype
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA tensor")
        if t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != (n_lambda, *self.shape):
            raise ValueError(f"{name} must be contiguous {dtype} of shape {(n_lambda, *self.shape)}")
        return t.data_ptr()

    def formal_solution(self, chi, S, I_bc=None, want_lstar=False, stream=None, out=None):
        import torch
        n = chi.shape[0]
        pc = self._check_field(chi, n, "chi")
        ps = self._check_field(S, n, "S")
        pb = None
        if I_bc is not None:
            if I_bc.dtype != self.dtype or tuple(I_bc.shape) != (n, self.nbc) or not I_bc.is_contiguous():
                raise ValueError(f"I_bc must be contiguous (n_lambda, {self.nbc}) of the grid dtype")
            pb = I_bc.data_ptr()
        J = out if out is not None else torch.empty_like(chi)
        L = torch.empty_like(chi) if want_lstar else None
        rt_formal_solution(self.handle, n, pc, ps, pb, J.data_ptr(), L.data_ptr() if L is not None else None,
                           _stream_ptr(stream))
        return J, L

    def formal_solution_dirs(self, chi, S, dirs, I_bc=None, want_lstar=False, stream=None):
        """Partial J (and Lambda*) over the listed directions (one shard of a solid-angle decomposition)."""
        import torch
        n = chi.shape[0]
        pc, ps = self._check_field(chi, n, "chi"), self._check_field(S, n, "S")
        pb = I_bc.data_ptr() if I_bc is not None else None
        J = torch.empty_like(chi)
        L = torch.empty_like(chi) if want_lstar else None
        rt_formal_solution_dirs(self.handle, n, pc, ps, pb, dirs, J.data_ptr(),
                                L.data_ptr() if L is not None else None, _stream_ptr(stream))
        return J, L

    def shard_directions(self, n_shards, shard):
        return rt_shard_directions(self.handle, n_shards, shard)

    def autotune(self, chi, S, stream=None):
        n = chi.shape[0]
        return rt_autotune(self.handle, n, self._check_field(chi, n, "chi"), self._check_field(S, n, "S"),
                           _stream_ptr(stream))

    def autotune_dirs(self, chi, S, dirs, stream=None):
        n = chi.shape[0]
        return rt_autotune_dirs(self.handle, n, self._check_field(chi, n, "chi"), self._check_field(S, n, "S"),
                                dirs, _stream_ptr(stream))

    def set_launch_shape(self, threads, rays, band=None):
        """band None: the grid's own tile kind; True/False: row bands / whole layers."""
        if band is None:
            rt_set_launch_shape(self.handle, threads, rays)
        else:
            rt_set_launch_shape_tiles(self.handle, threads, rays, 1 if band else 0)

    def set_anchor_shape(self, threads, rays, band=False):
        rt_set_anchor_shape(self.handle, threads, rays, 1 if band else 0)

    def lstar_stencil(self, chi, stream=None):
        """Nearest-neighbour Lambda* (n_lambda, 27, *grid shape) for the opacity chi."""
        import torch
        n = chi.shape[0]
        c = self._check_field(chi, n, "chi")
        out = torch.empty((n, 27) + tuple(chi.shape[1:]), dtype=chi.dtype, device=chi.device)
        rt_lstar_stencil(self.handle, n, c, out.data_ptr(), _stream_ptr(stream))
        return out

    def cache_bytes(self):
        """dict(device, host): bytes of the geometry cache in each memory."""
        return rt_cache_bytes(self.handle)

    def launch_shape(self):
        """dict(threads, rays, bundles, band) of the single-output sweep."""
        return rt_launch_shape(self.handle)

    def new_state(self, chi, eps, B, I_bc=None, J0=None):
        """Allocates the ALI state (J, S, Lambda*, norms) for a batch; J starts at B."""
        import torch
        n = chi.shape[0]
        st = RtState()
        st.struct_size = ctypes.sizeof(RtState)
        st.n_lambda = n
        st.chi = self._check_field(chi, n, "chi")
        st.eps = self._check_field(eps, n, "eps")
        st.B = self._check_field(B, n, "B")
        st.I_bc = I_bc.data_ptr() if I_bc is not None else None
        J = (B.double() if J0 is None else J0.double()).contiguous().clone()
        S = torch.empty_like(J)
        L = torch.empty_like(chi)
        rel = torch.zeros(n, dtype=torch.float64, device=chi.device)
        st.J, st.S, st.lstar, st.rel_change = J.data_ptr(), S.data_ptr(), L.data_ptr(), rel.data_ptr()
        st.lstar_valid = 0
        st.iter = 0
        # keep the tensors alive with the state
        st._keep = (chi, eps, B, I_bc, J, S, L, rel)
        return st

    @staticmethod
    def opts(tol=1e-8, max_iter=1000, ng_every=4, ng_start=4, reanchor=0, use_graph=False, net_every=0,
             method="ali", os_sweeps=0, os_method="jacobi"):
        """os_method: "jacobi" or "gauss-seidel" (colour order, see include/rt3d.h)."""
        o = RtSolveOpts()
        o.struct_size = ctypes.sizeof(RtSolveOpts)
        o.tol, o.max_iter, o.ng_every, o.ng_start, o.reanchor = tol, max_iter, ng_every, ng_start, reanchor
        o.use_graph = int(bool(use_graph))
        o.net_every = int(net_every)
        o.method = {"ali": 0, "bicgstab": 1}[method]
        o.os_sweeps = int(os_sweeps)
        o.os_method = {"jacobi": 0, "gauss-seidel": 1}[os_method]
        return o

    def set_preconditioner(self, blob):
        """blob: the network weights (bytes, see include/rt3d.h) or None."""
        rt_set_preconditioner(self.handle, blob)

    def precond_forward(self, features, out=None, stream=None):
        """Network output for a feature volume (Nz, Ny, Nx, 3) float32 on the GPU."""
        import torch
        if features.dtype != torch.float32 or not features.is_contiguous() or \
                tuple(features.shape) != (*self.shape, 3):
            raise ValueError(f"features must be contiguous float32 of shape {(*self.shape, 3)}")
        out = out if out is not None else torch.empty(self.shape, dtype=torch.float32, device=features.device)
        rt_precond_forward(self.handle, features.data_ptr(), out.data_ptr(), _stream_ptr(stream))
        return out

    def ali_step(self, state: RtState, opts: RtSolveOpts, stream=None):
        rt_ali_step(self.handle, state, opts, _stream_ptr(stream))

    def solve(self, state: RtState, opts: RtSolveOpts, stream=None):
        return rt_solve(self.handle, state, opts, _stream_ptr(stream))

    @staticmethod
    def state_tensors(state: RtState):
        chi, eps, B, I_bc, J, S, L, rel = state._keep
        return dict(J=J, S=S, lstar=L, rel_change=rel)


class SphereGrid(Grid):
    """A spherical grid handle.  Fields are torch tensors on the GPU shaped
    (n_lambda, Nphi, Ntheta, Nr) (r fastest); I_bc is (n_lambda, 3) =
    (I_out, I_core, J_sub)."""

    def __init__(self, Nr: int, Nt: int, Np: int, r_core: float, r_out: float, n_mu: int, n_phi: int,
                 prec: str = "f32", n_lambda_max: int = 1, lstar: str = "linear", source_distance: float = 0.0,
                 host_cache: bool = False, nonlocal_lstar: bool = False):
        d = sphere_desc(Nr, Nt, Np, r_core, r_out, n_mu, n_phi, prec, n_lambda_max, lstar, source_distance,
                        host_cache, nonlocal_lstar)
        self.desc = d
        self.shape = (Np, Nt, Nr)
        self.nbc = 3
        self.prec = prec
        self.n_lambda_max = n_lambda_max
        self.handle = rt_create_grid(d)
