"""Oracle: plain, slow, FP64 CPU reference for the 3D radiative-transfer hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2102_01734_amd``) and imports nothing from
it; the GPU library never imports it.

What it follows (Hauschildt & Baron, arXiv 2102.01734):
  * formal solution J = Lambda S along long characteristics      -- Sec. 2.2, eq. (frmsol)
  * S = (1 - eps) J + eps B                                       -- Sec. 2.2
  * operator splitting [1 - Lambda*(1-eps)] J_new = J_fs - Lambda*(1-eps) J_old
                                                                  -- Sec. 2.2, eq. (alo)
  * Lambda* = Lambda is a direct solution by matrix inversion    -- Sec. 2.2
  * the non-local (nearest-neighbour) Lambda*: Lambda restricted to the 27
    neighbours of each voxel, the OS system then solved as a sparse system
                                                                  -- Sec. 2.2, Sec. 3
  * BiCGStab as the linear solver                                 -- Sec. 4 ("Method")
  * the per-point steps of the formal solution                    -- Listing 1, steps 1-5
Ng acceleration (Ng 1974, Auer 1987) is not in the paper; it is written here
from its published least-squares definition.

The C part (``rt_oracle.c``) holds the tracker and the formal solution; the
solvers below are plain numpy around it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

LSTAR_LINEAR = 0
LSTAR_PARABOLIC = 1
_KINDS = {"linear": LSTAR_LINEAR, "parabolic": LSTAR_PARABOLIC}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_long)


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        L.orc_quadrature.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        L.orc_direction_vector.argtypes = [ctypes.c_double, ctypes.c_double, _dp]
        L.orc_trace_box.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, _ip, _ip, _ip, _dp, _dp]
        L.orc_trace_box.restype = ctypes.c_int
        L.orc_box_template.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       _ip, _ip, _ip, _dp, _dp]
        L.orc_box_template.restype = ctypes.c_int
        L.orc_moments.argtypes = [ctypes.c_double, _dp, _dp, _dp]
        L.orc_beta_limit.argtypes = [ctypes.c_double]
        L.orc_beta_limit.restype = ctypes.c_double
        L.orc_weights.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp, _dp, _dp]
        L.orc_weights.restype = ctypes.c_int
        L.orc_ray.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.orc_fs_box.argtypes = [ctypes.c_int] * 5 + [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                                      ctypes.c_int, _dp, _dp, ctypes.c_int]
        L.orc_fs_box.restype = ctypes.c_int
        L.orc_fs_box_dirs.argtypes = [ctypes.c_int] * 5 + [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                                           ctypes.c_int, ctypes.c_int, _ip, _dp, _dp, ctypes.c_int]
        L.orc_fs_box_dirs.restype = ctypes.c_int
        L.orc_ray_op.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_double, _dp]
        L.orc_fs_box_op.argtypes = [ctypes.c_int] * 5 + [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                                         ctypes.c_int, _dp]
        L.orc_fs_box_op.restype = ctypes.c_int
        L.orc_lstar_stencil_box.argtypes = [ctypes.c_int] * 5 + [_dp, ctypes.c_int, _dp, ctypes.c_int]
        L.orc_lstar_stencil_box.restype = ctypes.c_int
        L.orc_fs_box_sampled.argtypes = [ctypes.c_int] * 5 + [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                                              ctypes.c_int, ctypes.c_int, _lp, _dp, _dp,
                                                              ctypes.c_int]
        L.orc_fs_box_sampled.restype = ctypes.c_int
        L.orc_fs_1d.argtypes = [ctypes.c_int] * 3 + [_dp, _dp, ctypes.c_double, ctypes.c_double,
                                                     ctypes.c_int, _dp, _dp]
        L.orc_fs_1d.restype = ctypes.c_int
        L.orc_fs_1d_dirs.argtypes = [ctypes.c_int] * 3 + [_dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.orc_fs_1d_dirs.restype = ctypes.c_int
        L.orc_sph_spacing.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 2
        L.orc_sph_spacing.restype = ctypes.c_double
        L.orc_sph_rays.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 3 + [_dp, ctypes.c_int, _dp]
        L.orc_sph_rays.restype = ctypes.c_int
        L.orc_sph_char.argtypes = [ctypes.c_int] * 3 + [ctypes.c_double] * 2 + [_dp, _dp, ctypes.c_int, _ip, _dp, _dp]
        L.orc_sph_char.restype = ctypes.c_int
        L.orc_sph_irradiation.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp] + [ctypes.c_double] * 3
        L.orc_sph_irradiation.restype = ctypes.c_double
        L.orc_fs_sphere.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double] * 2 + [ctypes.c_int] * 2
                                    + [ctypes.c_double] * 2 + [_dp, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp, _dp,
                                                               ctypes.c_int])
        L.orc_fs_sphere.restype = ctypes.c_int
        L.orc_lstar_stencil_sphere.argtypes = ([ctypes.c_int] * 3 + [ctypes.c_double] * 2 + [ctypes.c_int] * 2
                                               + [_dp, ctypes.c_int, _dp, ctypes.c_int])
        L.orc_lstar_stencil_sphere.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_threads() -> int:
    n = os.environ.get("ORACLE_THREADS")
    if n:
        return max(1, int(n))
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


# --------------------------------------------------------------------------
# quadrature, geometry, weights
# --------------------------------------------------------------------------
def quadrature(n_mu: int, n_phi: int):
    """Midpoint directions equally spaced in mu and phi, equal weights (Sec. 3.1)."""
    n = n_mu * n_phi
    mu, phi, w = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_quadrature(n_mu, n_phi, _d(mu), _d(phi), _d(w))
    return mu, phi, w


def direction_vector(mu: float, phi: float):
    n3 = np.zeros(3)
    lib().orc_direction_vector(mu, phi, _d(n3))
    return n3


def box_template(Nz: int, mu: float, phi: float):
    """Segments of the characteristic entering column (0,0): dict(di, dj, kk, s, t0)."""
    az = abs(mu)
    cap = int(3.0 * (Nz / az) * 2.0 + 16)
    di = np.zeros(cap, np.int32); dj = np.zeros(cap, np.int32); kk = np.zeros(cap, np.int32)
    s = np.zeros(cap); t0 = np.zeros(cap)
    M = lib().orc_box_template(Nz, mu, phi, cap, di.ctypes.data_as(_ip), dj.ctypes.data_as(_ip),
                               kk.ctypes.data_as(_ip), _d(s), _d(t0))
    if M < 0:
        raise RuntimeError("trace failed")
    return dict(di=di[:M].copy(), dj=dj[:M].copy(), kk=kk[:M].copy(), s=s[:M].copy(), t0=t0[:M].copy())


def trace(Nz: int, n3):
    az = abs(n3[2])
    cap = int(3.0 * (Nz / az) * 2.0 + 16)
    di = np.zeros(cap, np.int32); dj = np.zeros(cap, np.int32); kk = np.zeros(cap, np.int32)
    s = np.zeros(cap); t0 = np.zeros(cap)
    M = lib().orc_trace_box(Nz, float(n3[0]), float(n3[1]), float(n3[2]), cap, di.ctypes.data_as(_ip),
                            dj.ctypes.data_as(_ip), kk.ctypes.data_as(_ip), _d(s), _d(t0))
    if M < 0:
        raise RuntimeError("trace failed")
    return dict(di=di[:M].copy(), dj=dj[:M].copy(), kk=kk[:M].copy(), s=s[:M].copy(), t0=t0[:M].copy())


def moments(D: float):
    e0, e1, e2 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_moments(float(D), ctypes.byref(e0), ctypes.byref(e1), ctypes.byref(e2))
    return e0.value, e1.value, e2.value


def beta_limit(D: float) -> float:
    return lib().orc_beta_limit(float(D))


def weights(D: float, Dp: float, last: bool = False):
    """(alpha, beta, gamma, used_linear) of one segment (Listing 1, step 4)."""
    a, b, g = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lin = lib().orc_weights(float(D), float(Dp), int(bool(last)), ctypes.byref(a), ctypes.byref(b),
                            ctypes.byref(g))
    return a.value, b.value, g.value, bool(lin)


def ray(tau, S, I_bc: float, kind: str = "linear"):
    """Intensities at the points of one characteristic and the local diagonal."""
    tau = _f64(tau); S = _f64(S)
    M = tau.size
    I = np.zeros(M); d = np.zeros(M)
    lib().orc_ray(M, _d(tau), _d(S), float(I_bc), _KINDS[kind], _d(I), _d(d))
    return I, d


# --------------------------------------------------------------------------
# formal solutions
# --------------------------------------------------------------------------
def fs_box(chi, S, I_top: float, I_bot: float, n_mu: int, n_phi: int, kind: str = "linear",
           threads: int | None = None, want_lstar: bool = True):
    """J = Lambda S (+ boundary term) and diagonal Lambda* on the periodic box.

    chi, S: arrays of shape (Nz, Ny, Nx), k = 0 the top layer.
    """
    chi = _f64(chi); S = _f64(S)
    Nz, Ny, Nx = chi.shape
    J = np.zeros_like(chi)
    L = np.zeros_like(chi) if want_lstar else None
    rc = lib().orc_fs_box(Nx, Ny, Nz, n_mu, n_phi, _d(chi), _d(S), float(I_top), float(I_bot),
                          _KINDS[kind], _d(J), _d(L) if L is not None else None,
                          threads or default_threads())
    if rc != 0:
        raise RuntimeError(f"orc_fs_box failed ({rc})")
    return J, L


def fs_box_op(chi, S, I_top: float, I_bot: float, n_mu: int, n_phi: int, op: str = "parabolic"):
    """J = Lambda_op S (+ boundary term): op "parabolic" is the formal solution
    itself, op "linear" the linear-interpolation operator (single thread)."""
    chi = _f64(chi); S = _f64(S)
    Nz, Ny, Nx = chi.shape
    J = np.zeros_like(chi)
    rc = lib().orc_fs_box_op(Nx, Ny, Nz, n_mu, n_phi, _d(chi), _d(S), float(I_top), float(I_bot),
                             _KINDS[op], _d(J))
    if rc != 0:
        raise RuntimeError(f"orc_fs_box_op failed ({rc})")
    return J


def ray_op(tau, S, I_bc: float, op: str = "parabolic"):
    """One characteristic of operator op: intensities at its points."""
    tau = _f64(tau); S = _f64(S)
    I = np.zeros_like(tau)
    lib().orc_ray_op(_KINDS[op], int(tau.size), _d(tau), _d(S), float(I_bc), _d(I))
    return I


def lstar_stencil(chi, n_mu: int, n_phi: int, op: str = "linear", threads: int | None = None):
    """Nearest-neighbour Lambda* of operator op: array (27, Nz, Ny, Nx); component
    c = (dz+1)*9 + (dy+1)*3 + (dx+1) holds Lambda_op[v, v + (dx, dy, dz)] (x, y periodic)."""
    chi = _f64(chi)
    Nz, Ny, Nx = chi.shape
    out = np.zeros((27,) + chi.shape)
    rc = lib().orc_lstar_stencil_box(Nx, Ny, Nz, n_mu, n_phi, _d(chi), _KINDS[op], _d(out),
                                     threads or default_threads())
    if rc != 0:
        raise RuntimeError(f"orc_lstar_stencil_box failed ({rc})")
    return out


def stencil_matrix(st):
    """The (N x N) sparse matrix of a 27-point stencil (27, Nz, Ny, Nx); entries of
    components that land on the same voxel (x or y period below 3) are summed;
    neighbours beyond the top or bottom layer do not exist."""
    import scipy.sparse as sp
    _, Nz, Ny, Nx = st.shape
    k, y, x = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    v = (k * Ny + y) * Nx + x
    rows, cols, vals = [], [], []
    for c in range(27):
        dz, dy, dx = c // 9 - 1, (c // 3) % 3 - 1, c % 3 - 1
        ku = k + dz
        ok = (ku >= 0) & (ku < Nz)
        u = (ku * Ny + (y + dy) % Ny) * Nx + (x + dx) % Nx
        rows.append(v[ok]); cols.append(u[ok]); vals.append(st[c][ok])
    n = Nx * Ny * Nz
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def fs_box_dirs(chi, S, I_top: float, I_bot: float, n_mu: int, n_phi: int, dirs, kind: str = "linear",
                threads: int | None = None, want_lstar: bool = False):
    """Partial angle sum of J (and Lambda*) over the listed directions only."""
    chi = _f64(chi); S = _f64(S)
    Nz, Ny, Nx = chi.shape
    dirs = np.ascontiguousarray(dirs, dtype=np.int32)
    J = np.zeros_like(chi)
    L = np.zeros_like(chi) if want_lstar else None
    rc = lib().orc_fs_box_dirs(Nx, Ny, Nz, n_mu, n_phi, _d(chi), _d(S), float(I_top), float(I_bot),
                               _KINDS[kind], int(dirs.size), dirs.ctypes.data_as(_ip), _d(J),
                               _d(L) if L is not None else None, threads or default_threads())
    if rc != 0:
        raise RuntimeError(f"orc_fs_box_dirs failed ({rc})")
    return J, L


def fs_box_sampled(chi, S, I_top: float, I_bot: float, n_mu: int, n_phi: int, vox, kind: str = "linear",
                   threads: int | None = None):
    """J and Lambda* at the listed flat voxel indices only."""
    chi = _f64(chi); S = _f64(S)
    Nz, Ny, Nx = chi.shape
    vox = np.ascontiguousarray(vox, dtype=np.int64)
    J = np.zeros(vox.size); L = np.zeros(vox.size)
    rc = lib().orc_fs_box_sampled(Nx, Ny, Nz, n_mu, n_phi, _d(chi), _d(S), float(I_top), float(I_bot),
                                  _KINDS[kind], int(vox.size), vox.ctypes.data_as(_lp), _d(J), _d(L),
                                  threads or default_threads())
    if rc != 0:
        raise RuntimeError(f"orc_fs_box_sampled failed ({rc})")
    return J, L


def fs_1d(chi_k, S_k, I_top: float, I_bot: float, n_mu: int, n_phi: int, kind: str = "linear"):
    """Formal solution of an x,y-homogeneous box, one template ray per direction."""
    chi_k = _f64(chi_k); S_k = _f64(S_k)
    Nz = chi_k.size
    J = np.zeros(Nz); L = np.zeros(Nz)
    rc = lib().orc_fs_1d(Nz, n_mu, n_phi, _d(chi_k), _d(S_k), float(I_top), float(I_bot),
                         _KINDS[kind], _d(J), _d(L))
    if rc != 0:
        raise RuntimeError("orc_fs_1d failed")
    return J, L


def fs_1d_dirs(chi_k, S_k, I_top: float, I_bot: float, n_mu: int, n_phi: int):
    chi_k = _f64(chi_k); S_k = _f64(S_k)
    Nz = chi_k.size
    out = np.zeros(n_mu * n_phi * Nz)
    rc = lib().orc_fs_1d_dirs(Nz, n_mu, n_phi, _d(chi_k), _d(S_k), float(I_top), float(I_bot), _d(out))
    if rc != 0:
        raise RuntimeError("orc_fs_1d_dirs failed")
    return out.reshape(n_mu * n_phi, Nz)


# --------------------------------------------------------------------------
# spherical grid
# --------------------------------------------------------------------------
class SphereGrid:
    """Voxels between r_c and r_out: Nr shells x Nt cones x Np half-planes, index (ip*Nt + it)*Nr + ir."""

    def __init__(self, Nr, Nt, Np, rc=1.0, ro=2.0):
        self.Nr, self.Nt, self.Np, self.rc, self.ro = int(Nr), int(Nt), int(Np), float(rc), float(ro)

    @property
    def n_vox(self):
        return self.Nr * self.Nt * self.Np

    def spacing(self):
        return lib().orc_sph_spacing(self.Nr, self.Nt, self.Np, self.rc, self.ro)

    def rays(self, n3):
        """Characteristics of direction n3: array (nc, 8) = p (3), t_a, t_b, kind (1 = leaves the core)."""
        n3 = _f64(n3)
        h = self.spacing()
        K = int(np.ceil(self.ro / h)) + 1
        cap = 2 * ((2 * K + 1) ** 2 + self.n_vox) + 16
        out = np.zeros(8 * cap)
        nc = lib().orc_sph_rays(self.Nr, self.Nt, self.Np, self.rc, self.ro, h, _d(n3), cap, _d(out))
        if nc < 0:
            raise RuntimeError("too many characteristics")
        return out[:8 * nc].reshape(nc, 8).copy()

    def segments(self, ch, n3):
        ch = _f64(ch); n3 = _f64(n3)
        cap = 4 * (self.Nr + self.Nt + self.Np) + 20
        vox = np.zeros(cap, np.int32); s = np.zeros(cap); t0 = np.zeros(cap)
        M = lib().orc_sph_char(self.Nr, self.Nt, self.Np, self.rc, self.ro, _d(ch), _d(n3), cap,
                               vox.ctypes.data_as(_ip), _d(s), _d(t0))
        return vox[:M].copy(), s[:M].copy(), t0[:M].copy()


def sph_irradiation(n_mu, n_phi, d, x, ro, dsrc, B_sub=1.0):
    return lib().orc_sph_irradiation(n_mu, n_phi, d, _d(_f64(x)), float(ro), float(dsrc), float(B_sub))


def fs_sphere(grid: SphereGrid, n_mu, n_phi, chi, S, Bv, I_out=0.0, dsrc=0.0, B_sub=1.0, kind="linear",
              threads=None):
    """J and Lambda* on the spherical grid; fields flat in voxel order."""
    chi = _f64(chi).ravel(); S = _f64(S).ravel(); Bv = _f64(Bv).ravel()
    J = np.zeros(grid.n_vox); L = np.zeros(grid.n_vox)
    rc = lib().orc_fs_sphere(grid.Nr, grid.Nt, grid.Np, grid.rc, grid.ro, n_mu, n_phi, float(dsrc), float(B_sub),
                             _d(chi), _d(S), _d(Bv), float(I_out), _KINDS[kind], _d(J), _d(L),
                             threads or default_threads())
    if rc != 0:
        raise RuntimeError(f"orc_fs_sphere failed ({rc})")
    return J, L


def lstar_stencil_sphere(grid: SphereGrid, n_mu, n_phi, chi, op: str = "linear", threads=None):
    """Nearest-neighbour Lambda* of operator op on the spherical grid: array (27, Np, Nt, Nr); component
    c = (dp+1)*9 + (dt+1)*3 + (dr+1) holds the element for the neighbour (ir+dr, it+dt, ip+dp), phi periodic."""
    chi = _f64(chi).ravel()
    out = np.zeros(27 * grid.n_vox)
    rc = lib().orc_lstar_stencil_sphere(grid.Nr, grid.Nt, grid.Np, grid.rc, grid.ro, n_mu, n_phi, _d(chi),
                                        _KINDS[op], _d(out), threads or default_threads())
    if rc != 0:
        raise RuntimeError(f"orc_lstar_stencil_sphere failed ({rc})")
    return out.reshape(27, grid.Np, grid.Nt, grid.Nr)


def stencil_matrix_sphere(st):
    """The sparse matrix of a spherical 27-point stencil (27, Np, Nt, Nr): phi periodic, r and theta bounded
    (entries of components that land on the same voxel are summed)."""
    import scipy.sparse as sp
    _, Np, Nt, Nr = st.shape
    p, t, r = np.meshgrid(np.arange(Np), np.arange(Nt), np.arange(Nr), indexing="ij")
    v = (p * Nt + t) * Nr + r
    rows, cols, vals = [], [], []
    for c in range(27):
        dp, dt, dr = c // 9 - 1, (c // 3) % 3 - 1, c % 3 - 1
        tu, ru = t + dt, r + dr
        ok = (tu >= 0) & (tu < Nt) & (ru >= 0) & (ru < Nr)
        u = (((p + dp) % Np) * Nt + tu) * Nr + ru
        rows.append(v[ok]); cols.append(u[ok]); vals.append(st[c][ok])
    n = Nr * Nt * Np
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


from .solvers import *  # noqa: E402,F401,F403
