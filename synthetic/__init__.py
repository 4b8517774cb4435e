"""Seeded synthetic inputs for the radiative-transfer workloads.

This module only generates input fields (opacity, thermal coupling, Planck
function, boundary intensities).  It holds none of the method's arithmetic,
and both the GPU library's tests/benchmark and the oracle draw their inputs
from here.

Recipes (stand-ins for the paper's PHOENIX model structures, which are not
available; the shapes follow the paper's test setups, Sec. 3.1 and 3.2):

* stratified opacity: layer k = 0 (top) .. N-1 has geometric-mean vertical
  optical depth tau_k = tau_min * r**k with r = (tau_max/tau_min)**(1/(N-1)),
  and the layer's optical thickness tau_k (sqrt(r) - 1/sqrt(r)) is its
  opacity per unit voxel edge, so the vertical optical depth is log-uniform
  over [tau_min, tau_max];
* log-normal 3D perturbation: chi *= 10**(sigma * g) with g a Gaussian random
  field of correlation exp(-d^2 / (2 l^2)), made by FFT-convolving N(0,1) noise
  with a Gaussian of standard deviation l/sqrt(2) (periodic in x,y, generated
  on twice the depth and cropped), rescaled to zero mean and unit variance;
* eps log-uniform per voxel or per wavelength; B = 1; no incoming intensity at
  the top, I = B entering at the bottom;
* spherical shell (r_core = 1, r_out = 2, uniform radial cells): the radial
  optical depth at shell centres is log-uniform from tau_min at the outer
  shell to tau_max at the inner one (the stratified recipe along r, divided
  by the radial cell size); a wavelength batch scales it by 10**U(-2, 2);
  eps = 1e-3, B = 1, I_core = B, no diffuse incoming intensity, and a point
  source at 5 r_out on the +z axis with mean intensity B at the sub-source
  point.

All fields are generated in float64 and, for single-precision workloads,
rounded once to float32; those rounded values are the inputs of every solver.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


def stratified_chi(Nz: int, tau_min: float = 1e-4, tau_max: float = 1e4) -> np.ndarray:
    """Per-layer opacity (unit voxel edge), k = 0 the top layer."""
    if Nz == 1:
        return np.array([tau_max - tau_min], dtype=np.float64)
    lr = np.log10(tau_max / tau_min) / (Nz - 1)
    r = 10.0 ** lr
    k = np.arange(Nz, dtype=np.float64)
    tau_k = tau_min * 10.0 ** (lr * k)
    return tau_k * (np.sqrt(r) - 1.0 / np.sqrt(r))


def gaussian_random_field(Nz: int, Ny: int, Nx: int, ell: float, seed: int) -> np.ndarray:
    """Zero-mean, unit-variance field with correlation exp(-d^2/(2 ell^2))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Nz2 = 2 * Nz
    noise = rng.standard_normal((Nz2, Ny, Nx))
    sig = ell / np.sqrt(2.0)

    def kern1d(n):
        d = np.arange(n, dtype=np.float64)
        d = np.minimum(d, n - d)
        return np.exp(-0.5 * (d / sig) ** 2)

    kz = np.fft.fft(kern1d(Nz2))[:, None, None]
    ky = np.fft.fft(kern1d(Ny))[None, :, None]
    kx = np.fft.rfft(kern1d(Nx))[None, None, :]
    F = np.fft.rfftn(noise) * kz * ky * kx
    g = np.fft.irfftn(F, s=noise.shape, axes=(0, 1, 2))[:Nz]
    g = g - g.mean()
    g = g / g.std()
    return g


@dataclasses.dataclass
class BoxCase:
    """One workload on the periodic box.  Arrays are [lambda][k][y][x]."""
    name: str
    Nx: int
    Ny: int
    Nz: int
    n_mu: int
    n_phi: int
    chi: np.ndarray          # (n_lambda, Nz, Ny, Nx)
    eps: np.ndarray          # (n_lambda, Nz, Ny, Nx)
    B: np.ndarray            # (n_lambda, Nz, Ny, Nx)
    I_bc: np.ndarray         # (n_lambda, 2): intensity entering at top, at bottom
    dtype: str               # "f64" or "f32": precision of the formal solution
    tol: float = 1e-8

    @property
    def n_lambda(self) -> int:
        return self.chi.shape[0]

    @property
    def n_dir(self) -> int:
        return self.n_mu * self.n_phi

    @property
    def n_vox(self) -> int:
        return self.Nx * self.Ny * self.Nz

    def vdu_per_fs(self) -> int:
        """voxel-direction updates of one formal solution over all wavelengths."""
        return self.n_vox * self.n_dir * self.n_lambda


def _round(a: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "f32":
        return a.astype(np.float32).astype(np.float64)
    return a.astype(np.float64)


def box_stratified(N: int = 33, Nz: Optional[int] = None, n_mu: int = 8, n_phi: int = 16,
                   eps: float = 1e-2, dtype: str = "f64", tau_min: float = 1e-4,
                   tau_max: float = 1e4, name: str = "box-stratified") -> BoxCase:
    """x,y-uniform stratified slab: the 33^3, 8x16-direction FP64 workload at its defaults."""
    Nz = N if Nz is None else Nz
    chi = np.broadcast_to(stratified_chi(Nz, tau_min, tau_max)[:, None, None], (Nz, N, N))
    chi = _round(np.array(chi), dtype)[None]
    e = np.full_like(chi, eps)
    e = _round(e, dtype)
    B = np.ones_like(chi)
    I_bc = np.array([[0.0, 1.0]])
    return BoxCase(name, N, N, Nz, n_mu, n_phi, chi, e, B, I_bc, dtype, tol=1e-8)


def box_lognormal(N: int = 129, Nz: Optional[int] = None, n_mu: int = 32, n_phi: int = 64,
                  sigma_dex: float = 1.0, ell: float = 8.0, field_seed: int = 1, eps_seed: int = 101,
                  eps_range=(-6.0, 0.0), dtype: str = "f32", name: str = "box-lognormal",
                  Ny: Optional[int] = None) -> BoxCase:
    """Stratified opacity times a log-normal 3D perturbation, eps log-uniform per voxel.

    Defaults: the 129^3, 32x64-direction single-precision workload."""
    Nz = N if Nz is None else Nz
    Ny = N if Ny is None else Ny
    g = gaussian_random_field(Nz, Ny, N, ell, field_seed)
    chi = stratified_chi(Nz)[:, None, None] * 10.0 ** (sigma_dex * g)
    rng = np.random.Generator(np.random.PCG64(eps_seed))
    e = 10.0 ** rng.uniform(eps_range[0], eps_range[1], size=chi.shape)
    chi = _round(chi, dtype)[None]
    e = _round(e, dtype)[None]
    B = np.ones_like(chi)
    I_bc = np.array([[0.0, 1.0]])
    return BoxCase(name, N, Ny, Nz, n_mu, n_phi, chi, e, B, I_bc, dtype, tol=1e-8)


def box_lognormal257(dtype: str = "f32") -> BoxCase:
    """The 257^3 box with 32x16 directions: the log-normal recipe of box_lognormal
    with its own seeds (field 4, eps 104)."""
    return box_lognormal(N=257, n_mu=32, n_phi=16, field_seed=4, eps_seed=104, dtype=dtype,
                         name="box-lognormal-257")


def box_batched(N: int = 129, Nz: Optional[int] = None, n_lambda: int = 64, n_mu: int = 32,
                n_phi: int = 32, scale_seed: int = 2, eps_seed: int = 102, field_seed: int = 1,
                dtype: str = "f32", name: str = "box-batched") -> BoxCase:
    """Wavelength batch on one structure: chi_l = f_l chi_1, f_l log-uniform in [1e-3, 1e3],
    eps_l log-uniform in [1e-5, 1e-1], uniform in space per wavelength."""
    Nz = N if Nz is None else Nz
    g = gaussian_random_field(Nz, N, N, 8.0, field_seed)
    chi1 = stratified_chi(Nz)[:, None, None] * 10.0 ** g
    rs = np.random.Generator(np.random.PCG64(scale_seed))
    f = 10.0 ** rs.uniform(-3.0, 3.0, size=n_lambda)
    re = np.random.Generator(np.random.PCG64(eps_seed))
    el = 10.0 ** re.uniform(-5.0, -1.0, size=n_lambda)
    chi = _round(f[:, None, None, None] * chi1[None], dtype)
    e = _round(np.broadcast_to(el[:, None, None, None], chi.shape).copy(), dtype)
    B = np.ones_like(chi)
    I_bc = np.tile(np.array([[0.0, 1.0]]), (n_lambda, 1))
    return BoxCase(name, N, N, Nz, n_mu, n_phi, chi, e, B, I_bc, dtype, tol=1e-8)


def random_box(Nx: int, Ny: int, Nz: int, n_mu: int, n_phi: int, seed: int, dtype: str = "f64",
               n_lambda: int = 1, chi_dex=(-2.0, 2.0), eps_dex=(-3.0, 0.0),
               name: str = "box-random") -> BoxCase:
    """Small heterogeneous box with iid log-uniform fields: parity-test input."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n_lambda, Nz, Ny, Nx)
    chi = _round(10.0 ** rng.uniform(chi_dex[0], chi_dex[1], size=shape), dtype)
    e = _round(10.0 ** rng.uniform(eps_dex[0], eps_dex[1], size=shape), dtype)
    B = _round(rng.uniform(0.5, 1.5, size=shape), dtype)
    I_bc = np.stack([rng.uniform(0.0, 0.5, size=n_lambda), rng.uniform(0.5, 1.5, size=n_lambda)], axis=1)
    return BoxCase(name, Nx, Ny, Nz, n_mu, n_phi, chi, e, B, I_bc, dtype)


def random_source(shape, seed: int, lo: float = 0.0, hi: float = 1.0, dtype: str = "f64") -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return _round(rng.uniform(lo, hi, size=shape), dtype)


@dataclasses.dataclass
class SphereCase:
    """One workload on a spherical grid.  Arrays are [lambda][iphi][itheta][ir]."""
    name: str
    Nr: int
    Nt: int
    Np: int
    r_core: float
    r_out: float
    n_mu: int
    n_phi: int
    source_distance: float    # in units of r_out; 0 = no point source
    chi: np.ndarray           # (n_lambda, Np, Nt, Nr)
    eps: np.ndarray
    B: np.ndarray
    I_bc: np.ndarray          # (n_lambda, 3): I_out, I_core, J_sub
    dtype: str
    tol: float = 1e-8

    @property
    def n_lambda(self) -> int:
        return self.chi.shape[0]

    @property
    def n_dir(self) -> int:
        return self.n_mu * self.n_phi

    @property
    def n_vox(self) -> int:
        return self.Nr * self.Nt * self.Np

    def vdu_per_fs(self) -> int:
        return self.n_vox * self.n_dir * self.n_lambda


def sphere_radial(Nr: int = 97, Nt: int = 65, Np: int = 129, n_mu: int = 32, n_phi: int = 32, n_lambda: int = 16,
                  tau_min: float = 1e-6, tau_max: float = 1e6, eps: float = 1e-3, scale_seed: int = 3,
                  source_distance: float = 5.0, dtype: str = "f32", name: str = "sphere-radial") -> SphereCase:
    """Irradiated spherical shell; defaults: the 97x65x129, 32x32-direction, 16-wavelength FP32 workload."""
    r_core, r_out = 1.0, 2.0
    dr = (r_out - r_core) / Nr
    chi_r = stratified_chi(Nr, tau_min, tau_max)[::-1] / dr      # ir = 0 is the innermost shell
    rs = np.random.Generator(np.random.PCG64(scale_seed))
    f = 10.0 ** rs.uniform(-2.0, 2.0, size=n_lambda)
    chi = f[:, None, None, None] * np.broadcast_to(chi_r[None, None, None, :], (1, Np, Nt, Nr))
    chi = _round(chi, dtype)
    e = _round(np.full_like(chi, eps), dtype)
    B = np.ones_like(chi)
    I_bc = np.tile(np.array([[0.0, 1.0, 1.0]]), (n_lambda, 1))
    return SphereCase(name, Nr, Nt, Np, r_core, r_out, n_mu, n_phi, source_distance, chi, e, B, I_bc, dtype)


def random_sphere(Nr: int, Nt: int, Np: int, n_mu: int, n_phi: int, seed: int, dtype: str = "f64",
                  n_lambda: int = 1, source_distance: float = 5.0, chi_dex=(-1.0, 1.5), eps_dex=(-3.0, 0.0),
                  name: str = "sphere-random") -> SphereCase:
    """Small heterogeneous spherical grid with iid log-uniform fields: parity-test input."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n_lambda, Np, Nt, Nr)
    chi = _round(10.0 ** rng.uniform(chi_dex[0], chi_dex[1], size=shape), dtype)
    e = _round(10.0 ** rng.uniform(eps_dex[0], eps_dex[1], size=shape), dtype)
    B = _round(rng.uniform(0.5, 1.5, size=shape), dtype)
    I_bc = _round(np.stack([rng.uniform(0.0, 0.3, size=n_lambda), rng.uniform(0.5, 1.5, size=n_lambda),
                            rng.uniform(0.5, 2.0, size=n_lambda)], axis=1), dtype)
    return SphereCase(name, Nr, Nt, Np, 1.0, 2.0, n_mu, n_phi, source_distance, chi, e, B, I_bc, dtype)


def fingerprint(case) -> str:
    """SHA-256 (hex) of a workload's input arrays and quadrature: the key under
    which a stored solution of that workload is filed.  Inputs only: the arrays
    are hashed as float64 in C order together with their shape."""
    import hashlib
    h = hashlib.sha256()
    for name in ("chi", "eps", "B", "I_bc"):
        a = np.ascontiguousarray(getattr(case, name), dtype=np.float64)
        h.update(name.encode())
        h.update(np.asarray(a.shape, dtype=np.int64).tobytes())
        h.update(a.tobytes())
    h.update(np.asarray([case.n_mu, case.n_phi], dtype=np.int64).tobytes())
    return h.hexdigest()
