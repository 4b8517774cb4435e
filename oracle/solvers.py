"""Oracle solvers around the FP64 formal solution (TEST INFRASTRUCTURE ONLY).

All of it is plain numpy on top of the C formal solution:
  * ``ali``      -- operator-splitting iteration with a diagonal Lambda*
                    (Sec. 2.2, eq. (alo)), optionally Ng-accelerated
  * ``bicgstab`` -- BiCGStab on (1 - (1-eps) Lambda) S = (1-eps) Lambda_bc + eps B,
                    the solver the paper lists for the OS system (Sec. 4)
  * ``lambda_matrix`` / ``direct`` -- Lambda built column by column and solved
                    by LU; Lambda* = Lambda is "a direct solution by matrix
                    inversion" (Sec. 2.2)
"""
from __future__ import annotations

import numpy as np

__all__ = ["BoxProblem", "Plane1DProblem", "SphereProblem", "ali", "ng_extrapolate", "bicgstab",
           "lambda_matrix", "direct", "lambda_iteration_radius", "os_colours", "gauss_seidel"]


class BoxProblem:
    """One wavelength on the periodic box: chi, eps, B of shape (Nz, Ny, Nx)."""

    periodic_axes = (False, True, True)

    def __init__(self, chi, eps, B, I_top, I_bot, n_mu, n_phi, kind="linear", threads=None):
        from . import fs_box
        self._fs_box = fs_box
        self.chi = np.ascontiguousarray(chi, dtype=np.float64)
        shape = self.chi.shape
        self.eps = np.broadcast_to(np.asarray(eps, dtype=np.float64), shape).copy()
        self.B = np.broadcast_to(np.asarray(B, dtype=np.float64), shape).copy()
        self.I_top, self.I_bot = float(I_top), float(I_bot)
        self.n_mu, self.n_phi = int(n_mu), int(n_phi)
        self.kind = kind
        self.threads = threads
        self.n_fs = 0
        self._lstar = None

    @property
    def shape(self):
        return self.chi.shape

    def fs(self, S, bc=True, want_lstar=False):
        self.n_fs += 1
        J, L = self._fs_box(self.chi, S, self.I_top if bc else 0.0, self.I_bot if bc else 0.0,
                            self.n_mu, self.n_phi, self.kind, self.threads, want_lstar)
        if want_lstar:
            self._lstar = L
        return (J, L) if want_lstar else J

    def lstar(self):
        if self._lstar is None:
            self.fs(np.zeros(self.shape), want_lstar=True)
        return self._lstar

    def lstar_stencil(self):
        """Nearest-neighbour Lambda* (27, Nz, Ny, Nx) of the operator selected by kind."""
        from . import lstar_stencil
        return lstar_stencil(self.chi, self.n_mu, self.n_phi, self.kind, self.threads)

    def lstar_nonlocal(self):
        """The nearest-neighbour Lambda* as a sparse matrix."""
        from . import stencil_matrix
        return stencil_matrix(self.lstar_stencil())


class Plane1DProblem(BoxProblem):
    """x,y-homogeneous box reduced to its layers: chi, eps, B of shape (Nz,)."""

    def __init__(self, chi_k, eps, B, I_top, I_bot, n_mu, n_phi, kind="linear"):
        from . import fs_1d
        self._fs_1d = fs_1d
        self.chi = np.ascontiguousarray(chi_k, dtype=np.float64)
        shape = self.chi.shape
        self.eps = np.broadcast_to(np.asarray(eps, dtype=np.float64), shape).copy()
        self.B = np.broadcast_to(np.asarray(B, dtype=np.float64), shape).copy()
        self.I_top, self.I_bot = float(I_top), float(I_bot)
        self.n_mu, self.n_phi = int(n_mu), int(n_phi)
        self.kind = kind
        self.threads = None
        self.n_fs = 0
        self._lstar = None

    def fs(self, S, bc=True, want_lstar=False):
        self.n_fs += 1
        J, L = self._fs_1d(self.chi, S, self.I_top if bc else 0.0, self.I_bot if bc else 0.0,
                           self.n_mu, self.n_phi, self.kind)
        if want_lstar:
            self._lstar = L
        return (J, L) if want_lstar else J


class SphereProblem(BoxProblem):
    """One wavelength on a spherical grid: chi, eps, B of shape (Np, Nt, Nr);
    boundary values I_out (entering through r_out), I_core (leaving the core)
    and the point-source irradiation J_sub at distance dsrc * r_out (Sec. 3.2)."""

    def __init__(self, grid, chi, eps, B, I_out, I_core, n_mu, n_phi, dsrc=0.0, J_sub=0.0, kind="linear",
                 threads=None):
        from . import fs_sphere
        self._fs_sphere = fs_sphere
        self.grid = grid
        self.chi = np.ascontiguousarray(chi, dtype=np.float64).reshape(grid.Np, grid.Nt, grid.Nr)
        shape = self.chi.shape

        def field(x):
            x = np.asarray(x, dtype=np.float64)
            return (x.reshape(shape) if x.size == self.chi.size else np.broadcast_to(x, shape)).copy()
        self.eps = field(eps)
        self.B = field(B)
        self.I_out, self.I_core = float(I_out), float(I_core)
        self.dsrc, self.J_sub = float(dsrc), float(J_sub)
        self.n_mu, self.n_phi = int(n_mu), int(n_phi)
        self.kind = kind
        self.threads = threads
        self.n_fs = 0
        self._lstar = None

    periodic_axes = (True, False, False)

    def lstar_stencil(self):
        """Nearest-neighbour Lambda* (27, Np, Nt, Nr) of the operator selected by kind."""
        from . import lstar_stencil_sphere
        return lstar_stencil_sphere(self.grid, self.n_mu, self.n_phi, self.chi, self.kind, self.threads)

    def lstar_nonlocal(self):
        from . import stencil_matrix_sphere
        return stencil_matrix_sphere(self.lstar_stencil())

    def fs(self, S, bc=True, want_lstar=False):
        self.n_fs += 1
        core = np.full(self.chi.size, self.I_core if bc else 0.0)
        J, L = self._fs_sphere(self.grid, self.n_mu, self.n_phi, self.chi, S, core,
                               I_out=self.I_out if bc else 0.0, dsrc=self.dsrc, B_sub=self.J_sub if bc else 0.0,
                               kind=self.kind, threads=self.threads)
        J = J.reshape(self.chi.shape)
        L = L.reshape(self.chi.shape)
        if want_lstar:
            self._lstar = L
        return (J, L) if want_lstar else J


def ng_extrapolate(x0, x1, x2, x3):
    """Ng (1974) acceleration in the weighted least-squares form (Auer 1987).

    With delta_i = x_i - x_{i+1}, Q1 = delta_0 - delta_1, Q2 = delta_0 - delta_2,
    choose (a, b) minimising sum w (delta_0 - a Q1 - b Q2)^2 with w = 1/x0^2,
    and return (1-a-b) x0 + a x1 + b x2.  Returns None if the 2x2 system is
    (nearly) singular.
    """
    d0, d1, d2 = x0 - x1, x1 - x2, x2 - x3
    Q1, Q2 = d0 - d1, d0 - d2
    w = 1.0 / (x0 * x0)
    A11 = np.sum(w * Q1 * Q1)
    A12 = np.sum(w * Q1 * Q2)
    A22 = np.sum(w * Q2 * Q2)
    b1 = np.sum(w * d0 * Q1)
    b2 = np.sum(w * d0 * Q2)
    det = A11 * A22 - A12 * A12
    if not (det > 1e-10 * A11 * A22) or not np.isfinite(det):
        return None
    a = (b1 * A22 - b2 * A12) / det
    b = (b2 * A11 - b1 * A12) / det
    return (1.0 - a - b) * x0 + a * x1 + b * x2


def os_colours(shape, periodic=(False, True, True)):
    """Colour class of every voxel of a 3-axis grid for the Gauss-Seidel sweeps
    of the OS system: c0*9 + c1*3 + c2 with c_i = index mod 2 along axis i,
    except that on an odd periodic axis of length >= 3 the last index takes
    class 2, since it neighbours the first one across the period.  The box
    (Nz, Ny, Nx) is periodic in y and x; the sphere (Np, Nt, Nr) in phi.
    (A reading: the paper names Gauss-Seidel without an ordering.)"""
    def axis(N, per):
        c = np.arange(N) % 2
        if per and N >= 3 and N % 2 == 1:
            c[N - 1] = 2
        return c

    a, b, c = (axis(N, per) for N, per in zip(shape, periodic))
    return a[:, None, None] * 9 + b[None, :, None] * 3 + c[None, None, :]


def _gs_plan(A, colours):
    import scipy.sparse as sps
    A = sps.csr_matrix(A)
    d = A.diagonal()
    off = (A - sps.diags(d)).tocsr()
    cls = np.asarray(colours).ravel()
    return d, [(idx, off[idx]) for idx in (np.flatnonzero(cls == c) for c in range(27)) if idx.size]


def _gs_sweeps(plan, r, x, sweeps):
    d, blocks = plan
    x = np.array(x, dtype=np.float64)
    for _ in range(sweeps):
        for idx, rows in blocks:
            x[idx] = (r[idx] - rows @ x) / d[idx]
    return x


def gauss_seidel(A, r, x, colours, sweeps):
    """``sweeps`` Gauss-Seidel sweeps on A x = r (A sparse): each voxel v in
    turn, in ascending colour class, takes x_v = (r_v - sum_{u != v} A_vu x_u)
    / A_vv with the newest values of the others.  No two voxels of one class
    are coupled (see os_colours), so the voxels of a class are updated
    together."""
    return _gs_sweeps(_gs_plan(A, colours), r, x, sweeps)


def ali(prob, tol=1e-8, max_iter=10000, ng=True, ng_start=4, ng_every=4, J0=None,
        lstar=None, record=False, inner_jacobi=0, inner_gs=0):
    """Operator-splitting (ALI) iteration (Sec. 2.2, eq. (alo)).

    Each step: J_fs = Lambda S_old (+ boundary term);
               [1 - Lambda*(1-eps)] J_new = J_fs - Lambda*(1-eps) J_old;
               S_new = (1-eps) J_new + eps B.
    Stops when max |J_new - J_old| / |J_new| < tol.  Ng acceleration is applied
    to the last four iterates every ``ng_every`` plain steps once ``ng_start``
    steps have been taken; the iterate history restarts after each application.
    ``lstar`` overrides the diagonal (e.g. zeros for plain Lambda iteration, a
    full matrix for the Lambda* = Lambda special case, or a scipy sparse matrix
    such as the nearest-neighbour Lambda*).  With a sparse Lambda* the OS
    system is solved exactly, or, with ``inner_jacobi`` = k > 0, by k Jacobi
    sweeps on [1 - Lambda*(1-eps)] dJ = J_fs - J_old started from the
    diagonal solution, or with ``inner_gs`` = k > 0 by k Gauss-Seidel sweeps
    in colour order (see gauss_seidel) from the same start (the OS solvers of
    Sec. 3).
    """
    import scipy.sparse as sps
    import scipy.sparse.linalg as spla
    eps, B = prob.eps, prob.B
    L = prob.lstar() if lstar is None else lstar
    J = B.copy() if J0 is None else np.array(J0, dtype=np.float64)
    S = (1.0 - eps) * J + eps * B
    hist = []
    trace = []
    converged = False
    it = 0
    if sps.issparse(L):
        om = (1.0 - eps).ravel()
        A = (sps.identity(J.size, format="csr") - L @ sps.diags(om)).tocsr()
        Adiag = A.diagonal()
        Aoff = (A - sps.diags(Adiag)).tocsr()
        gs_plan = _gs_plan(A, os_colours(J.shape, prob.periodic_axes)) if inner_gs > 0 else None
    for it in range(1, max_iter + 1):
        Jfs = prob.fs(S)
        if sps.issparse(L):
            r = (Jfs - J).ravel()
            if inner_gs > 0:
                x = _gs_sweeps(gs_plan, r, r / Adiag, inner_gs)
            elif inner_jacobi > 0:
                x = r / Adiag
                for _ in range(inner_jacobi):
                    x = (r - Aoff @ x) / Adiag
            else:
                x = spla.spsolve(A.tocsc(), r)
            Jn = J + x.reshape(J.shape)
        elif np.ndim(L) == 2 and L.shape[0] == J.size:
            # full-matrix Lambda*: solve [1 - Lambda*(1-eps)] J_new = J_fs - Lambda*(1-eps) J_old
            A = np.eye(J.size) - L * (1.0 - eps.ravel())[None, :]
            rhs = Jfs.ravel() - L @ ((1.0 - eps.ravel()) * J.ravel())
            Jn = np.linalg.solve(A, rhs).reshape(J.shape)
        else:
            Jn = (Jfs - L * (1.0 - eps) * J) / (1.0 - L * (1.0 - eps))
        rel = float(np.max(np.abs(Jn - J) / np.abs(Jn)))
        J = Jn
        S = (1.0 - eps) * J + eps * B
        if record:
            trace.append(rel)
        if rel < tol:
            converged = True
            break
        hist.append(J.copy())
        if len(hist) > 4:
            hist.pop(0)
        if ng and it >= ng_start and len(hist) == 4 and ng_every > 0:
            x = ng_extrapolate(hist[3], hist[2], hist[1], hist[0])
            if x is not None:
                J = x
                S = (1.0 - eps) * J + eps * B
            hist = []
    return dict(J=J, S=S, iters=it, converged=converged, n_fs=it, trace=trace)


def bicgstab(prob, rtol=1e-12, max_iter=5000, S0=None):
    """BiCGStab (van der Vorst 1992, as in the 'Templates' book) on
        (1 - (1-eps) Lambda) S = (1-eps) Lambda_bc + eps B
    with the diagonal preconditioner 1 - (1-eps) Lambda*.  Returns the fixed
    point S and J = Lambda S + Lambda_bc (one more formal solution).
    """
    eps, B = prob.eps, prob.B
    om = 1.0 - eps
    Lst = prob.lstar()
    Mdiag = 1.0 - om * Lst
    Jbc = prob.fs(np.zeros(prob.shape), bc=True)

    def A(x):
        return x - om * prob.fs(x, bc=False)

    b = om * Jbc + eps * B
    x = (B.copy() if S0 is None else np.array(S0, dtype=np.float64))
    r = b - A(x)
    rhat = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(x); p = np.zeros_like(x)
    bnorm = np.linalg.norm(b)
    it = 0
    for it in range(1, max_iter + 1):
        rho = float(np.vdot(rhat, r))
        if rho == 0.0:
            break
        beta = (rho / rho_old) * (alpha / omega) if it > 1 else 0.0
        p = r + beta * (p - omega * v) if it > 1 else r.copy()
        phat = p / Mdiag
        v = A(phat)
        alpha = rho / float(np.vdot(rhat, v))
        s = r - alpha * v
        if np.linalg.norm(s) <= rtol * bnorm:
            x = x + alpha * phat
            r = s
            break
        shat = s / Mdiag
        t = A(shat)
        omega = float(np.vdot(t, s)) / float(np.vdot(t, t))
        x = x + alpha * phat + omega * shat
        r = s - omega * t
        rho_old = rho
        if np.linalg.norm(r) <= rtol * bnorm:
            break
    S = x
    J = prob.fs(S, bc=True)
    res = float(np.linalg.norm(b - A(S)) / bnorm)
    return dict(J=J, S=S, iters=it, residual=res)


def lambda_matrix(prob):
    """Lambda column by column (unit S per voxel, zero boundary) and Lambda_bc."""
    n = int(np.prod(prob.shape))
    Lam = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[:] = 0.0
        e[j] = 1.0
        Lam[:, j] = prob.fs(e.reshape(prob.shape), bc=False).ravel()
    Jbc = prob.fs(np.zeros(prob.shape), bc=True).ravel()
    return Lam, Jbc


def direct(prob, Lam=None, Jbc=None):
    """Fixed point by LU: (1 - diag(1-eps) Lambda) S = (1-eps) Lambda_bc + eps B."""
    if Lam is None:
        Lam, Jbc = lambda_matrix(prob)
    om = (1.0 - prob.eps).ravel()
    A = np.eye(Lam.shape[0]) - om[:, None] * Lam
    S = np.linalg.solve(A, om * Jbc + prob.eps.ravel() * prob.B.ravel())
    J = Lam @ S + Jbc
    return dict(J=J.reshape(prob.shape), S=S.reshape(prob.shape), Lam=Lam, Jbc=Jbc)


def lambda_iteration_radius(prob, n_iter=200, seed=0):
    """Spectral radius of the Lambda-iteration amplification (1-eps) Lambda by power iteration."""
    rng = np.random.default_rng(seed)
    x = rng.random(prob.shape) + 0.5
    lam = 0.0
    for _ in range(n_iter):
        y = (1.0 - prob.eps) * prob.fs(x, bc=False)
        lam = float(np.linalg.norm(y) / np.linalg.norm(x))
        x = y / np.linalg.norm(y)
    return lam
