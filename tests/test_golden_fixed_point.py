"""The stored fixed point of the 129^3 log-normal box (CPU).

tests/golden/box129_fixed_point.npz is written by
tests/golden/make_box129_fixed_point.py from the oracle alone: FP64
non-local Ng-ALI (Sec. 2.2, eq. (alo); the nearest-neighbour Lambda* of
Sec. 2 with Jacobi OS sweeps, Sec. 3) until the change per step stopped
falling.  These checks hold the file to the workload it names and to the
fixed-point equation J = Lambda S(J) + Lambda_bc, S = (1-eps) J + eps B,
evaluated by the oracle's formal solution at sampled voxels, one by one."""
import os

import numpy as np
import pytest

import synthetic as sy

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "box129_fixed_point.npz")


@pytest.fixture(scope="module")
def golden():
    with np.load(GOLDEN, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def test_file_matches_the_workload(golden):
    case = sy.box_lognormal(dtype="f32")
    assert str(golden["fingerprint"]) == sy.fingerprint(case)
    assert golden["J"].shape == (case.Nz, case.Ny, case.Nx) and golden["J"].dtype == np.float32
    assert np.all(np.isfinite(golden["J"])) and float(golden["J"].min()) > 0.0


def test_run_reached_the_double_precision_floor(golden):
    """The last 8 steps changed J by less than 2e-8 (the FP64 rounding of the
    formal solution amplified by the OS update at eps ~ 1e-6), and the full
    formal solution of the stored FP64 iterate left a residual below 1e-9."""
    trace = np.asarray(golden["trace"])
    assert int(golden["steps"]) == trace.size >= 24
    assert float(trace[-8:].max()) < 2e-8
    assert float(golden["residual"]) < 1e-9


def test_sampled_fixed_point_equation(orc, golden):
    """|Lambda S(J) + Lambda_bc - J| / J at 24 voxels, with S from the stored
    float32 J: the float32 rounding of J (6e-8) sets the level."""
    case = sy.box_lognormal(dtype="f32")
    J = golden["J"].astype(np.float64)
    eps, B = case.eps[0].astype(np.float64), case.B[0].astype(np.float64)
    S = (1.0 - eps) * J + eps * B
    vox = np.unique(np.random.default_rng(0).integers(0, J.size, 24))
    Js, _ = orc.fs_box_sampled(case.chi[0], S, case.I_bc[0, 0], case.I_bc[0, 1], case.n_mu, case.n_phi, vox)
    r = np.abs(Js - J.ravel()[vox]) / J.ravel()[vox]
    print("sampled residual", r.max())
    assert r.max() < 2e-7
