"""Writes the double-precision fixed point of the 129^3 log-normal box with the oracle only.

Workload: the 129^3 periodic box of ``synthetic.box_lognormal`` (stratified
opacity times a log-normal perturbation, eps log-uniform 1e-6..1 per voxel,
B = 1, no light entering at the top, I = B entering at the bottom), 32 x 64
directions, inputs rounded once to float32 (the single-precision workload's
inputs, read exactly in float64 by the oracle).

Solver: the oracle's operator-splitting iteration (Sec. 2.2, eq. (alo)) with
the nearest-neighbour Lambda* of the linear-interpolation operator (Sec. 2:
the paper's production choice; Sec. 3: Jacobi as the OS solver, 16 sweeps per
step started from the diagonal solution) and Ng acceleration every 4 steps.
The fixed point does not depend on Lambda*, Ng or the sweep count; they only
shorten the path.  The run is split into chunks of 8 steps, which reproduces
the unsplit Ng schedule exactly (the Ng history restarts after every
extrapolation), and J is checkpointed between chunks.  It stops when the
largest relative change per step stops falling (the double-precision floor
of the iteration) or after ``--max-steps``.  One more formal solution then
gives the residual max |Lambda S(J) + Lambda_bc - J| / J of the stored J.

Output (``numpy.savez_compressed``, no pickled objects): ``J`` float32
(Nz, Ny, Nx), ``fingerprint`` (``synthetic.fingerprint`` of the workload),
``trace`` (largest relative change of every step), ``residual``, ``steps``,
``threads``, ``seconds``.

Only ``oracle/`` and ``synthetic/`` are used.  On 8 host threads the run takes
about three hours (one formal solution about 290 s).

    python tests/golden/make_box129_fixed_point.py --out tests/golden/box129_fixed_point.npz
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic as sy  # noqa: E402

CHUNK = 8          # steps per chunk: a multiple of the Ng period, so chunks reproduce the unsplit run
JACOBI_SWEEPS = 16


def log(msg: str) -> None:
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


class LoggedProblem(oracle.BoxProblem):
    """The oracle's box problem, printing one line per formal solution."""

    def fs(self, S, bc=True, want_lstar=False):
        t = time.time()
        out = super().fs(S, bc=bc, want_lstar=want_lstar)
        log(f"formal solution {self.n_fs} ({time.time() - t:.0f} s)")
        return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "box129_fixed_point.npz"))
    ap.add_argument("--work", default=os.path.join(ROOT, "_work", "golden129"),
                    help="checkpoint directory (J after every chunk)")
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    ap.add_argument("--max-steps", type=int, default=48)
    ap.add_argument("--N", type=int, default=129, help="grid size (smaller values for a quick trial)")
    args = ap.parse_args()

    case = sy.box_lognormal(N=args.N, dtype="f32")
    fp = sy.fingerprint(case)
    log(f"workload {case.name} {case.Nx}x{case.Ny}x{case.Nz}, {case.n_mu}x{case.n_phi} directions, "
        f"fingerprint {fp[:16]}, {args.threads} threads")
    prob = LoggedProblem(case.chi[0], case.eps[0], case.B[0], case.I_bc[0, 0], case.I_bc[0, 1],
                         case.n_mu, case.n_phi, kind="linear", threads=args.threads)
    t_start = time.time()
    os.makedirs(args.work, exist_ok=True)
    ck = os.path.join(args.work, f"checkpoint_{fp[:16]}.npz")
    J = None
    trace: list[float] = []
    if os.path.exists(ck):
        with np.load(ck) as z:
            J = z["J"].copy()
            trace = [float(x) for x in z["trace"]]
        log(f"resuming after {len(trace)} steps from {ck}")

    t = time.time()
    L = prob.lstar_nonlocal()
    log(f"nearest-neighbour Lambda* built ({time.time() - t:.0f} s, {L.nnz} elements)")

    while len(trace) < args.max_steps:
        r = oracle.ali(prob, tol=0.0, max_iter=CHUNK, ng=True, ng_start=4, ng_every=4, J0=J, lstar=L,
                       record=True, inner_jacobi=JACOBI_SWEEPS)
        J = r["J"]
        trace += [float(x) for x in r["trace"]]
        np.savez(ck, J=J, trace=np.asarray(trace))
        log(f"steps {len(trace)}: last change {trace[-1]:.3e}, chunk minimum {min(r['trace']):.3e}")
        if len(trace) >= 2 * CHUNK:
            prev, last = min(trace[-2 * CHUNK:-CHUNK]), min(trace[-CHUNK:])
            if last > 0.5 * prev:
                log("change per step no longer falling: double-precision floor reached")
                break

    S = (1.0 - prob.eps) * J + prob.eps * prob.B
    Jfs = prob.fs(S)
    residual = float(np.max(np.abs(Jfs - J) / np.abs(J)))
    seconds = time.time() - t_start
    log(f"residual max|Lambda S(J) + Lambda_bc - J|/J = {residual:.3e}; {seconds:.0f} s in all")
    np.savez_compressed(args.out, J=J.astype(np.float32), fingerprint=np.asarray(fp),
                        trace=np.asarray(trace), residual=np.asarray(residual),
                        steps=np.asarray(len(trace)), threads=np.asarray(args.threads),
                        seconds=np.asarray(seconds))
    log(f"wrote {args.out} ({os.path.getsize(args.out) / 1e6:.1f} MB)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
