#!/usr/bin/env python3
"""Throughput benchmark of the radiative-transfer hot path on one MI355X.

One step = one operator-splitting (ALI) iteration through the C ABI
(rt_ali_step), replayed as a captured HIP graph: the single-precision formal
solution of every (wavelength, direction) item in one persistent launch, the
fixed-order reduction of the workgroup partial sums, the operator-splitting
update of J and S (double precision), the per-wavelength convergence norm,
and Ng extrapolation (double precision) every fourth step.  The default
workload is the wavelength batch: 64 wavelengths of uneven optical depth on
the 129^3 periodic box with 1024 directions.  The metric is voxel-direction
updates per second (VDU/s): voxels x directions x wavelengths of one formal
solution, divided by the time of one step.

Prints one JSON line: the throughput, the roofline position of the timed
kernel (algorithmic flops of a characteristic point over its measured launch
time against the vector ALU peak, and algorithmic bytes of a voxel-direction
update against the HBM peak), its HBM traffic when counters taken on the
current kernel source and launch shape are on file, the oracle's CPU rate on
a sample, and -- as extra keys -- the single-wavelength 129^3 x 2048 line,
one GPU's share of a solid-angle split and the time to solution.
"""
import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic floating-point operations of one characteristic point (one
# voxel visit of one ray): optical step 3, exp 1, moments 5, reciprocal of
# D D'(D+D') 4, alpha 7, beta 4, gamma 4, intensity update 8 (4 FMA), J 2.
FLOPS_PER_POINT = 38
# Non-packed vector issue rate of MI355X: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
# = 39.3e12 lane-ops/s, i.e. 78.6 TFLOP/s counting an FMA as 2 (the FP64
# vector peak; non-packed FP32 issues at the same rate).
PEAK_TFLOPS = 78.6
# HBM3E peak of MI355X and the algorithmic bytes of one voxel-direction update
# of a single-precision sweep: chi and S of the voxel read once per direction.
PEAK_HBM_GBS = 8000.0
BYTES_PER_VDU = 8
GOLDEN_129 = os.path.join(ROOT, "tests", "golden", "box129_fixed_point.npz")

WORKLOADS = {
    "lognormal129": dict(N=129, n_mu=32, n_phi=64),
    "lognormal65": dict(N=65, n_mu=16, n_phi=32),
    # the 257^3 box (band tiles: a 257 x 257 layer does not fit one LDS tile; not the default line)
    "lognormal257": dict(N=257, n_mu=32, n_phi=16, field_seed=4, eps_seed=104),
    # 64 wavelengths of uneven optical depth in one launch per step (not the default line)
    "batched129": dict(N=129, n_mu=32, n_phi=32, n_lambda=64),
    # irradiated spherical shell, 16 wavelengths (not the default line)
    "sphere97": dict(Nr=97, Nt=65, Np=129, n_mu=32, n_phi=32, n_lambda=16),
}


def progress(msg: str) -> None:
    """One progress line on stderr (stdout carries only the result line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def fs_source_hash() -> str:
    """Hash of the box sweep kernel's sources (the kernel file and its point arithmetic)."""
    h = hashlib.sha256()
    for name in ("fs_box.hip", "fs_point.hpp"):
        with open(os.path.join(ROOT, "paper_2102_01734_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str, ls: dict, profiles_dir: str = os.path.join(ROOT, "profiles")):
    """HBM bytes per launch from a committed counter summary of this workload
    (profiles/fs_box_<workload>_traffic*.md) taken on the current kernel source
    and on this launch shape (`ls` as Grid.launch_shape() gives it); else None."""
    here = (str(ls["threads"]), str(ls["rays"]), str(ls["bundles"]), "band" if ls["band"] else "layer")
    for path in sorted(glob.glob(os.path.join(profiles_dir, f"fs_box_{workload}_traffic*.md"))):
        txt = open(path).read()
        m_hash = re.search(r"fs_box\.hip sha256\[:16\]:\s*([0-9a-f]+)", txt)
        m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
        m_shape = re.search(r"launch_shape:\s*(\d+),(\d+),(\d+),(band|layer)", txt)
        if not m_hash or not m_bytes or not m_shape or m_hash.group(1) != fs_source_hash():
            continue
        if m_shape.groups() == here:
            return float(m_bytes.group(1))
    return None


def cpu_baseline(case, n_sub: int, n_sub_1: int, lam: int = 0):
    """The oracle, as it stands, on a bounded sample of wavelength `lam`: all
    voxels, n_sub of the directions spread over the sphere on all host
    threads, and n_sub_1 of them on one thread."""
    import numpy as np

    import oracle
    import synthetic as sy
    nd = case.n_dir
    S = sy.random_source(case.chi.shape[1:], seed=7, lo=0.2, hi=1.0, dtype="f32")
    chi = case.chi[lam]
    threads = oracle.default_threads()
    oracle.fs_box_dirs(chi[:2], S[:2], 0.0, 1.0, case.n_mu, case.n_phi, np.array([0], np.int32), threads=threads)

    def timed(n, th):
        dirs = np.unique(np.linspace(0, nd - 1, n).round().astype(np.int32))
        t0 = time.perf_counter()
        oracle.fs_box_dirs(chi, S, case.I_bc[lam, 0], case.I_bc[lam, 1], case.n_mu, case.n_phi, dirs, threads=th)
        wall = time.perf_counter() - t0
        return case.n_vox * dirs.size / wall, dirs.size, wall

    v, nd_all, wall = timed(n_sub, threads)
    v1, nd_1, wall1 = timed(n_sub_1, 1)
    what = f"wavelength {lam} of {case.n_lambda}, " if case.n_lambda > 1 else ""
    return {"value": v, "unit": "VDU/s", "cores": threads, "kind": "oracle",
            "sample": f"one FP64 formal solution of {what}{nd_all} of the {nd} directions over all "
                      f"{case.n_vox} voxels ({wall:.1f} s wall on {threads} threads)",
            "single_core": {"value": v1, "unit": "VDU/s", "cores": 1,
                            "sample": f"{nd_1} of the {nd} directions, all voxels ({wall1:.1f} s wall)"}}


def one_gpu_share(case, shape, n_gpus: int = 8, reps: int = 3):
    """One GPU's part of an n_gpus solid-angle decomposition: the single-precision
    formal solution over shard 0 of the visit-balanced direction shards (no
    all-reduce, which this one-GPU run cannot show).  Two layouts are timed:
    the full run's launch shape (tuned on all directions: few directions leave
    few workgroups per direction and the shallowest sets the time) and band
    tiles autotuned on the shard's own directions (more row bundles per
    direction); the faster one is reported."""
    import torch

    import paper_2102_01734_amd as rt
    import synthetic as sy
    dev = dict(dtype=torch.float32, device="cuda")
    chi = torch.tensor(case.chi, **dev)
    S = torch.tensor(sy.random_source(case.chi.shape, seed=7, lo=0.2, hi=1.0, dtype="f32"), **dev)
    Ib = torch.tensor(case.I_bc, **dev)
    M = [rt.rt_box_template(case.Nz, case.n_mu, case.n_phi, d)["s"].size for d in range(case.n_dir)]

    def timed(tune_on_share):
        g = rt.Grid(case.Nx, case.Ny, case.Nz, case.n_mu, case.n_phi, "f32", 1, band_tiles=tune_on_share)
        shards = [g.shard_directions(n_gpus, k) for k in range(n_gpus)]
        dirs = shards[0]
        if tune_on_share:
            g.autotune_dirs(chi[:1].contiguous(), S[:1].contiguous(), dirs)
        elif shape:
            g.set_launch_shape(*shape)
        ls = g.launch_shape()
        g.formal_solution_dirs(chi, S, dirs, I_bc=Ib)
        torch.cuda.synchronize()
        rt.rt_profile_read(g.handle)
        rt.rt_profile_enable(g.handle, True)
        t0 = time.perf_counter()
        for _ in range(reps):
            g.formal_solution_dirs(chi, S, dirs, I_bc=Ib)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        fs_ms, n, _ = rt.rt_profile_read(g.handle)
        g.close()
        return shards, dirs, wall, fs_ms / max(n, 1), ls

    shards, dirs, wall_l, k_l, ls_l = timed(False)
    _, _, wall_b, k_b, ls_b = timed(True)
    loads = [sum(M[d] for d in s) for s in shards]
    wall, kern, ls = (wall_b, k_b, ls_b) if wall_b < wall_l else (wall_l, k_l, ls_l)
    return {"gpus": n_gpus, "directions": int(len(dirs)), "visit_imbalance": max(loads) / (sum(loads) / n_gpus),
            "ms_per_fs": wall * 1e3, "kernel_ms": kern,
            "vdu_per_s": case.n_vox * len(dirs) / wall,
            "launch_shape": {"threads": ls["threads"], "rays_per_thread": ls["rays"], "bundles": ls["bundles"],
                             "tiles": "band" if ls["band"] else "layer"},
            "full_run_shape_ms_per_fs": wall_l * 1e3, "share_tuned_band_ms_per_fs": wall_b * 1e3}


def time_to_solution(case, net_every: int = 12, tol: float = 1e-6, shape=None, net_path=None):
    """Wall seconds of rt_solve, both to the stopping tolerance `tol` (which lands
    below 1e-5 relative error on this workload) and to the target error 1e-5
    itself (the fewest steps whose J is within 1e-5 of the reference, found by
    re-running with a step limit), for plain double-precision Ng-ALI,
    single-precision defect-corrected Ng-ALI, the latter with the learned
    correction, Ng-ALI with the nearest-neighbour Lambda* (single precision
    with Jacobi and with Gauss-Seidel OS sweeps, double precision with Jacobi;
    the stencil build is inside the timed call) and BiCGStab (the
    single-precision runs use the launch shape tuned for the throughput line,
    the double-precision runs one tuned on a double-precision grid); each
    with its max relative J error against a double-precision Ng-ALI solution
    iterated to 1e-9 change (at most 80 steps)."""
    import torch

    import paper_2102_01734_amd as rt
    blob_path = net_path or os.path.join(ROOT, "paper_2102_01734_amd", "data", "precond_box.rtun")
    blob = open(blob_path, "rb").read()
    import synthetic as sy
    # the double-precision legs get their own tuned sweep shape (setup, not timed)
    g64 = rt.Grid(case.Nx, case.Ny, case.Nz, case.n_mu, case.n_phi, "f64", 1)
    chi64 = torch.tensor(case.chi[:1], dtype=torch.float64, device="cuda")
    S64 = torch.tensor(sy.random_source(case.chi[:1].shape, seed=7, lo=0.2, hi=1.0), dtype=torch.float64,
                       device="cuda")
    g64.autotune(chi64, S64)
    ls64 = g64.launch_shape()
    shape64 = (ls64["threads"], ls64["rays"], bool(ls64["band"]))
    g64.close()
    del chi64, S64

    def run(prec, tol_, max_iter, net=0, method="ali", nonlocal_lstar=False, os_method="jacobi"):
        dt = torch.float32 if prec == "f32" else torch.float64
        dev = dict(dtype=dt, device="cuda")
        g = rt.Grid(case.Nx, case.Ny, case.Nz, case.n_mu, case.n_phi, prec, 1, nonlocal_lstar=nonlocal_lstar)
        if prec == "f32" and shape:
            g.set_launch_shape(*shape)  # the single-precision sweep shape tuned for the throughput line
        if prec == "f32":
            g.set_anchor_shape(*shape64)  # double-precision anchors as tuned on a double grid
        if prec == "f64":
            g.set_launch_shape(*shape64)
        if net:
            g.set_preconditioner(blob)
        st = g.new_state(*(torch.tensor(a, **dev) for a in (case.chi, case.eps, case.B, case.I_bc)))
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(s):
            status, rep = g.solve(st, g.opts(tol=tol_, max_iter=max_iter, use_graph=True, net_every=net,
                                             method=method, os_method=os_method), stream=s)
        s.synchronize()
        wall = time.perf_counter() - t0
        J = g.state_tensors(st)["J"].clone()
        g.close()
        return J, status, rep, wall

    gpu_ref, _, rref, _ = run("f64", 1e-9, 80)
    progress(f"time to solution: GPU double-precision reference {rref.iters} steps")
    target = 1e-5
    import struct
    n_lev = struct.unpack_from("<I", blob, 8)[0]
    out = {"tol": tol, "target_error": target, "f64_launch_shape": list(shape64),
           "network": {"channels": list(struct.unpack_from(f"<{n_lev}I", blob, 12)),
                       "blob": os.path.relpath(blob_path, ROOT)},
           "protocol": "seconds = wall time of rt_solve stopped at max|dJ/J| < tol; seconds_to_target = wall time "
                       "of a fresh rt_solve limited to the fewest steps (iterations) whose J is within the target "
                       "of the reference (binary search over the step limit; error evaluation not timed)"}
    golden = load_golden(case)
    if golden is not None:
        ref = torch.tensor(golden["J"], dtype=torch.float64, device="cuda")[None]
        out["reference"] = (f"oracle fixed point (FP64 CPU, {golden['steps']} steps of non-local Ng-ALI, residual "
                            f"max|Lambda S(J) + Lambda_bc - J|/J {golden['residual']:.1e}), stored in float32")
        out["gpu_fp64_reference_error"] = float(((gpu_ref - ref).abs() / ref.abs()).max())
        out["gpu_fp64_reference"] = f"double-precision Ng-ALI on the GPU, {rref.iters} steps"
    else:
        ref = gpu_ref
        out["reference"] = (f"double-precision Ng-ALI on the GPU, {rref.iters} steps (last max |dJ/J| "
                            f"{rref.max_rel_change:.1e}); unverified: no oracle fixed point of this workload on file")

    def err_of(J):
        return float(((J - ref).abs() / ref.abs()).max())

    gs = "gauss-seidel"
    for name, prec, net, method, tol_m, nl, osm in (
            ("plain_f64_ng_ali", "f64", 0, "ali", tol, False, "jacobi"),
            ("f32_defect_corrected_ng_ali", "f32", 0, "ali", tol, False, "jacobi"),
            ("f32_learned", "f32", net_every, "ali", tol, False, "jacobi"),
            ("f32_nonlocal_ng_ali", "f32", 0, "ali", tol, True, "jacobi"),
            ("f32_nonlocal_gs_ng_ali", "f32", 0, "ali", tol, True, gs),
            ("f64_nonlocal_ng_ali", "f64", 0, "ali", tol, True, "jacobi"),
            ("bicgstab_f64", "f64", 0, "bicgstab", 1e-8, False, "jacobi")):
        J, status, rep, wall = run(prec, tol_m, 300, net, method, nl, osm)
        err = err_of(J)
        progress(f"time to solution: {name} {rep.iters} steps {wall:.2f} s error {err:.2e}")
        out[name] = {"seconds": wall, "steps": rep.iters, "formal_solutions": rep.n_fs, "fp64_fs": rep.n_fs64,
                     "status": status, "max_rel_error": err, "tol": tol_m}
        if nl:
            out[name]["os_sweeps"] = f"16 {osm}"
        if net:
            out[name].update(net_every=net, accepted=rep.n_net_accept, rejected=rep.n_net_reject)
        # fewest steps reaching the target error (errors fall with the step limit)
        lo, hi, best = 1, rep.iters, None
        if err <= target:
            best = (rep.iters, wall, err, rep.n_fs)
            while lo < hi:
                mid = (lo + hi) // 2
                Jm, _, repm, wallm = run(prec, 1e-30, mid, net, method, nl, osm)
                em = err_of(Jm)
                progress(f"time to solution: {name} limited to {mid} steps: error {em:.2e}, {wallm:.2f} s")
                if em <= target:
                    hi = mid
                    best = (mid, wallm, em, repm.n_fs)
                else:
                    lo = mid + 1
        if best:
            out[name].update(steps_to_target=best[0], seconds_to_target=best[1], error_at_target=best[2],
                             formal_solutions_to_target=best[3])
    base = out["plain_f64_ng_ali"]["seconds"]
    out["speedup_f32_vs_plain"] = base / out["f32_defect_corrected_ng_ali"]["seconds"]
    out["speedup_learned_vs_plain"] = base / out["f32_learned"]["seconds"]
    out["speedup_bicgstab_vs_plain"] = base / out["bicgstab_f64"]["seconds"]
    out["speedup_f32_nonlocal_vs_plain"] = base / out["f32_nonlocal_ng_ali"]["seconds"]
    if "seconds_to_target" in out["plain_f64_ng_ali"]:
        b0 = out["plain_f64_ng_ali"]["seconds_to_target"]
        out["speedup_to_target_vs_plain"] = {k: b0 / v["seconds_to_target"] for k, v in out.items()
                                             if isinstance(v, dict) and "seconds_to_target" in v}
    return out


def load_golden(case):
    """The oracle's stored fixed point of this workload (written by
    tests/golden/make_box129_fixed_point.py), if its input fingerprint matches."""
    import numpy as np

    import synthetic as sy
    if not os.path.exists(GOLDEN_129):
        return None
    with np.load(GOLDEN_129, allow_pickle=False) as z:
        if str(z["fingerprint"]) != sy.fingerprint(case):
            return None
        return {"J": z["J"].astype(np.float64), "steps": int(z["steps"]), "residual": float(z["residual"])}


def cpu_baseline_sphere(case, lam: int = 0):
    """The oracle's spherical formal solution, as it stands, on wavelength `lam`
    of the spherical workload: all voxels, a 4 x 8 direction quadrature on all
    host threads and a 2 x 4 one on one thread (its cost grows linearly with
    the directions, so VDU/s carry over to the full 32 x 32 set)."""
    import numpy as np

    import oracle
    import synthetic as sy
    g = oracle.SphereGrid(case.Nr, case.Nt, case.Np, case.r_core, case.r_out)
    S = sy.random_source(case.chi.shape[1:], seed=7, lo=0.2, hi=1.0, dtype="f32").ravel()
    I_out, I_core, J_sub = case.I_bc[lam]
    bv = np.full(case.n_vox, I_core)
    threads = oracle.default_threads()

    def timed(n_mu, n_phi, th):
        t0 = time.perf_counter()
        oracle.fs_sphere(g, n_mu, n_phi, case.chi[lam], S, bv, I_out=I_out, dsrc=case.source_distance,
                         B_sub=J_sub, threads=th)
        wall = time.perf_counter() - t0
        return case.n_vox * n_mu * n_phi / wall, wall

    v, wall = timed(4, 8, threads)
    v1, wall1 = timed(2, 4, 1)
    return {"value": v, "unit": "VDU/s", "cores": threads, "kind": "oracle",
            "sample": f"one FP64 formal solution of wavelength {lam} of {case.n_lambda} over all {case.n_vox} voxels "
                      f"with a 4 x 8 direction quadrature ({wall:.1f} s wall on {threads} threads)",
            "single_core": {"value": v1, "unit": "VDU/s", "cores": 1,
                            "sample": f"2 x 4 directions, all voxels ({wall1:.1f} s wall)"}}


def bench_sphere(args, w):
    """The spherical workload: one ALI step over the wavelength batch per step."""
    import torch

    import paper_2102_01734_amd as rt
    import synthetic as sy
    case = sy.sphere_radial(Nr=w["Nr"], Nt=w["Nt"], Np=w["Np"], n_mu=w["n_mu"], n_phi=w["n_phi"],
                            n_lambda=w["n_lambda"])
    dev = dict(dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    g = rt.SphereGrid(case.Nr, case.Nt, case.Np, case.r_core, case.r_out, case.n_mu, case.n_phi, "f32",
                      case.n_lambda, source_distance=case.source_distance, host_cache=args.host_cache)
    t_build = time.perf_counter() - t0
    progress(f"spherical geometry cache built in {t_build:.1f} s")
    info = g.info()
    st = g.new_state(torch.tensor(case.chi, **dev), torch.tensor(case.eps, **dev), torch.tensor(case.B, **dev),
                     torch.tensor(case.I_bc, **dev))
    opts = g.opts(tol=1e-30, max_iter=1, ng_every=4, ng_start=4)
    for _ in range(args.warmup):
        g.ali_step(st, opts)
    torch.cuda.synchronize()
    rt.rt_profile_read(g.handle)
    rt.rt_profile_enable(g.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.ali_step(st, opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fs_ms, fs_launches, fs_points = rt.rt_profile_read(g.handle)
    rt.rt_profile_enable(g.handle, False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    vdu = case.vdu_per_fs()
    fs_ms_launch = fs_ms / max(fs_launches, 1)
    points_launch = fs_points / max(fs_launches, 1)
    achieved = FLOPS_PER_POINT * points_launch / (fs_ms_launch * 1e-3) / 1e12
    out = {
        "metric": "voxel-direction updates/s (formal solution)", "value": vdu / (ms_per_step * 1e-3),
        "unit": "VDU/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sphere r x theta x phi = {case.Nr}x{case.Nt}x{case.Np}, {case.n_mu}x{case.n_phi} "
                               f"directions, {case.n_lambda} wavelengths, radial tau 1e-6..1e6, point source at 5 r_out; "
                               "step = one ALI iteration over the batch",
                   "voxels": case.n_vox, "directions": case.n_dir, "wavelengths": case.n_lambda,
                   "vdu_per_step": vdu, "visits_per_vdu": info["n_visits"] / (case.n_vox * case.n_dir),
                   "cache_chunks": info["n_workgroups"], "cache_build_s": t_build,
                   "cache_bytes": g.cache_bytes()},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS, "traffic": None,
                     "kernel": "fs_sphere_kernel<float,float,J> + sphere_gather (per chunk)",
                     "kernel_ms_per_launch": fs_ms_launch, "launches": fs_launches,
                     "flops_per_point": FLOPS_PER_POINT, "points_per_launch": points_launch},
    }
    if not args.no_solve:
        out["time_to_solution"] = sphere_time_to_solution(case, g, args.host_cache)
    g.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_sphere(case)
        progress("CPU baseline timed")
    print(json.dumps(out), flush=True)


def sphere_time_to_solution(case, g_diag, host_cache, tol: float = 1e-6):
    """Wall seconds of rt_solve over the whole wavelength batch on the
    spherical workload (all single precision, defect-corrected, Ng every 4
    steps, graph-captured plain steps): the diagonal Lambda*, and the
    nearest-neighbour one with 16 Jacobi or Gauss-Seidel sweeps per step (the
    stencil build inside the timed call); each with its max relative J error
    against the non-local solve iterated to 1e-9 change (the fixed point of
    the float-geometry operator; no FP64 geometry cache is built here)."""
    import torch

    import paper_2102_01734_amd as rt
    dev = dict(dtype=torch.float32, device="cuda")

    def solve(g, tol_, os_method="jacobi"):
        st = g.new_state(*(torch.tensor(a, **dev) for a in (case.chi, case.eps, case.B, case.I_bc)))
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(s):
            status, rep = g.solve(st, g.opts(tol=tol_, max_iter=300, use_graph=not host_cache,
                                             os_method=os_method), stream=s)
        s.synchronize()
        wall = time.perf_counter() - t0
        return g.state_tensors(st)["J"].clone(), status, rep, wall

    out = {"tol": tol, "wavelengths": case.n_lambda}
    legs = {"f32_diagonal_ng_ali": solve(g_diag, tol)}
    progress(f"sphere time to solution: diagonal {legs['f32_diagonal_ng_ali'][2].iters} steps")
    if host_cache:
        out["nonlocal"] = "skipped: the nearest-neighbour Lambda* needs the geometry cache in device memory"
        refJ = None
    else:
        t0 = time.perf_counter()
        gn = rt.SphereGrid(case.Nr, case.Nt, case.Np, case.r_core, case.r_out, case.n_mu, case.n_phi, "f32",
                           case.n_lambda, source_distance=case.source_distance, nonlocal_lstar=True)
        progress(f"sphere time to solution: non-local grid built in {time.perf_counter() - t0:.1f} s")
        refJ, st_ref, rep_ref, wall_ref = solve(gn, 1e-9)
        out["reference"] = (f"FP32 defect-corrected non-local Ng-ALI with Jacobi sweeps to max |dJ/J| < 1e-9, "
                            f"{rep_ref.iters} steps, status {st_ref}")
        legs["f32_nonlocal_jacobi_ng_ali"] = solve(gn, tol, "jacobi")
        legs["f32_nonlocal_gs_ng_ali"] = solve(gn, tol, "gauss-seidel")
        gn.close()
    for name, (J, status, rep, wall) in legs.items():
        out[name] = {"seconds": wall, "steps": rep.iters, "formal_solutions": rep.n_fs, "fp64_fs": rep.n_fs64,
                     "status": status}
        if refJ is not None:
            out[name]["max_rel_error"] = float(((J.double() - refJ.double()).abs() / refJ.double().abs()).max())
        progress(f"sphere time to solution: {name} {rep.iters} steps {wall:.2f} s")
    if "f32_nonlocal_jacobi_ng_ali" in out:
        base = out["f32_diagonal_ng_ali"]["seconds"]
        out["speedup_nonlocal_jacobi"] = base / out["f32_nonlocal_jacobi_ng_ali"]["seconds"]
        out["speedup_nonlocal_gs"] = base / out["f32_nonlocal_gs_ng_ali"]["seconds"]
    return out


def box_line(case, name: str, steps: int, warmup: int, shape_arg=None, autotune=True):
    """Throughput of ALI steps on a box workload, replayed as captured HIP
    graphs on one stream, with the sweep's launch time from event nodes in
    the graph.  Returns (result dict, tuned shape)."""
    import torch

    import paper_2102_01734_amd as rt
    import synthetic as sy
    dev = dict(dtype=torch.float32, device="cuda")
    chi = torch.tensor(case.chi, **dev)
    eps = torch.tensor(case.eps, **dev)
    B = torch.tensor(case.B, **dev)
    Ibc = torch.tensor(case.I_bc, **dev)
    g = rt.Grid(case.Nx, case.Ny, case.Nz, case.n_mu, case.n_phi, "f32", case.n_lambda)
    # launch-shape autotuning (setup, not timed): on up to 8 wavelengths spread
    # over the batch, so that a batch is tuned on its own mix of optical depths
    if shape_arg:
        g.set_launch_shape(*shape_arg)
    elif autotune:
        pick = sorted(set(round(x) for x in torch.linspace(0, case.n_lambda - 1, min(8, case.n_lambda)).tolist()))
        S0 = torch.tensor(sy.random_source((len(pick),) + case.chi.shape[1:], seed=7, lo=0.2, hi=1.0, dtype="f32"),
                          **dev)
        g.autotune(chi[pick].contiguous(), S0)
        del S0
    ls = g.launch_shape()
    shape = (ls["threads"], ls["rays"], bool(ls["band"]))
    progress(f"{name}: launch shape {shape}, {ls['bundles']} bundles")
    info = g.info()
    st = g.new_state(chi, eps, B, Ibc)
    opts = g.opts(tol=1e-30, max_iter=1, ng_every=4, ng_start=4, use_graph=True)
    s = torch.cuda.Stream()
    rt.rt_profile_enable(g.handle, True)  # before the warm-up: the profiled graph is captured there
    with torch.cuda.stream(s):
        for _ in range(warmup):
            g.ali_step(st, opts, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    rt.rt_profile_read(g.handle)
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        for _ in range(steps):
            g.ali_step(st, opts, stream=s)
    s.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fs_ms, fs_launches, fs_points = rt.rt_profile_read(g.handle)
    rt.rt_profile_enable(g.handle, False)
    rel = g.state_tensors(st)["rel_change"].cpu().numpy()
    g.close()
    del st
    torch.cuda.synchronize()

    ms_per_step = (t1 - t0) * 1e3 / steps
    vdu = case.vdu_per_fs()
    fs_ms_launch = fs_ms / max(fs_launches, 1)
    points_launch = fs_points / max(fs_launches, 1)
    achieved = FLOPS_PER_POINT * points_launch / (fs_ms_launch * 1e-3) / 1e12
    hbm = BYTES_PER_VDU * vdu / (fs_ms_launch * 1e-3) / 1e9
    traffic = read_traffic(name, ls)
    progress(f"{name}: {steps} timed steps, {ms_per_step:.1f} ms per step, sweep {fs_ms_launch:.1f} ms")
    if case.n_lambda == 1:
        wl = (f"box {case.Nx}^3 periodic x,y, {case.n_mu}x{case.n_phi} directions, stratified opacity (tau 1e-4..1e4) "
              "x log-normal perturbation (1 dex, l=8), eps 1e-6..1 per voxel; step = one ALI iteration (FP32 formal "
              "solution + reduction + FP64 update + norm, Ng every 4), HIP-graph replay")
    else:
        wl = (f"box {case.Nx}^3 periodic x,y, {case.n_mu}x{case.n_phi} directions, {case.n_lambda} wavelengths "
              "(opacity scale 10^U(-3,3), eps 10^U(-5,-1) per wavelength) in one persistent launch per step; step = "
              "one ALI iteration over the batch (FP32 formal solution, FP64 update, Ng and norms), HIP-graph replay")
    out = {
        "metric": "voxel-direction updates/s (formal solution)", "value": vdu / (ms_per_step * 1e-3),
        "unit": "VDU/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl, "name": name, "voxels": case.n_vox, "directions": case.n_dir,
                   "wavelengths": case.n_lambda, "vdu_per_step": vdu,
                   "visits_per_vdu": points_launch / vdu, "workgroups": info["n_workgroups"],
                   "launch_shape": {"threads": ls["threads"], "rays_per_thread": ls["rays"],
                                    "bundles": ls["bundles"], "tiles": "band" if ls["band"] else "layer"}},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS, "traffic": traffic,
                     "hbm": {"achieved": hbm, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": hbm / PEAK_HBM_GBS,
                             "bytes_per_vdu": BYTES_PER_VDU},
                     "kernel": "fs_box_kernel<float,J>", "kernel_ms_per_launch": fs_ms_launch,
                     "launches": fs_launches, "flops_per_point": FLOPS_PER_POINT,
                     "points_per_launch": points_launch, "vdu_per_launch": vdu},
        "last_rel_change": float(rel.max()),
    }
    return out, shape


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched129", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-solution comparison")
    ap.add_argument("--net", default=None, help="network blob for the learned leg (default: the shipped one)")
    ap.add_argument("--no-extra", action="store_true",
                    help="batched workload: skip the single-wavelength line, the one-GPU share and time to solution")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--shape", default=None, help="fix the launch shape THREADS,RAYS[,BAND] (BAND 1: row-band tiles) instead of autotuning")
    ap.add_argument("--host-cache", action="store_true",
                    help="sphere workload: keep the geometry cache in host memory and stream it (SmallGPU mode)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU; --gpus must be 1 (the solid-angle sharding across "
              "GPUs is not implemented; one GPU's share is measured as one_gpu_share)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = 1 << 28
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": 4 * n, "bytes_written": 4 * n,
                          "launches": 3}), flush=True)
        return

    import synthetic as sy

    w = WORKLOADS[args.workload]
    if "Nr" in w:
        return bench_sphere(args, w)

    def make(wname):
        ww = WORKLOADS[wname]
        if "n_lambda" in ww:
            return sy.box_batched(N=ww["N"], n_lambda=ww["n_lambda"], n_mu=ww["n_mu"], n_phi=ww["n_phi"])
        return sy.box_lognormal(N=ww["N"], n_mu=ww["n_mu"], n_phi=ww["n_phi"], field_seed=ww.get("field_seed", 1),
                                eps_seed=ww.get("eps_seed", 101))

    case = make(args.workload)
    progress(f"workload {args.workload} generated")
    shape_arg = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
    out, shape = box_line(case, args.workload, args.steps, args.warmup, shape_arg, not args.no_autotune)

    # the single-wavelength 129^3 x 2048 line and what runs on it
    single = case if case.n_lambda == 1 else None
    if case.n_lambda > 1 and not args.no_extra:
        single = make("lognormal129")
        line1, shape1 = box_line(single, "lognormal129", 10, 3, None, not args.no_autotune)
        out["lognormal129"] = {k: line1[k] for k in ("value", "unit", "ms_per_step", "config", "roofline")}
    else:
        shape1 = shape
    if single is not None and not (case.n_lambda > 1 and args.no_extra):
        out["one_gpu_share"] = one_gpu_share(single, shape1)
        progress("one-GPU share timed")
        if not args.no_solve:
            out["time_to_solution"] = time_to_solution(single, shape=shape1, net_path=args.net)
    if not args.no_cpu_baseline:
        # about 4e8 voxel-directions on all threads, 3.4e7 on one
        n_sub = max(8, min(case.n_dir, round(4.1e8 / case.n_vox)))
        n_sub_1 = max(2, min(case.n_dir, round(3.4e7 / case.n_vox)))
        out["cpu_baseline"] = cpu_baseline(case, n_sub, n_sub_1)
        progress("CPU baseline timed")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
