#!/usr/bin/env python3
"""Benchmark: DOF-CG-iterations/s of the effective-stiffness solve at 256^3.

Workload (synthetic): 3D 256^3 voxels, two-phase microstructure from a
seeded Gaussian random field (correlation length 8 voxels, seed 3)
thresholded at 0, E 1 : 1000, nu 0.25 / 0.35, all 6 unit macro strains
solved together, mixed precision (FP32 stencil/FFT/vector updates, FP64
reductions and reliable-update residuals), tol 1e-6 on ||r||/||f||.

One step = one cell_effective_stiffness call (load vectors, PCG for the 6
loads, FP64 residual refreshes, homogenisation).  value = sum over steps and
loads of 3 n iterations / wall time.  The inputs are resident on the GPU
before timing starts.

Besides the headline line it reports (same JSON object):
  * roofline: the kernel with the largest share of GPU time, its algorithmic
    bytes per launch (the byte model of the design notes) divided by its
    average launch time (HIP events on the library's stream, timed region);
  * fp64: the same solve in FP64 to tol 1e-6 (time to solution, speed-up of
    mixed over FP64) and the normwise C* error of both against an FP64
    solve at tol 1e-10;
  * cpu_baseline: the CPU oracle (numpy/scipy FP64) timed on this host on a
    bounded sample: 6 PCG iterations on one load of a 128^3 periodic
    sub-block of the same field.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def byte_model(kind, n, prec_bytes):
    """Algorithmic HBM bytes per load per launch of each kernel kind (3D).

    A real field is 3 n values, its packed half spectrum the same size.
    """
    f = 3 * n * prec_bytes
    return {
        "k_apply": 2 * f,      # read p, write q (+ material once per launch)
        "x_fwd": 3 * f,        # read q and the x-transformed residual R; write R
        "y_fwd": 2 * f,        # read R, write the spectrum
        "last": 2 * f,         # read/write spectrum
        "y_inv": 2 * f,
        "x_inv": 5 * f,        # read spectrum, p, x; write x, p
    }[kind]


def source_sha256():
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2004_05197_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kind, workload):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE) recorded in
    profiles/traffic_<workload>.json, or None if absent or taken on other
    kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != source_sha256() or kind not in t.get("kernels", {}):
        return None
    k = t["kernels"][kind]
    return round(k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"])


def cpu_baseline(E, nu, sub=128, iters=6):
    from oracle import fem, matfree
    Es = np.ascontiguousarray(E[:sub, :sub, :sub])
    nus = np.ascontiguousarray(nu[:sub, :sub, :sub])
    g = fem.Grid((sub, sub, sub))
    pre = matfree.FourierPreconditioner(g, *matfree.reference_medium(Es, nus, 3))
    t0 = time.perf_counter()
    matfree.pcg(g, Es, nus, np.eye(6)[0], tol=1e-30, maxit=iters, precond=pre)
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    return {
        "value": 3 * g.n * iters / dt,
        "unit": "DOF-CG-iterations/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{iters} PCG iterations (FP64 numpy matrix-free K-apply, single thread; "
                  f"scipy.fft preconditioner on {cores} workers) on load eps_11 of a {sub}^3 "
                  f"periodic sub-block of the {E.shape[0]}^3 field, preconditioner setup excluded, "
                  f"{dt:.1f} s",
    }


def bench_uneven(args, B, ms, progress):
    """The uneven batch: args.cells sphere cells (seeds 1000..), sizes from
    {32,48,64,96}, 6 unit loads each, one batched mixed-precision solve."""
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    cells = list(ms.random_cells(args.cells, workers=workers))
    progress(f"generated {len(cells)} cells in {time.perf_counter() - t0:.1f} s")
    import torch
    b = B.Batch([(c["n"],) * 3 for c in cells], precision=B.MIXED, tol=1e-6)
    for i, c in enumerate(cells):
        b.set_material(i, c["E"].ravel(), c["nu"].ravel())
    if not args.no_tune:
        t_tune = time.perf_counter()
        b.autotune()
        progress(f"autotune of {b.groups} groups in {time.perf_counter() - t_tune:.2f} s")
    for i in range(args.warmup):
        C, infos = b.effective_stiffness()
        progress(f"warmup {i}: {infos[0]['seconds']:.2f} s")
    b.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = np.zeros(len(cells))
    for i in range(args.steps):
        C, infos = b.effective_stiffness()
        iters += [sum(inf["iters"]) for inf in infos]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = b.profile_read()
    b.profile(False)
    b.close()
    nvox = np.array([c["n"] ** 3 for c in cells], dtype=np.float64)
    value = float((3 * nvox * iters).sum() / dt)
    kinds = ["k_apply", "x_fwd", "y_fwd", "last", "y_inv", "x_inv"]
    dom = max(kinds, key=lambda k: prof[k][0])
    ms_tot, launches = prof[dom]
    # per slot: one launch per iteration (+ the initial preconditioning for
    # the FFT passes); material bytes of the K-apply not counted
    extra = 0 if dom == "k_apply" else 6 * args.steps
    alg_bytes = float(((iters + extra) * np.array([byte_model(dom, n, 4) for n in nvox])).sum())
    achieved = alg_bytes / (ms_tot * 1e-3) / 1e9
    progress(f"timed {args.steps} steps in {dt:.3f} s")
    return {
        "metric": "DOF-CG-iterations/sec, uneven batch (mixed, tol 1e-6)",
        "value": value,
        "unit": "DOF-CG-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"uneven{len(cells)}: {len(cells)} RSA sphere cells (seeds 1000+k), sizes from "
                        "{32,48,64,96}^3, vf 0.1-0.4, contrast 10-100, nu 0.3, 6 unit loads each, one "
                        "batched mixed-precision solve, tol 1e-6",
            "cells": len(cells),
            "voxels": int(nvox.sum()),
            "groups": {str(n): int((nvox == n ** 3).sum()) for n in (32, 48, 64, 96)},
        },
        "roofline": {
            "bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_launch_ms": round(ms_tot / launches, 4), "launches": launches,
        },
        "kernel_ms": {k: round(v[0], 2) for k, v in prof.items()},
        "cpu_baseline": None,
    }


# Algorithmic floating-point operations of one tangent product K_T(u) p per
# voxel (3D): the six Kuhn simplices, each evaluated once (the per-simplex
# count of the design notes: F and grad p 45, inverse and det 42, ln J 1,
# (F^-1 dG) and (F^-1 dG F^-1) 92, coefficients 3, dP 45, nodal forces 48)
HYPER_FLOPS_PER_SIMPLEX = 276
HYPER_FLOPS_PER_VOXEL = 6 * HYPER_FLOPS_PER_SIMPLEX
# vector FP32 FMA rate without packed FP32: 256 CUs x 64 lanes x 2 flops
# x 2.4 GHz (the published 157.3 TFLOP/s counts packed FP32 issue)
ALU_F32_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12


def hyper_loads(d=3, amp=0.05):
    """Six macroscopic gradients: uniaxial stretches 1 + amp along x, y, z
    and simple shears amp in the yz, xz and xy planes."""
    F = np.tile(np.eye(d), (6, 1, 1))
    for a in range(3):
        F[a, a, a] += amp
    for J, (a, b) in enumerate([(1, 2), (0, 2), (0, 1)]):
        F[3 + J, a, b] = amp
    return F


def cpu_baseline_hyper(E, nu, Fb, sub=18):
    from oracle import fem, hyper
    Es = np.ascontiguousarray(E[:sub, :sub, :sub])
    nus = np.ascontiguousarray(nu[:sub, :sub, :sub])
    g = fem.Grid((sub, sub, sub))
    t0 = time.perf_counter()
    out = hyper.newton(g, Es, nus, Fb, tol=1e-30, maxit=1)
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0))
    return {
        "value": 3 * g.n * out["iterations"] / dt,
        "unit": "DOF-Newton-iterations/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"1 Newton iteration (explicit sparse tangent assembly, sparse direct solve, energy line "
                  f"search; numpy/scipy FP64) for the stretch load on a {sub}^3 periodic sub-block of the "
                  f"{E.shape[0]}^3 field, {dt:.1f} s",
    }


def bench_hyper(args, B, ms, progress):
    """Neo-Hookean Newton-PCG: the grf3d geometry with phase contrast
    args.contrast (default 1:10; at 1:1000 the tangent turns indefinite under
    these loads and the Newton safeguards dominate), six 5 % stretch/shear
    loads batched, mixed precision inner solves (tol 1e-6), Newton tolerance
    1e-8 of the load scale."""
    import torch
    n1 = args.n
    n = n1 ** 3
    E, nu = ms.two_phase_grf(n1, seed=3, E_hard=args.contrast)
    Fb = hyper_loads()
    cell = B.Cell((n1, n1, n1), precision=B.MIXED, tol=1e-6)
    cell.set_material(torch.from_numpy(E.ravel()).cuda(), torch.from_numpy(nu.ravel()).cuda())
    sched = cell.schedule
    if not args.no_tune:
        sched = cell.autotune()
        progress(f"autotune: schedule {sched}")
    for i in range(args.warmup):
        P, info = cell.solve_hyper(Fb, tol=1e-8)
        progress(f"warmup {i}: newton {info['newton_iters']} cg {info['cg_iters']} {info['seconds']:.2f} s")
    cell.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cg_total, newton_total = 0, 0
    for i in range(args.steps):
        P, info = cell.solve_hyper(Fb, tol=1e-8)
        cg_total += sum(info["cg_iters"])
        newton_total += sum(info["newton_iters"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = cell.profile_read()
    cell.profile(False)
    cell.close()
    progress(f"timed {args.steps} steps in {dt:.3f} s: newton {info['newton_iters']} cg {info['cg_iters']} "
             f"status {info['status']}")
    kinds = ["k_apply", "x_fwd", "y_fwd", "last", "y_inv", "x_inv", "residual"]
    dom = max(kinds, key=lambda k: prof[k][0])
    ms_k, launches_k = prof["k_apply"]
    flops = cg_total * n * HYPER_FLOPS_PER_VOXEL
    achieved = flops / (ms_k * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu:
        progress("cpu oracle baseline ...")
        cpu = cpu_baseline_hyper(E, nu, Fb[0])
    return {
        "metric": "DOF-CG-iterations/sec of the neo-Hookean Newton-PCG at 256^3 (mixed inner solves)",
        "value": 3 * n * cg_total / dt,
        "unit": "DOF-CG-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"hyper_grf3d_{n1}: {n1}^3 voxels, the thresholded Gaussian random field of the "
                        f"linear workload with E 1:{args.contrast:g} (nu 0.25/0.35), compressible neo-Hookean, six loads "
                        "(stretches 1.05 along x, y, z; shears 0.05 in yz, xz, xy) in one batched Newton "
                        "solve, inner PCG mixed precision tol 1e-6, Newton tol 1e-8",
            "voxels": n,
            "loads": 6,
            "contrast": args.contrast,
            "newton_iters": info["newton_iters"],
            "indefinite_steps": info["indefinite_steps"],
            "cg_iters": info["cg_iters"],
            "schedule": list(sched),
        },
        "dof_newton_iter_per_s": 3 * n * newton_total / dt,
        "roofline": {
            "bound": "alu", "kernel": "k_apply (neo-Hookean tangent)", "achieved": round(achieved, 2),
            "peak": round(ALU_F32_PEAK_TFLOPS, 1), "unit": "TFLOP/s", "frac": round(achieved / ALU_F32_PEAK_TFLOPS, 4),
            "traffic": measured_traffic("k_apply", f"hyper_grf3d_{n1}"), "avg_launch_ms": round(ms_k / launches_k, 4),
            "launches": launches_k, "flops_per_voxel": HYPER_FLOPS_PER_VOXEL, "dominant_kernel": dom,
        },
        "kernel_ms": {k: round(v[0], 2) for k, v in prof.items()},
        "gpu_busy_frac": round(sum(v[0] for v in prof.values()) * 1e-3 / dt, 4),
        "cpu_baseline": cpu,
    }


def cpu_baseline_surrogate(E, nu, M, sub=16):
    from oracle import fem, surrogate as sg
    sub = M * max(1, sub // M)  # the sampling step divides the sub-block
    Es = np.ascontiguousarray(E[:sub, :sub, :sub])
    nus = np.ascontiguousarray(nu[:sub, :sub, :sub])
    g = fem.Grid((sub, sub, sub))
    t0 = time.perf_counter()
    sg.effective_stiffness(g, Es, nus, M, 3)
    dt = time.perf_counter() - t0
    return {
        "value": 6 * 3 * g.n / dt,
        "unit": "DOF-solves/s",
        "cores": len(os.sched_getaffinity(0)),
        "kind": "oracle",
        "sample": f"surrogate stencils (M {M}, cubic), surrogate matrix and bordered direct solve of the six unit "
                  f"loads (numpy/scipy FP64, SuperLU) on a {sub}^3 periodic sub-block of the {E.shape[0]}^3 field, "
                  f"{dt:.1f} s",
    }


def cpu_baseline_adjoint(E, nu, sub=18):
    from oracle import fem
    Es = np.ascontiguousarray(E[:sub, :sub, :sub])
    nus = np.ascontiguousarray(nu[:sub, :sub, :sub])
    g = fem.Grid((sub, sub, sub))
    t0 = time.perf_counter()
    _, _, u = fem.effective_stiffness(g, Es, nus)
    fem.dC_dE(g, Es, nus, u, fem.unit_loads(3))
    dt = time.perf_counter() - t0
    return {
        "value": 6 * 3 * g.n / dt,
        "unit": "DOF-solves/s",
        "cores": len(os.sched_getaffinity(0)),
        "kind": "oracle",
        "sample": f"direct solve of the six unit loads and dC*/dE over all voxels (numpy/scipy FP64, SuperLU) "
                  f"on a {sub}^3 periodic sub-block of the {E.shape[0]}^3 field, {dt:.1f} s",
    }


def bench_surrogate(args, B, ms, progress):
    """Surrogate stencil operator: log-normal E (sigma 1, correlation length
    args.ell voxels) at args.n^3, nu 0.3, the six unit loads, mixed precision
    tol 1e-6; C* of the surrogate solutions (sampling step args.M, cubic
    B-splines) against the exact matrix-free path on the same field."""
    import torch
    n1 = args.n
    n = n1 ** 3
    E, nu = ms.lognormal_field(n1, 7, ell=args.ell, sigma=1.0)
    cell = B.Cell((n1, n1, n1), precision=B.MIXED, tol=1e-6)
    cell.set_material(torch.from_numpy(E.ravel()).cuda(), torch.from_numpy(nu.ravel()).cuda())
    if not args.no_tune:
        cell.autotune()
    C_exact, info_exact = cell.effective_stiffness()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C_exact, info_exact = cell.effective_stiffness()
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - t0
    setup = cell.set_surrogate(args.M, 3)
    progress(f"exact {t_exact:.3f} s iters {info_exact['iters']}; surrogate setup {setup:.2f} s")
    for i in range(args.warmup):
        cell.effective_stiffness()
    cell.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for i in range(args.steps):
        C_sr, info = cell.effective_stiffness()
        iters += sum(info["iters"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = cell.profile_read()
    cell.profile(False)
    cell.close()
    ms_k, launches = prof["k_apply"]
    # algorithmic bytes per launch with 6 active loads: the stencil (63 FP32
    # values per node) once, p read and q written per load
    alg = 63 * 4 * n + 6 * 24 * n
    achieved = alg / (ms_k / launches * 1e-3) / 1e9
    err = float(np.abs(C_sr - C_exact).max() / np.abs(C_exact).max())
    progress(f"timed {args.steps} steps in {dt:.3f} s, iters {info['iters']}, C error {err:.3e}")
    return {
        "metric": "DOF-CG-iterations/sec of the surrogate-stencil solve at 256^3 (mixed, tol 1e-6)",
        "value": 3 * n * iters / dt,
        "unit": "DOF-CG-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"surrogate_lognormal_{n1}: {n1}^3 voxels, log-normal E (sigma 1, correlation length "
                        f"{args.ell:g} voxels, seed 7), nu 0.3, six unit loads, surrogate stencil functions "
                        f"sampled every {args.M} nodes with cubic B-splines, mixed precision tol 1e-6",
            "voxels": n, "M": args.M, "q": 3, "iters": info["iters"],
            "exact_iters": info_exact["iters"],
        },
        "dof_solves_per_s": 6 * 3 * n / (dt / args.steps),
        "surrogate_setup_s": round(setup, 3),
        "exact_time_to_solution_s": round(t_exact, 4),
        "surrogate_time_to_solution_s": round(dt / args.steps, 4),
        "C_rel_err_surrogate_vs_exact": err,
        "roofline": {
            "bound": "hbm", "kernel": "k_apply (surrogate stencil)", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "avg_launch_ms": round(ms_k / launches, 4), "launches": launches, "bytes_per_launch": alg,
        },
        "kernel_ms": {k: round(v[0], 2) for k, v in prof.items()},
        "cpu_baseline": None if args.no_cpu else cpu_baseline_surrogate(E, nu, args.M),
    }


def bench_adjoint(args, B, ms, progress):
    """Adjoint gradient: 128^3 log-normal E (correlation length 6 voxels,
    sigma 1, seed 5), nu 0.3, J = C*_1111 + C*_2323; one step = the six
    unit-load solve (FP64, tol 1e-10) plus dJ/dE over all voxels."""
    import torch
    n1 = args.n if args.n != 256 else 128
    n = n1 ** 3
    E, nu = ms.lognormal_field(n1, seed=5)
    cell = B.Cell((n1, n1, n1), precision=B.FP64, tol=1e-10)
    cell.set_material(torch.from_numpy(E.ravel()).cuda(), torch.from_numpy(nu.ravel()).cuda())
    dJ = np.zeros((6, 6))
    dJ[0, 0] = dJ[3, 3] = 1.0
    g = torch.empty(n, dtype=torch.float64, device="cuda")
    if not args.no_tune:
        cell.autotune()
    for i in range(args.warmup):
        cell.effective_stiffness()
        cell.adjoint(dJ, out=g)
    torch.cuda.synchronize()
    t_solve = t_grad = 0.0
    iters = 0
    for i in range(args.steps):
        t0 = time.perf_counter()
        C, info = cell.effective_stiffness()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cell.adjoint(dJ, out=g)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_solve += t1 - t0
        t_grad += t2 - t1
        iters += sum(info["iters"])
    cell.close()
    gh = g.cpu().numpy()
    J = C[0, 0] + C[3, 3]
    euler = abs(float(np.dot(gh, E.ravel())) - J) / J
    progress(f"{args.steps} steps: solve {t_solve:.3f} s, gradient {t_grad * 1e3:.2f} ms, Euler gap {euler:.2e}")
    dt = t_solve + t_grad
    return {
        "metric": "DOF-CG-iterations/sec of the 128^3 FP64 solve with the adjoint gradient",
        "value": 3 * n * iters / dt,
        "unit": "DOF-CG-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": f"adjoint_lognormal_{n1}: {n1}^3 voxels, log-normal E (correlation length 6 voxels, "
                        "sigma 1, seed 5), nu 0.3, six unit loads in FP64 to tol 1e-10, J = C*_1111 + C*_2323, "
                        "dJ/dE over every voxel",
            "voxels": n, "iters": info["iters"],
        },
        "gradient_ms": round(t_grad / args.steps * 1e3, 3),
        "solve_ms": round(t_solve / args.steps * 1e3, 3),
        "euler_identity_gap": euler,
        "dof_solves_per_s": 6 * 3 * n / (dt / args.steps),
        "cpu_baseline": None if args.no_cpu else cpu_baseline_adjoint(E, nu),
    }


def copy_bandwidth(torch, mib=1024, reps=5):
    """Device-to-device copy rate (GB/s of read + write traffic) of a plain
    torch copy of `mib` MiB, best of `reps`: the practically reachable HBM
    rate that the roofline fraction can be compared with."""
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps + 1):
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2 * mib * (1 << 20) / (best * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="keep the default kernel schedule")
    ap.add_argument("--schedule", default=None,
                    help="six comma-separated ints: use this kernel schedule instead of tuning")
    ap.add_argument("--workload", default="grf3d", choices=["grf3d", "uneven", "hyper", "surrogate", "adjoint"],
                    help="grf3d: the 256^3 headline workload; uneven: the batch of sphere cells; "
                         "hyper: the neo-Hookean Newton-PCG on the grf3d geometry")
    ap.add_argument("--cells", type=int, default=512, help="cells of the uneven batch")
    ap.add_argument("--contrast", type=float, default=10.0, help="phase contrast of the hyper workload")
    ap.add_argument("--M", type=int, default=4, help="sampling step of the surrogate workload")
    ap.add_argument("--ell", type=float, default=32.0, help="correlation length of the surrogate workload")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the cell solve runs on one GPU (it is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2004_05197_amd import binding as B
    from paper_2004_05197_amd import microstructures as ms

    torch.cuda.set_device(0)

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.copy_probe:
        a = torch.empty(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.workload == "uneven":
        print(json.dumps(bench_uneven(args, B, ms, progress)), flush=True)
        return
    if args.workload == "hyper":
        print(json.dumps(bench_hyper(args, B, ms, progress)), flush=True)
        return
    if args.workload == "surrogate":
        print(json.dumps(bench_surrogate(args, B, ms, progress)), flush=True)
        return
    if args.workload == "adjoint":
        print(json.dumps(bench_adjoint(args, B, ms, progress)), flush=True)
        return
    n1 = args.n
    n = n1 ** 3
    E, nu = ms.two_phase_grf(n1, seed=3)
    Ed = torch.from_numpy(E.ravel()).cuda()
    nud = torch.from_numpy(nu.ravel()).cuda()
    torch.cuda.synchronize()


    # ---------------------------------------------------------------- mixed
    cell = B.Cell((n1, n1, n1), precision=B.MIXED, tol=1e-6)
    cell.set_material(Ed, nud)
    if args.schedule:
        cell.schedule = tuple(int(v) for v in args.schedule.split(","))
    sched = cell.schedule
    if not args.no_tune and not args.schedule:
        t_tune = time.perf_counter()
        sched = cell.autotune()
        progress(f"autotune: schedule {sched} in {time.perf_counter() - t_tune:.2f} s")
    for i in range(args.warmup):
        C_mixed, info = cell.effective_stiffness()
        progress(f"warmup {i}: iters {info['iters']} {info['seconds']:.2f} s")
    cell.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters_total = 0
    per_step = []
    for i in range(args.steps):
        C_mixed, info = cell.effective_stiffness()
        iters_total += sum(info["iters"])
        per_step.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = cell.profile_read()
    cell.profile(False)
    dt = t1 - t0
    progress(f"timed {args.steps} steps in {dt:.3f} s, iters {per_step[-1]['iters']}, "
             f"refinements {per_step[-1]['refinements']}")
    dof_iter = 3 * n * iters_total
    value = dof_iter / dt
    mixed_tts = dt / args.steps
    cell.close()
    del cell

    # roofline of the dominant kernel (largest GPU time in the timed region)
    kinds = ["k_apply", "x_fwd", "y_fwd", "last", "y_inv", "x_inv"]
    dom = max(kinds, key=lambda k: prof[k][0])
    ms_tot, launches = prof[dom]
    load_launches = iters_total + (0 if dom == "k_apply" else 6 * args.steps)
    alg_bytes = load_launches * byte_model(dom, n, 4)
    if dom == "k_apply":
        alg_bytes += launches * 8 * n
    achieved = alg_bytes / (ms_tot * 1e-3) / 1e9
    gpu_ms = sum(prof[k][0] for k in prof)
    copy_gbs = copy_bandwidth(torch)
    roofline = {
        "bound": "hbm",
        "kernel": dom,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(dom, f"grf3d_{n1}"),
        "avg_launch_ms": round(ms_tot / launches, 4),
        "launches": launches,
        "bytes_per_launch": round(alg_bytes / launches),
        "copy_gbs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
    }
    # whole-iteration byte model: all six kernels
    all_bytes = sum((iters_total + (0 if k == "k_apply" else 6 * args.steps)) * byte_model(k, n, 4)
                    for k in kinds) + prof["k_apply"][1] * 8 * n
    loop_ms = sum(prof[k][0] for k in kinds)
    kernel_ms = {k: round(v[0], 2) for k, v in prof.items()}

    # ---------------------------------------------------------------- fp64
    fp64 = None
    if not args.no_fp64:
        with B.Cell((n1, n1, n1), precision=B.FP64, tol=1e-10) as c64:
            c64.set_material(Ed, nud)
            C_ref, info_ref = c64.effective_stiffness()
            progress(f"fp64 tol 1e-10: iters {info_ref['iters']} {info_ref['seconds']:.2f} s")
        with B.Cell((n1, n1, n1), precision=B.FP64, tol=1e-6) as c64:
            c64.set_material(Ed, nud)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            C_64, info_64 = c64.effective_stiffness()
            torch.cuda.synchronize()
            fp64_tts = time.perf_counter() - t2
            progress(f"fp64 tol 1e-6: iters {info_64['iters']} {fp64_tts:.2f} s")
        err = lambda C: float(np.abs(C - C_ref).max() / np.abs(C_ref).max())
        fp64 = {
            "time_to_solution_s": round(fp64_tts, 4),
            "iters": info_64["iters"],
            "dof_cg_iter_per_s": 3 * n * sum(info_64["iters"]) / fp64_tts,
            "mixed_time_to_solution_s": round(mixed_tts, 4),
            "speedup_mixed_over_fp64": round(fp64_tts / mixed_tts, 3),
            "C_err_mixed_vs_fp64_tol1e-10": err(C_mixed),
            "C_err_fp64_tol1e-6_vs_fp64_tol1e-10": err(C_64),
        }

    cpu = None
    if not args.no_cpu:
        progress("cpu oracle baseline ...")
        cpu = cpu_baseline(E, nu)

    out = {
        "metric": "DOF-CG-iterations/sec at 256^3 (mixed vs FP64, rel err <=1e-6); % HBM roofline",
        "value": value,
        "unit": "DOF-CG-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"grf3d_{n1}: {n1}^3 voxels, thresholded Gaussian random field (ell 8, seed 3), "
                        "E 1:1000, nu 0.25/0.35, 6 unit loads batched, mixed precision (FP32 bulk, "
                        "FP64 reductions and residual refreshes), tol 1e-6",
            "voxels": n,
            "loads": 6,
            "iters_per_step": per_step[-1]["iters"],
            "refinements_per_step": per_step[-1]["refinements"],
            "schedule": list(sched),
        },
        "roofline": roofline,
        "iteration_byte_model_frac": round(all_bytes / (loop_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "iteration_byte_model_frac_of_copy": round(all_bytes / (loop_ms * 1e-3) / 1e9 / copy_gbs, 4),
        "kernel_ms": kernel_ms,
        "gpu_busy_frac": round(gpu_ms * 1e-3 / dt, 4),
        "fp64": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
