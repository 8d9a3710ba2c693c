#!/usr/bin/env python3
"""Benchmark: DOF-CG-iterations/s of the effective-stiffness solve at 256^3.

Workload (synthetic): 3D 256^3 voxels, two-phase microstructure from a
seeded Gaussian random field (correlation length 8 voxels, seed 3)
thresholded at 0, E 1 : 1000, nu 0.25 / 0.35, all 6 unit macro strains
solved together, mixed precision (FP32 stencil/FFT/vector updates, FP64
reductions and reliable-update residuals), tol 1e-6 on ||r||/||f||.

One step = one cell_effective_stiffness call (load vectors, PCG for the 6
loads, FP64 residual refreshes, homogenisation), run as in production: the
kernel schedule pinned (HEADLINE_SCHEDULE; --tune runs the autotuner), the
PCG chunks replayed from captured HIP graphs, no per-kernel events.  value
= 3 n x (iterations of the six loads) / median wall time of the timed steps
(steps are deterministic: every step runs the same iterations).  The inputs
are resident on the GPU before timing starts.

Besides the headline line it reports (same JSON object):
  * roofline: the kernel with the largest share of GPU time, its algorithmic
    bytes per launch (the byte model of the design notes) divided by its
    average launch time, from HIP events around every launch of one more
    step run with eager launches after the timed ones; traffic from the
    committed counter summary of the same kernels and schedule;
  * iteration: the bytes of a whole step over its median wall time, as a
    fraction of 8 TB/s (this schedule's bytes and the 72 B per
    DOF-iteration of the textbook fused schedule);
  * fp64: the same solve in FP64 to tol 1e-6 (median time to solution under
    the same protocol, speed-up of mixed over FP64) and the normwise C*
    error of both against an FP64 solve at tol 1e-10;
  * cpu_baseline: the CPU oracle (numpy/scipy FP64) timed on this host on a
    bounded sample: 6 PCG iterations on one load of a 128^3 periodic
    sub-block of the same field; with --cpu-full also 3 iterations at the
    full size and the time to solution extrapolated from them.

`--workload` selects the other measured workloads (uneven batch, neo-Hookean,
surrogate operator, adjoint gradient, the 64^3 sphere cell);
`summarize-stats` / `summarize-traffic` write the profiles/ summaries from
rocprofv3 CSV output of this script.
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


def measured_traffic(kind, workload, sched=None):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE) recorded in
    profiles/traffic_<workload>.json, or None if absent, taken on other
    kernel sources or under another kernel schedule."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != source_sha256() or kind not in t.get("kernels", {}):
        return None
    if sched is not None and t.get("schedule") is not None and list(t["schedule"]) != list(sched):
        return None
    k = t["kernels"][kind]
    return round(k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"])


def kernel_variant(kind, sched, n1=256, fp64=False):
    """Compiled kernel that a schedule selects for one kernel kind (3D grid
    n1^3, uniform spacing), named as rocprofv3 lists it."""
    T = "double" if fp64 else "float"
    tile, tz, xv, yv, zv, zr = sched
    if kind == "k_apply":
        tiles = ([(32, 8), (16, 16), (64, 4), (32, 16), (16, 32)] if fp64 else
                 [(64, 4), (32, 8), (16, 16), (64, 8), (32, 16)])
        bx, by = tiles[tile]
        return f"k_stencil3t<{T}, {T}, 0, true, {bx}, {by}>"
    if kind in ("x_fwd", "x_inv"):
        v, rp = xv & 1, xv >> 1
        return (f"k_xfwd<{T}, {n1 // 2}, {v}, {rp}, 0>" if kind == "x_fwd" else f"k_xinv<{T}, {n1 // 2}, {v}, {rp}>")
    if kind in ("y_fwd", "y_inv"):
        return f"k_ypass<{T}, {n1}, {'true' if kind == 'y_inv' else 'false'}, {yv & 1}, {yv >> 1}>"
    B = 4 if fp64 else 8
    tx, nth = [(B, 512), (B // 2, 512), (B, 768), (2 * B, 1024)][zv]
    return f"k_zpass<{T}, {n1}, {tx}, {zr}, {nth}>"


def cpu_full_size(E, nu, gpu_iters, iters=3):
    """The CPU oracle's matrix-free PCG (numpy K-apply, scipy.fft
    preconditioner, FP64) on one load of the full grid: time per iteration,
    and the time to solve every load, extrapolated from it with the GPU's
    FP64 iteration counts."""
    from oracle import fem, matfree
    g = fem.Grid(E.shape[::-1])
    t0 = time.perf_counter()
    pre = matfree.FourierPreconditioner(g, *matfree.reference_medium(E, nu, 3))
    t_setup = time.perf_counter() - t0
    its = []
    t0 = time.perf_counter()
    matfree.pcg(g, E, nu, np.eye(6)[0], tol=1e-30, maxit=iters, precond=pre,
                callback=lambda it, rel: its.append(time.perf_counter()))
    dt = time.perf_counter() - t0
    s_it = dt / iters
    cores = len(os.sched_getaffinity(0))
    return {
        "s_per_iteration": round(s_it, 3),
        "value": 3 * g.n / s_it,
        "unit": "DOF-CG-iterations/s",
        "cores": cores,
        "kind": "oracle",
        "iterations_timed": iters,
        "timed_s": round(dt, 2),
        "preconditioner_setup_s": round(t_setup, 2),
        "time_to_solution_s_extrapolated": round(s_it * sum(gpu_iters) + t_setup, 1),
        "extrapolation": f"s/iteration x the GPU FP64 iteration counts {list(gpu_iters)} summed over the loads, "
                         "plus the preconditioner setup; not a measured solve",
        "sample": f"{iters} PCG iterations on load eps_11 of the full {g.shape[0]}^3 cell (FP64 numpy matrix-free "
                  f"K-apply, single thread; scipy.fft on {cores} workers), the initial residual and "
                  "preconditioning included",
    }


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


def cpu_baseline_uneven(cells, budget_s=20.0, max_n=48):
    """The oracle's whole FP64 PCG solve (matrix-free numpy K-apply, scipy.fft
    preconditioner, tol 1e-6) of load eps_11 for the first cells of the
    batch of at most max_n^3 voxels (one larger cell alone would exceed the
    budget), until about budget_s of host time is spent."""
    from oracle import fem, matfree
    done, dofit, t_all = [], 0.0, 0.0
    for c in cells:
        n1 = c["n"]
        if n1 > max_n:
            continue
        g = fem.Grid((n1,) * 3)
        t0 = time.perf_counter()
        pre = matfree.FourierPreconditioner(g, *matfree.reference_medium(c["E"], c["nu"], 3))
        _, it, _ = matfree.pcg(g, c["E"], c["nu"], np.eye(6)[0], tol=1e-6, precond=pre)
        t_all += time.perf_counter() - t0
        dofit += 3 * g.n * it
        done.append(f"{n1}^3 {it} it")
        if t_all >= budget_s:
            break
    cores = len(os.sched_getaffinity(0))
    return {"value": dofit / t_all, "unit": "DOF-CG-iterations/s", "cores": cores, "kind": "oracle",
            "sample": f"whole FP64 PCG solves of load eps_11 to tol 1e-6 (numpy matrix-free K-apply, single "
                      f"thread; scipy.fft preconditioner on {cores} workers; setup included) of the first "
                      f"{len(done)} cells of the batch with at most {max_n}^3 voxels ({', '.join(done)}), "
                      f"{t_all:.1f} s"}


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
    # timed steps as in production (graphs, no events), then one step with
    # eager launches and per-kernel events for the kernel times
    times = []
    iters = np.zeros(len(cells))
    for i in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C, infos = b.effective_stiffness()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        it = np.array([sum(inf["iters"]) for inf in infos], dtype=np.float64)
        assert i == 0 or np.array_equal(it, iters)
        iters = it
    dt = float(np.median(times))
    b.profile(True)
    _, infos_p = b.effective_stiffness()
    prof = b.profile_read()
    b.profile(False)
    prof_s = infos_p[0]["seconds"]
    b.close()
    nvox = np.array([c["n"] ** 3 for c in cells], dtype=np.float64)
    value = float((3 * nvox * iters).sum() / dt)
    gpu_ms = sum(v[0] for v in prof.values())
    kinds = ["k_apply", "x_fwd", "y_fwd", "last", "y_inv", "x_inv"]
    dom = max(kinds, key=lambda k: prof[k][0])
    ms_tot, launches = prof[dom]
    # per slot: one launch per iteration (+ the initial preconditioning for
    # the FFT passes); material bytes of the K-apply not counted
    extra = 0 if dom == "k_apply" else 6
    alg_bytes = float(((iters + extra) * np.array([byte_model(dom, n, 4) for n in nvox])).sum())
    achieved = alg_bytes / (ms_tot * 1e-3) / 1e9
    progress(f"timed {args.steps} steps: median {dt:.3f} s (profiled step {prof_s:.3f} s, kernels {gpu_ms / 1e3:.3f} s)")
    return {
        "metric": "DOF-CG-iterations/sec, uneven batch (mixed, tol 1e-6)",
        "value": value,
        "unit": "DOF-CG-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "timing": "median wall time of the timed batched effective-stiffness calls (captured graphs)",
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
        "kernel_ms_profiled_step": {k: round(v[0], 2) for k, v in prof.items()},
        "profiled_step_s": round(prof_s, 4),
        "gpu_busy_frac_profiled_step": round(gpu_ms * 1e-3 / prof_s, 4),
        "kernel_time_over_timed_step": round(gpu_ms * 1e-3 / dt, 4),
        "cpu_baseline": None if args.no_cpu else cpu_baseline_uneven(cells),
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


def bench_spheres64(args, B, ms, progress):
    """The 64^3 sphere cell: RSA spheres r 4-8 voxels, vf 0.3, seed 2,
    E 1:100, nu 0.3, all six unit loads; FP64 to tol 1e-10 and mixed to
    tol 1e-7 (C* error of the mixed solve against the FP64 one).  The CPU
    baseline is the oracle's whole FP64 PCG solve of load eps_11 at the same
    size and tolerance, timed end to end."""
    import torch
    n1 = 64
    n = n1 ** 3
    E, nu, vf = ms.spheres_cell(n1, 0.3, seed=2, contrast=100.0)
    Ed = torch.from_numpy(E.ravel()).cuda()
    nud = torch.from_numpy(nu.ravel()).cuda()
    res = {}
    for key, prec, tol in (("fp64", B.FP64, 1e-10), ("mixed", B.MIXED, 1e-7)):
        with B.Cell((n1,) * 3, precision=prec, tol=tol) as c:
            c.set_material(Ed, nud)
            if not args.no_tune:
                c.autotune()
            for _ in range(args.warmup):
                c.effective_stiffness()
            C, times, infos = timed_steps(c, args.steps, torch)
        med = float(np.median(times))
        res[key] = dict(C=C, med=med, iters=infos[-1]["iters"], relres=infos[-1]["relres"])
        progress(f"{key}: median {med * 1e3:.2f} ms, iters {infos[-1]['iters']}")
    err = float(np.abs(res["mixed"]["C"] - res["fp64"]["C"]).max() / np.abs(res["fp64"]["C"]).max())
    value = 3 * n * sum(res["mixed"]["iters"]) / res["mixed"]["med"]
    cpu = None
    if not args.no_cpu:
        from oracle import fem, matfree
        progress("cpu oracle: full FP64 PCG of load eps_11 ...")
        g = fem.Grid((n1,) * 3)
        t0 = time.perf_counter()
        pre = matfree.FourierPreconditioner(g, *matfree.reference_medium(E, nu, 3))
        u, it, rel = matfree.pcg(g, E, nu, np.eye(6)[0], tol=1e-10, precond=pre)
        dt = time.perf_counter() - t0
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": 3 * n * it / dt, "unit": "DOF-CG-iterations/s", "cores": cores, "kind": "oracle",
               "time_to_solution_s": round(dt, 2), "iters": it, "relres": rel,
               "gpu_fp64_time_to_solution_s_one_load": round(res["fp64"]["med"] / 6, 5),
               "sample": f"the whole solve of load eps_11 at {n1}^3 (FP64 numpy matrix-free K-apply, single thread; "
                         f"scipy.fft preconditioner on {cores} workers; symbol setup included), tol 1e-10, "
                         f"{it} iterations, {dt:.1f} s"}
    return {
        "metric": "DOF-CG-iterations/sec, 64^3 sphere cell (mixed, tol 1e-7)",
        "value": value, "unit": "DOF-CG-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["mixed"]["med"] * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"spheres3d_64: 64^3 RSA spheres (r 4-8, vf target 0.3, achieved {vf:.3f}, seed 2), "
                               "E 1:100, nu 0.3, six unit loads",
                   "voxels": n, "iters_mixed": res["mixed"]["iters"], "iters_fp64": res["fp64"]["iters"]},
        "fp64": {"time_to_solution_s": round(res["fp64"]["med"], 5),
                 "dof_cg_iter_per_s": 3 * n * sum(res["fp64"]["iters"]) / res["fp64"]["med"],
                 "speedup_mixed_over_fp64": round(res["fp64"]["med"] / res["mixed"]["med"], 3),
                 "C_err_mixed_tol1e-7_vs_fp64_tol1e-10": err},
        "cpu_baseline": cpu,
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


# ------------------------------------------------- rocprofv3 summaries
# `python bench.py summarize-stats ...` / `summarize-traffic ...` turn the
# CSV output of rocprofv3 runs of this script into the text summaries kept
# under profiles/ (and the JSON that roofline.traffic reads).

KIND_PATTERNS = [("k_apply", "k_stencil"), ("x_fwd", "k_xfwd<"), ("y_fwd", "k_ypass<"), ("last", "k_zpass<"),
                 ("y_inv", "k_ypass<"), ("x_inv", "k_xinv<")]


def kernel_kind(name):
    """Iteration kernel kind of a rocprofv3 kernel name (FP32 iteration
    variants only), or None."""
    if "k_stencil3t<float, float, 0" in name or "k_stencil_rw<" in name:
        return "k_apply"
    if "<float" not in name:
        return None
    if "k_xfwd<" in name:
        return "x_fwd" if name.split(">")[0].rstrip().endswith(" 0") else None
    if "k_ypass<" in name:
        return "y_inv" if ", true," in name else "y_fwd"
    if "k_zpass<" in name:
        return "last"
    if "k_xinv<" in name:
        return "x_inv"
    return None


def _csv_rows(directory, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {directory}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _bench_line(path):
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{") and '"metric"' in line:
                return json.loads(line)
    raise SystemExit(f"no bench JSON line in {path}")


def summarize_stats(argv):
    ap = argparse.ArgumentParser(prog="bench.py summarize-stats")
    ap.add_argument("stats_dir")
    ap.add_argument("bench_out", help="the bench.py output of the profiled run (its JSON line)")
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--note", default=None, help="a closing sentence")
    ap.add_argument("--top", type=int, default=0, help="list only the N kernels with the most time")
    a = ap.parse_args(argv)
    rows = _csv_rows(a.stats_dir, "kernel_stats.csv")
    line = _bench_line(a.bench_out)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    n = line["config"]["voxels"]
    iters = line["config"].get("iters_per_step")
    desc = f"ms_per_step = {line['ms_per_step']}"
    if iters is not None:
        desc += f", schedule = {line['config'].get('schedule')}, iterations per load = {iters}"
    elif line.get("roofline"):
        rl = line["roofline"]
        desc += (f"; dominant kernel {rl.get('kernel')} at {rl.get('achieved')} GB/s algorithmic "
                 f"({100 * rl.get('frac', 0):.1f} % of 8 TB/s, average launch {rl.get('avg_launch_ms')} ms "
                 f"over {rl.get('launches')} launches)")
    elif line["config"].get("iters") is not None:
        desc += f", iterations per load = {line['config']['iters']}"
    out = [f"# {a.title}", "",
           f"Workload: {line['config']['workload']}.", "",
           "Command (run from the repository root on one MI355X):", "", "```", a.command, "```", "",
           f"Bench line of the same run: value = {line['value']:.4g} {line['unit']}, {desc}.", "",
           "| kernel | calls | total ms | avg us | % GPU time |", "|---|---:|---:|---:|---:|"]
    shown = rows[:a.top] if a.top > 0 else rows
    for r in shown:
        out.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    if len(shown) < len(rows):
        rest = rows[len(shown):]
        out.append(f"| ({len(rest)} more kernels) | {sum(int(r['Calls']) for r in rest)} | "
                   f"{sum(float(r['TotalDurationNs']) for r in rest) / 1e6:.2f} | | "
                   f"{sum(float(r['Percentage']) for r in rest):.2f} |")
    if iters is None:
        if a.note:
            out += ["", a.note]
        with open(a.out, "w") as fh:
            fh.write("\n".join(out) + "\n")
        print(a.out)
        return
    out += ["", "Algorithmic bandwidth of the iteration kernels from their average launch time above "
            "(byte model of bench.py per active load; launches counted over the solves of the run, "
            "whose loads converge at different iterations):", "",
            "| kind | kernel | B per voxel and load | avg active loads | avg ms | algorithmic GB/s | % of 8 TB/s |",
            "|---|---|---:|---:|---:|---:|---:|"]
    for kind in ("k_apply", "x_fwd", "y_fwd", "last", "y_inv", "x_inv"):
        cand = [r for r in rows if kernel_kind(r["Name"]) == kind]
        if not cand:
            continue
        r = max(cand, key=lambda r: int(r["Calls"]))
        calls = int(r["Calls"])
        nsolve = max(1, round(calls / (max(iters) + (0 if kind == "k_apply" else 1))))
        load_launches = nsolve * (sum(iters) + (0 if kind == "k_apply" else len(iters)))
        avg_loads = load_launches / calls
        bpl = byte_model(kind, n, 4) * avg_loads + (8 * n if kind == "k_apply" else 0)
        ms = float(r["AverageNs"]) / 1e6
        gbs = bpl / (ms * 1e-3) / 1e9
        out.append(f"| {kind} | `{r['Name'].split('(')[0]}` | {byte_model(kind, n, 4) / n:.0f} | {avg_loads:.3f} | "
                   f"{ms:.4f} | {gbs:.0f} | {100 * gbs / HBM_PEAK_GBS:.1f} |")
    if a.note:
        out += ["", a.note]
    with open(a.out, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print(a.out)


def summarize_traffic(argv):
    ap = argparse.ArgumentParser(prog="bench.py summarize-traffic")
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("bench_out", help="the bench.py output of one of the counter runs (its JSON line)")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--commands", nargs=2, required=True)
    ap.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args(argv)
    line = _bench_line(a.bench_out)
    n = line["config"]["voxels"]
    iters = line["config"]["iters_per_step"]
    per = {}
    cal = {}
    for counter, d in (("FETCH_SIZE", a.fetch_dir), ("WRITE_SIZE", a.write_dir)):
        vals = {}
        best_copy = 0.0
        for r in _csv_rows(d, "counter_collection.csv"):
            if r.get("Counter_Name") != counter:
                continue
            name, v = r["Kernel_Name"], float(r["Counter_Value"])
            if "copyBuffer" in name:
                best_copy = max(best_copy, v)
                continue
            vals.setdefault(name, []).append(v)
        copy_kib = a.copy_mib * 1024.0
        if best_copy <= 0:
            raise SystemExit(f"no copy dispatch for {counter}")
        cal[counter] = {"KiB": best_copy, "factor": copy_kib / best_copy}
        for name, v in vals.items():
            kind = kernel_kind(name)
            if kind is None:
                continue
            per.setdefault(kind, {})[name] = per.get(kind, {}).get(name, {})
            per[kind][name][counter] = (len(v), sum(v) / len(v) * 1024.0 * cal[counter]["factor"])
    kernels = {}
    for kind, names in per.items():
        name = max(names, key=lambda nm: names[nm].get("FETCH_SIZE", (0, 0))[0])
        launches, fetch = names[name].get("FETCH_SIZE", (0, 0.0))
        _, write = names[name].get("WRITE_SIZE", (0, 0.0))
        nsolve = max(1, round(launches / (max(iters) + (0 if kind == "k_apply" else 1))))
        load_launches = nsolve * (sum(iters) + (0 if kind == "k_apply" else len(iters)))
        model = byte_model(kind, n, 4) * load_launches / launches + (8 * n if kind == "k_apply" else 0)
        kernels[kind] = {"name": name, "launches": launches, "fetch_bytes_per_launch": fetch,
                         "write_bytes_per_launch": write, "model_bytes_per_launch": model}
    t = {"workload": a.workload, "source_sha256": source_sha256(), "schedule": line["config"].get("schedule"),
         "calibration": {"copy_bytes": a.copy_mib << 20, "FETCH_SIZE_KiB": cal["FETCH_SIZE"]["KiB"],
                         "WRITE_SIZE_KiB": cal["WRITE_SIZE"]["KiB"],
                         "fetch_factor": cal["FETCH_SIZE"]["factor"], "write_factor": cal["WRITE_SIZE"]["factor"]},
         "commands": a.commands, "kernels": kernels}
    base = os.path.join(ROOT, "profiles", f"traffic_{a.workload}")
    with open(base + ".json", "w") as fh:
        json.dump(t, fh, indent=1)
    out = [f"# HBM traffic per launch: PCG iteration kernels, {a.workload} workload", "",
           "Counters: rocprofv3 `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE` (separate runs, KiB per dispatch), "
           f"each scaled by the factor that makes the same counter read {a.copy_mib} MiB for a plain device copy "
           f"of that size (`bench.py --copy-probe {a.copy_mib}`):", "",
           f"* FETCH_SIZE of the copy: {cal['FETCH_SIZE']['KiB']:.0f} KiB -> factor {cal['FETCH_SIZE']['factor']:.3f}",
           f"* WRITE_SIZE of the copy: {cal['WRITE_SIZE']['KiB']:.0f} KiB -> factor {cal['WRITE_SIZE']['factor']:.3f}",
           "", f"Kernel schedule: {t['schedule']}.", "", "Commands:", "", "```"] + a.commands + ["```", "",
           "| kind | kernel | launches | fetch MiB/launch | write MiB/launch | model MiB/launch | traffic / model |",
           "|---|---|---:|---:|---:|---:|---:|"]
    for kind in ("k_apply", "x_fwd", "y_fwd", "last", "y_inv", "x_inv"):
        if kind not in kernels:
            continue
        k = kernels[kind]
        tot = k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
        out.append(f"| {kind} | `{k['name'].split('(')[0]}` | {k['launches']} | {k['fetch_bytes_per_launch'] / 2**20:.1f} | "
                   f"{k['write_bytes_per_launch'] / 2**20:.1f} | {k['model_bytes_per_launch'] / 2**20:.1f} | "
                   f"{tot / k['model_bytes_per_launch']:.3f} |")
    out += ["", f"Kernel sources (csrc/*.hip, *.h) sha256 at measurement: `{t['source_sha256']}`. bench.py reports "
            "these bytes as `roofline.traffic` only while the sources hash to this value and the schedule matches."]
    with open(base + ".md", "w") as fh:
        fh.write("\n".join(out) + "\n")
    print(base + ".json", base + ".md")


# gfx950: 256 CUs x 4 SIMDs; a 64-lane FP32/FP64 VALU instruction (not
# packed) occupies its SIMD for 4 cycles
SIMDS = 1024
VALU_CYCLES = 4
CLOCK_HZ = 2.4e9


def summarize_counters(argv):
    ap = argparse.ArgumentParser(prog="bench.py summarize-counters")
    ap.add_argument("pmc_dirs", nargs="+", help="rocprofv3 --pmc output directories (one per pass)")
    ap.add_argument("--bench-out", required=True, help="the bench.py output of one of the runs (its JSON line)")
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--commands", nargs="+", required=True)
    a = ap.parse_args(argv)
    line = _bench_line(a.bench_out)
    n = line["config"]["voxels"]
    iters = line["config"]["iters_per_step"]
    per = {}  # kind -> name -> counter -> [values]
    dur = {}  # kind -> name -> [ns]
    for d in a.pmc_dirs:
        seen = set()
        for r in _csv_rows(d, "counter_collection.csv"):
            kind = kernel_kind(r["Kernel_Name"])
            if kind is None:
                continue
            name = r["Kernel_Name"].split("(")[0]
            per.setdefault(kind, {}).setdefault(name, {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
            key = (r["Dispatch_Id"], name)
            if key not in seen:
                seen.add(key)
                dur.setdefault(kind, {}).setdefault(name, []).append(
                    float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
    out = [f"# {a.title}", "", f"Workload: {line['config']['workload']}.", "",
           f"Kernel schedule: {line['config'].get('schedule')}. Counter passes (one rocprofv3 run each):", "",
           "```"] + a.commands + ["```", "",
           "Per launch, averaged over the launches of the run (counters summed over the whole device). "
           "A unit is one voxel of one active load case. VALU-busy = SQ_INSTS_VALU x 4 cycles / "
           f"({SIMDS} SIMDs x launch duration x {CLOCK_HZ / 1e9:.1f} GHz); the durations are those of the "
           "counter runs (dispatches serialised by the collection).", ""]
    rows = []
    for kind in ("k_apply", "x_fwd", "y_fwd", "last", "y_inv", "x_inv"):
        if kind not in per:
            continue
        name = max(per[kind], key=lambda nm: max(len(v) for v in per[kind][nm].values()))
        c = {k: sum(v) / len(v) for k, v in per[kind][name].items()}
        launches = max(len(v) for v in per[kind][name].values())
        nsolve = max(1, round(launches / (max(iters) + (0 if kind == "k_apply" else 1))))
        load_launches = nsolve * (sum(iters) + (0 if kind == "k_apply" else len(iters)))
        units = n * load_launches / launches
        ns = sum(dur[kind][name]) / len(dur[kind][name])
        rows.append((kind, name, launches, units, ns, c))
    names = sorted({k for r in rows for k in r[5]})
    out += ["| kind | kernel | launches | units / launch | avg us | " + " | ".join(f"`{k}`" for k in names) + " |",
            "|---|---|---:|---:|---:|" + "---:|" * len(names)]
    for kind, name, launches, units, ns, c in rows:
        out.append(f"| {kind} | `{name}` | {launches} | {units:.4g} | {ns / 1e3:.1f} | " +
                   " | ".join(f"{c[k]:.4g}" if k in c else "-" for k in names) + " |")
    out += ["", "Derived:", "", "| kind | VALU instr / wave | VALU instr / unit (per lane) | LDS instr / unit | "
            "VMEM instr / unit | VALU-busy | L2 hit rate |", "|---|---:|---:|---:|---:|---:|---:|"]
    for kind, name, launches, units, ns, c in rows:
        def g(k):
            return c.get(k)
        waves = g("SQ_WAVES")
        valu = g("SQ_INSTS_VALU")
        vw = f"{valu / waves:.0f}" if valu and waves else "-"
        vu = f"{valu * 64 / units:.0f}" if valu else "-"
        lu = f"{g('SQ_INSTS_LDS') * 64 / units:.1f}" if g("SQ_INSTS_LDS") else "-"
        vm = (g("SQ_INSTS_VMEM_RD") or 0) + (g("SQ_INSTS_VMEM_WR") or 0)
        mu = f"{vm * 64 / units:.2f}" if vm else "-"
        busy = f"{valu * VALU_CYCLES / (SIMDS * ns * 1e-9 * CLOCK_HZ):.2f}" if valu else "-"
        hit = (f"{g('TCC_HIT_sum') / (g('TCC_HIT_sum') + g('TCC_MISS_sum')):.2f}"
               if g("TCC_HIT_sum") is not None and g("TCC_MISS_sum") else "-")
        out.append(f"| {kind} | {vw} | {vu} | {lu} | {mu} | {busy} | {hit} |")
    with open(a.out, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print(a.out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="keep the default kernel schedule (other workloads)")
    ap.add_argument("--tune", action="store_true",
                    help="grf3d: autotune the kernel schedules instead of the pinned headline schedules")
    ap.add_argument("--cpu-full", action="store_true",
                    help="grf3d: also time the CPU oracle at the full grid size (3 PCG iterations)")
    ap.add_argument("--schedule", default=None,
                    help="six comma-separated ints: use this kernel schedule instead of tuning")
    ap.add_argument("--workload", default="grf3d",
                    choices=["grf3d", "uneven", "hyper", "surrogate", "adjoint", "spheres64"],
                    help="grf3d: the 256^3 headline workload; uneven: the batch of sphere cells; "
                         "hyper: the neo-Hookean Newton-PCG on the grf3d geometry; spheres64: the 64^3 "
                         "sphere cell with the whole CPU oracle solve")
    ap.add_argument("--cells", type=int, default=512, help="cells of the uneven batch")
    ap.add_argument("--contrast", type=float, default=10.0, help="phase contrast of the hyper workload")
    ap.add_argument("--M", type=int, default=4, help="sampling step of the surrogate workload")
    ap.add_argument("--ell", type=float, default=32.0, help="correlation length of the surrogate workload")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    if len(sys.argv) > 1 and sys.argv[1] in ("summarize-stats", "summarize-traffic", "summarize-counters"):
        {"summarize-stats": summarize_stats, "summarize-traffic": summarize_traffic,
         "summarize-counters": summarize_counters}[sys.argv[1]](sys.argv[2:])
        return
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
    if args.workload == "spheres64":
        print(json.dumps(bench_spheres64(args, B, ms, progress)), flush=True)
        return
    print(json.dumps(bench_grf3d(args, B, ms, progress, torch)), flush=True)


# Kernel schedules the headline workload runs (stencil tile, z extent, x, y
# and last-pass variants; see the autotuner): pinned so that the timed run,
# the rocprofv3 kernel-time summary and the traffic counters all measure the
# same compiled variants.  `--tune` runs the autotuner instead.
HEADLINE_SCHEDULE = {"mixed": (1, 64, 3, 0, 0, 0), "fp64": (0, 64, 1, 2, 0, 1)}


def timed_steps(cell, steps, torch):
    """Wall time of each effective-stiffness call (graphs on, no events),
    with a synchronisation on both sides of every step."""
    times, infos = [], []
    C = None
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C, info = cell.effective_stiffness()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        infos.append(info)
    return C, times, infos


def bench_grf3d(args, B, ms, progress, torch):
    n1 = args.n
    n = n1 ** 3
    E, nu = ms.two_phase_grf(n1, seed=3)
    Ed = torch.from_numpy(E.ravel()).cuda()
    nud = torch.from_numpy(nu.ravel()).cuda()
    torch.cuda.synchronize()

    def setup(precision, tol, key):
        cell = B.Cell((n1, n1, n1), precision=precision, tol=tol)
        cell.set_material(Ed, nud)
        if args.schedule:
            cell.schedule = tuple(int(v) for v in args.schedule.split(","))
        elif args.tune:
            t_tune = time.perf_counter()
            cell.autotune()
            progress(f"autotune ({key}): schedule {cell.schedule} in {time.perf_counter() - t_tune:.2f} s")
        elif n1 == 256:
            cell.schedule = HEADLINE_SCHEDULE[key]
        return cell

    # ---------------------------------------------------------------- mixed
    cell = setup(B.MIXED, 1e-6, "mixed")
    sched = cell.schedule
    for i in range(args.warmup):
        C_mixed, info = cell.effective_stiffness()
        progress(f"warmup {i}: iters {info['iters']} {info['seconds']:.2f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C_mixed, times, per_step = timed_steps(cell, args.steps, torch)
    dt = time.perf_counter() - t0
    med = float(np.median(times))
    iters_step = sum(per_step[-1]["iters"])
    progress(f"timed {args.steps} steps in {dt:.3f} s (median {med * 1e3:.1f} ms, min {min(times) * 1e3:.1f}, "
             f"max {max(times) * 1e3:.1f}), iters {per_step[-1]['iters']}, "
             f"refinements {per_step[-1]['refinements']}")
    assert all(sum(i["iters"]) == iters_step for i in per_step)
    value = 3 * n * iters_step / med
    # per-kernel times: one more step with eager launches and HIP events
    # around every kernel on the library's stream (graph replays carry no
    # per-kernel timestamps); the same kernels as the timed steps
    cell.profile(True)
    _, info_p = cell.effective_stiffness()
    prof = cell.profile_read()
    cell.profile(False)
    prof_step_s = info_p["seconds"]
    cell.close()
    del cell

    # roofline of the dominant kernel (largest GPU time in the profiled step)
    kinds = ["k_apply", "x_fwd", "y_fwd", "last", "y_inv", "x_inv"]
    dom = max(kinds, key=lambda k: prof[k][0])
    ms_tot, launches = prof[dom]
    load_launches = iters_step + (0 if dom == "k_apply" else 6)
    alg_bytes = load_launches * byte_model(dom, n, 4)
    if dom == "k_apply":
        alg_bytes += launches * 8 * n
    achieved = alg_bytes / (ms_tot * 1e-3) / 1e9
    gpu_ms = sum(prof[k][0] for k in prof)
    copy_gbs = copy_bandwidth(torch)
    roofline = {
        "bound": "hbm",
        "kernel": dom,
        "variant": kernel_variant(dom, sched),
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(dom, f"grf3d_{n1}", sched),
        "avg_launch_ms": round(ms_tot / launches, 4),
        "launches": launches,
        "bytes_per_launch": round(alg_bytes / launches),
        "timing": "HIP events around every launch of one profiled step (eager launches), after the timed steps",
        "copy_gbs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 4),
    }
    # whole-iteration fractions on the wall time of a timed step: the bytes
    # of this schedule (64 B per DOF-iteration, FP32) and of the textbook
    # fused schedule (72 B per DOF-iteration)
    step_bytes = sum((iters_step + (0 if k == "k_apply" else 6)) * byte_model(k, n, 4) for k in kinds) \
        + prof["k_apply"][1] * 8 * n
    loop_ms = sum(prof[k][0] for k in kinds)
    iteration = {
        "bytes_per_dof_iter": round(step_bytes / (3 * n * iters_step), 2),
        "frac_wall": round(step_bytes / med / 1e9 / HBM_PEAK_GBS, 4),
        "frac_wall_72B_model": round(72.0 * value / 1e9 / HBM_PEAK_GBS, 4),
        "frac_of_copy_wall": round(step_bytes / med / 1e9 / copy_gbs, 4),
        "frac_kernel_time": round(step_bytes / (loop_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }

    # ---------------------------------------------------------------- fp64
    fp64 = None
    if not args.no_fp64:
        with B.Cell((n1, n1, n1), precision=B.FP64, tol=1e-10) as c64:
            c64.set_material(Ed, nud)
            if n1 == 256 and not args.tune:
                c64.schedule = HEADLINE_SCHEDULE["fp64"]
            C_ref, info_ref = c64.effective_stiffness()
            progress(f"fp64 tol 1e-10: iters {info_ref['iters']} {info_ref['seconds']:.2f} s")
        c64 = setup(B.FP64, 1e-6, "fp64")
        for i in range(max(1, args.warmup)):
            c64.effective_stiffness()
        C_64, t64, inf64 = timed_steps(c64, max(2, min(args.steps, 5)), torch)
        sched64 = c64.schedule
        c64.close()
        fp64_tts = float(np.median(t64))
        progress(f"fp64 tol 1e-6: iters {inf64[-1]['iters']} median {fp64_tts:.3f} s over {len(t64)} steps")
        err = lambda C: float(np.abs(C - C_ref).max() / np.abs(C_ref).max())
        fp64 = {
            "time_to_solution_s": round(fp64_tts, 4),
            "iters": inf64[-1]["iters"],
            "schedule": list(sched64),
            "dof_cg_iter_per_s": 3 * n * sum(inf64[-1]["iters"]) / fp64_tts,
            "mixed_time_to_solution_s": round(med, 4),
            "speedup_mixed_over_fp64": round(fp64_tts / med, 3),
            "C_err_mixed_vs_fp64_tol1e-10": err(C_mixed),
            "C_err_fp64_tol1e-6_vs_fp64_tol1e-10": err(C_64),
            "timing": "median of timed steps, same protocol as the mixed line (warm, graphs on)",
        }

    cpu = None
    if not args.no_cpu:
        progress("cpu oracle baseline ...")
        cpu = cpu_baseline(E, nu)
    cpu_full = None
    if args.cpu_full:
        progress("cpu oracle at the full size ...")
        iters64 = fp64["iters"] if fp64 else per_step[-1]["iters"]
        cpu_full = cpu_full_size(E, nu, iters64)

    out = {
        "metric": "DOF-CG-iterations/sec at 256^3 (mixed vs FP64, rel err <=1e-6); % HBM roofline",
        "value": value,
        "unit": "DOF-CG-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(med * 1e3, 3),
        "mean_ms_per_step": round(dt / args.steps * 1e3, 3),
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
            "timing": "median wall time of the timed effective-stiffness calls (captured graphs, no events)",
        },
        "roofline": roofline,
        "iteration": iteration,
        "kernel_ms_profiled_step": {k: round(v[0], 2) for k, v in prof.items()},
        "profiled_step_s": round(prof_step_s, 4),
        "gpu_busy_frac": round(gpu_ms * 1e-3 / prof_step_s, 4),
        "fp64": fp64,
        "cpu_baseline": cpu,
        "cpu_full_size": cpu_full,
    }
    return out


if __name__ == "__main__":
    main()
