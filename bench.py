#!/usr/bin/env python3
"""Throughput of the laplacianFoam hot path on one MI355X.

A step is one implicit-Euler time step of the 256^3 z-graded box (expansion
ratio 10, fixedValue 273/573 K on the x walls, zeroGradient elsewhere,
DT = 1e-3, dt = 1e-3): assembly of ddt(T) - laplacian(DT, T) into the LDU
matrix and its PCG solve (diagonal preconditioner, normalised residual 1e-9),
FP64.  The metric is cell-PCG-iterations per second over the timed steps
(cells x PCG iterations / wall time of the whole steps, assembly included).

Inputs are resident in HBM before the timed region; warmup steps run first,
then T is reset to T0 so the timed steps are steps 1..K of the workload.

Also reported: the dominant kernel's roofline (algorithmic bytes per launch /
average device duration, from HIP events on the library's stream during a
separate pass over the same steps), HBM traffic from rocprofv3 counters when
the kernel is unchanged since they were taken, and the oracle's rate on a
bounded sample on the host CPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
# The serving leg runs persistent batched kernels on several streams next to
# multi-kernel solves on others; with HIP's default of 4 hardware queues per
# process, streams share queues and a short kernel waits behind a long one.
# Set before the HIP runtime starts (torch is imported later).
os.environ.setdefault("GPU_MAX_HW_QUEUES", "16")

METRIC = "cell-PCG-iters/sec + Amul/PCG HBM GB/s (% peak), FP64 vs mixed @1e-8; p99"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
KERNEL_SOURCES = ["paper_2507_18268_amd/csrc/lf_pcg.hip", "paper_2507_18268_amd/csrc/lf_kernels.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_amul_dot_graded256.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


MIXED_SOURCES = ["paper_2507_18268_amd/csrc/lf_mixed.hip", "paper_2507_18268_amd/csrc/lf_kernels.h"]
MIXED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mx_amul_graded256.json")
GRAD_SOURCES = ["paper_2507_18268_amd/csrc/lf_grad.hip"]
GRAD_LABEL = "256^3 box graded in z (ratio 10) and skewed"
GRAD_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_grad_band_skewed256.json")
GRAD_ROWS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_grad_rows_permuted192.json")


def kernel_source_hash(sources=None):
    h = hashlib.sha256()
    for rel in (sources or KERNEL_SOURCES):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def amul_bytes(n_cells, n_faces, value_bytes=8, addressed=True, unit_diag=False):
    """Algorithmic bytes of one LDU product: x, diag and Ax once per cell, the
    coefficient once per face and, when the faces are addressed (owner and
    neighbour lists), their two int32 addresses.  A structured numbering (the
    band layout) needs no addresses: the neighbour of row c across band k is
    c + d_k.  A matrix with unit diagonal (the Jacobi-scaled one) has no
    diagonal to read."""
    per_cell = 2 if unit_diag else 3
    return per_cell * value_bytes * n_cells + (value_bytes + (8 if addressed else 0)) * n_faces


def layout_bytes(mesh, layout_name, value_bytes=8, unit_diag=False):
    """Bytes one LDU product must move in the layout it runs in: p, diag and Ap
    per cell (no diag with a unit diagonal) plus, for the band layout, one
    coefficient per band slot (no indices); for the row layout, per stored
    entry its coefficient and int32 column, and one uint8 row length per
    cell."""
    import numpy as np
    N = mesh.n_cells
    if layout_name == "bands":
        K = np.unique(mesh.neighbour.astype(np.int64) - mesh.owner).size
        return (2 if unit_diag else 3) * value_bytes * N + value_bytes * K * N
    rl = np.bincount(mesh.owner, minlength=N) + np.bincount(mesh.neighbour, minlength=N)
    pad = (-N) % 64
    E = int(np.concatenate([rl, np.zeros(pad, rl.dtype)]).reshape(-1, 64).max(axis=1).sum()) * 64
    return 3 * value_bytes * N + (value_bytes + 4) * E + N


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(p, budget_s):
    """The oracle (single thread, FP64) on the first step(s) of the same
    workload, the calling thread pinned to one host core."""
    from oracle import oracle
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[0]
    os.sched_setaffinity(0, {core})
    try:
        steps, solve_s, iters = 0, 0.0, 0
        T = p.T0.copy()
        t_start = time.perf_counter()
        while steps < p.steps:
            T, st, _ = oracle.run(p.mesh, p.bcs, p.DT, p.dt, 1, T)
            steps += 1
            solve_s += st[0]["solve_s"]
            iters += st[0]["n_iter"]
            if time.perf_counter() - t_start > budget_s:
                break
    finally:
        os.sched_setaffinity(0, set(allowed))
    return {"value": p.mesh.n_cells * iters / solve_s, "unit": "cell-PCG-iters/s", "cores": 1,
            "kind": "oracle", "host_cpu": host_cpu_model(), "pinned_core": core,
            "host_cores_visible": len(allowed),
            "sample": f"first {steps} time step(s) of the same workload, PCG solve time only, "
                      f"{iters} iterations, {solve_s:.2f} s, one host thread pinned to core {core}"}


def run_mixed(L, torch, p, mesh, prob64, T0, args):
    """Precision form on the same workload: timed like the FP64 run, then an
    untimed pass stepping both forms side by side for the per-step error."""
    N = p.mesh.n_cells
    opts = L.make_opts(tol=prob64.opts.tol, rel_tol=prob64.opts.rel_tol,
                       max_iter=prob64.opts.max_iter, precision=L.LF_PREC_MIXED,
                       inner_tol=args.inner_tol)
    pm = L.Problem(mesh, p.bcs, p.DT, p.dt, opts)
    pm.set_T(T0)
    if args.warmup > 0:
        pm.step(args.warmup)
    pm.set_T(T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, _ = pm.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    inner = sum(s["n_iter"] for s in stats)
    # kernel profile of the same steps
    pm.set_T(T0)
    pm.profile(True)
    pm.step(args.steps)
    torch.cuda.synchronize()
    prof = pm.profile_read()
    pm.profile(False)
    # per-step error on the same system (each step starts from the precision
    # form's own T_n): against the FP64 path at the same tolerance (itself
    # checked against the oracle), and against an FP64 solve of that system
    # converged to round-off (tol 1e-13), for both forms
    ref_opts = L.make_opts(tol=1e-13, rel_tol=0.0, max_iter=prob64.opts.max_iter)
    pref = L.Problem(mesh, p.bcs, p.DT, p.dt, ref_opts)
    a = torch.empty(N, dtype=torch.float64, device="cuda")
    b = torch.empty(N, dtype=torch.float64, device="cuda")
    t = torch.empty(N, dtype=torch.float64, device="cuda")
    pm.set_T(T0)
    n_acc = min(args.steps, args.accuracy_steps)
    e_mf, e_mt, e_ft = [], [], []
    for _ in range(n_acc):
        pm.get_T(a)
        prob64.set_T(a)
        pref.set_T(a)
        pm.step(1)
        prob64.step(1)
        pref.step(1)
        pm.get_T(a)
        prob64.get_T(b)
        pref.get_T(t)
        e_mf.append(float(((a - b).abs() / b.abs()).max()))
        e_mt.append(float(((a - t).abs() / t.abs()).max()))
        e_ft.append(float(((b - t).abs() / t.abs()).max()))
    banded = pm.layout() == L.LF_LAYOUT_BANDS
    walk = pm.amul_form()
    # the FP32 inner product takes the block walk with the FP64 one when the
    # box's nx is a multiple of 4
    nx = int(p.mesh.shape[0]) if getattr(p.mesh, "shape", None) is not None else 0
    inner_box = walk == 2 and nx % 4 == 0
    pref.close()
    pm.close()
    kernels = {k: {"avg_us": 1e3 * ms / n, "launches": n} for k, (ms, n) in prof.items()}
    return {"value_cell_steps_per_s": N * args.steps / wall, "inner_tol": opts.inner_tol,
            "kernel_avg_us": kernels,
            "roofline": mixed_roofline(kernels, N, p.mesh.n_faces, banded, walk, inner_box),
            "accuracy_steps": n_acc,
            "accuracy_reading": "per step on the same system: each step of the precision form, of "
                                "the FP64 path at tol 1e-9 (itself within 1e-8 of the oracle in the "
                                "parity tests) and of an FP64 solve converged to tol 1e-13 starts "
                                "from the precision form's own T_n; the precision form refines to "
                                "0.1 tol",
            "max_rel_T_err_vs_converged_fp64_max": max(e_mt),
            "fp64_at_tol_max_rel_T_err_vs_converged_fp64_max": max(e_ft),
            "max_rel_T_err_vs_converged_fp64_first_steps": e_mt[:5],
            "fp64_at_tol_err_vs_converged_first_steps": e_ft[:5],
            "ms_per_step": wall * 1e3 / args.steps,
            "inner_iters_per_step_mean": inner / len(stats),
            "outer_passes_per_step_mean": sum(s["n_outer"] for s in stats) / len(stats),
            "inner_cell_iters_per_s": N * inner / wall,
            "all_converged": all(s["converged"] == 1 for s in stats),
            "max_rel_T_err_vs_fp64_at_tol_max": max(e_mf),
            "max_rel_T_err_vs_fp64_at_tol_first_steps": e_mf[:5],
            "speedup_vs_fp64_time_to_tol": None}


# Bytes each kernel of the precision form must move per launch, band layout
# (FP32 inner vectors and coefficients, FP64 outer fields); per cell and per
# internal face.  The inner product reads the FP32 scaled coefficient of each
# face once (unit diagonal, not read).
MIXED_KERNEL_BYTES = {
    "inner_amul_dot": ("p, q (FP32) per cell + FP32 coefficient per face", 8, 4),
    "inner_update": ("q, s, r read and r written (FP32) per cell", 16, 0),
    "inner_direction": ("r, p, y read and p, y written (FP32) per cell", 20, 0),
    "mixed_residual": ("diag, source, T (FP64), p (FP32) read, r, y (FP32) written per cell "
                       "+ FP64 coefficient per face", 36, 8),
    "mixed_prep": ("s (FP32) per cell + FP64 coefficient read and FP32 written per face", 4, 12),
    "mixed_correct": ("T read and written (FP64), y, p, s read (FP32) per cell", 28, 0),
}


def mixed_roofline(kernels, n_cells, n_faces, banded, walk, inner_box=False):
    """Roofline of the precision form's kernels: algorithmic bytes (above) over
    the average launch time; the dominant one (largest total time) in the
    roofline object, every one in its table.  Counter traffic for the inner
    product when the record matches the sources."""
    table = {}
    for k, (what, per_cell, per_face) in MIXED_KERNEL_BYTES.items():
        if k not in kernels:
            continue
        b = per_cell * n_cells + per_face * n_faces
        us = kernels[k]["avg_us"]
        gbps = b / (us * 1e-6) / 1e9
        table[k] = {"bytes_per_launch": b, "bytes": what, "avg_us": us, "GBps": gbps,
                    "frac": gbps / HBM_PEAK_GBS, "launches": kernels[k]["launches"]}
    if not table or not banded:
        return {"kernels": table}
    dom = max(table, key=lambda k: table[k]["avg_us"] * table[k]["launches"])
    d = table[dom]
    kname = {"inner_amul_dot": "k_mx_amul_dot_box" if inner_box else ("k_mx_amul_dot_walk" if walk else "k_mx_amul_dot"),
             "inner_update": "k_mx_update", "inner_direction": "k_mx_direction",
             "mixed_residual": {0: "k_mx_residual", 1: "k_mx_residual_walk", 2: "k_mx_residual_box"}[walk],
             "mixed_prep": "k_mx_scale", "mixed_correct": "k_mx_correct"}[dom]
    roof = {"kernel": kname, "bound": "hbm", "achieved": d["GBps"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": d["frac"], "traffic": None,
            "algorithmic_bytes_per_launch": d["bytes_per_launch"], "avg_launch_us": d["avg_us"],
            "kernels": table}
    if os.path.exists(MIXED_TRAFFIC_FILE):
        with open(MIXED_TRAFFIC_FILE) as f:
            tr = json.load(f)
        if (tr.get("source_sha256") == kernel_source_hash(MIXED_SOURCES) and tr.get("n_cells") == n_cells
                and tr.get("kernel") == kname):
            roof["traffic"] = tr["hbm_bytes_per_launch"]
            roof["traffic_GBps"] = roof["traffic"] / (d["avg_us"] * 1e-6) / 1e9
            roof["traffic_frac"] = roof["traffic_GBps"] / HBM_PEAK_GBS
    return roof


def run_config_leg(L, torch, name, steps, warmup=1, skew=False, precond=None):
    """Another config of the workload family, timed like the main line: `steps`
    time steps from T0 after `warmup` steps, wall clock around the whole steps.
    skew: the config's box mapped by synth.SKEW (non-orthogonal faces), so every
    step also runs the Laplacian's explicit non-orthogonal correction."""
    import synth
    t = time.perf_counter()
    p = synth.build_config(name, steps=steps)
    if skew:
        p.mesh = synth.affine(p.mesh, synth.SKEW)
    N = p.mesh.n_cells
    log(f"[bench] {name}{' skewed' if skew else ''}: {N} cells, mesh generated in {time.perf_counter() - t:.1f} s")
    pc_name = precond or p.precond
    precond = {"dic": L.LF_PC_DIC, "amg": L.LF_PC_AMG}.get(pc_name, L.LF_PC_DIAGONAL)
    precision = L.LF_PREC_MIXED if p.precision == "mixed" else L.LF_PREC_FP64
    opts = L.make_opts(tol=synth.TOL, rel_tol=synth.REL_TOL, max_iter=synth.MAX_ITER,
                       precond=precond, precision=precision)
    mesh = L.Mesh(p.mesh, gradient=skew, non_orthogonal=skew)
    prob = L.Problem(mesh, p.bcs, p.DT, p.dt, opts)
    T0 = torch.from_numpy(p.T0).cuda()
    prob.set_T(T0)
    if warmup > 0:
        prob.step(warmup)
    prob.set_T(T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, _ = prob.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    iters = sum(s["n_iter"] for s in stats)
    out = {"n_cells": N, "steps": steps, "precond": pc_name, "precision": p.precision,
           "layout": "bands" if prob.layout() == L.LF_LAYOUT_BANDS else "rows",
           "ms_per_step": wall * 1e3 / steps, "iters_per_step_mean": iters / steps,
           "cell_iters_per_s": N * iters / wall, "us_per_iteration": wall * 1e6 / max(iters, 1),
           "all_converged": all(s["converged"] == 1 for s in stats)}
    if skew:
        out["mesh"] = "skewed (non-orthogonal correction every step)"
    prob.close()
    mesh.close()
    log(f"[bench] {name}: {out['ms_per_step']:.3f} ms/step, {out['iters_per_step_mean']:.1f} iterations")
    return out


PAPER_SIDES = (100, 200, 300, 400)     # the four box meshes of the paper's evaluation
PAPER_DT, PAPER_STEPS, PAPER_DIFFUSIVITY = 0.2, 500, 1e-4


# steps per side in the default run: the two small boxes in full, the two
# large ones bounded (their per-step figures scale to the 500 steps)
PAPER_BOUNDED_STEPS = {100: 500, 200: 500, 300: 100, 400: 40}


def run_paper_sweep(L, torch, sides=PAPER_SIDES, steps=PAPER_STEPS, preconds=("diagonal",)):
    """The paper's evaluation shapes: uniform unit boxes of n^3 cells, 500 time
    steps of 0.2 s (100 s simulated), PCG with the diagonal preconditioner, FP64.
    The diffusivity is not given there: 1e-4 m^2/s.  Boundary conditions and
    T0 as the other configs.  Assembly and solver time are the library's own
    per-step event timings, summed; total is the wall clock of the steps.
    steps: an int for every side, or a dict side -> steps; a run shorter than
    500 steps also reports the per-step times scaled to 500.  Each side runs
    once per preconditioner in `preconds` ("diagonal", "amg") on the same
    device mesh."""
    import synth
    out = []
    for n in sides:
        n_steps = steps[n] if isinstance(steps, dict) else steps
        t = time.perf_counter()
        mesh_h = synth.box_mesh(n, n, n)
        T0 = synth.initial_field(mesh_h.n_cells, 20250724)
        gen = time.perf_counter() - t
        mesh = L.Mesh(mesh_h)
        N, F = mesh_h.n_cells, mesh_h.n_faces
        del mesh_h
        T0d = torch.from_numpy(T0).cuda()
        for pc in preconds:
            opts = L.make_opts(tol=synth.TOL, rel_tol=synth.REL_TOL, max_iter=synth.MAX_ITER,
                               precond=L.LF_PC_AMG if pc == "amg" else L.LF_PC_DIAGONAL)
            prob = L.Problem(mesh, synth.fixed_x_bcs(), PAPER_DIFFUSIVITY, PAPER_DT, opts)
            prob.set_T(T0d)
            prob.step(2)                      # warm-up (graph capture, first launches)
            prob.set_T(T0d)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            stats, _ = prob.step(n_steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            rec = {"side": n, "precond": pc, "n_cells": N, "n_faces": F, "steps": n_steps, "dt": PAPER_DT,
                   "DT": PAPER_DIFFUSIVITY, "assembly_s": sum(x["assemble_ms"] for x in stats) / 1e3,
                   "solver_s": sum(x["solve_ms"] for x in stats) / 1e3, "total_s": wall,
                   "ms_per_step": wall * 1e3 / n_steps,
                   "iters_per_step_mean": sum(x["n_iter"] for x in stats) / n_steps,
                   "cell_iters_per_s": N * sum(x["n_iter"] for x in stats) / wall,
                   "all_converged": all(x["converged"] == 1 for x in stats), "mesh_generation_s": gen}
            if n_steps != PAPER_STEPS:
                k = PAPER_STEPS / n_steps
                rec["scaled_to_500_steps"] = {"assembly_s": rec["assembly_s"] * k,
                                              "solver_s": rec["solver_s"] * k, "total_s": wall * k}
            log(f"[bench] paper shape {n}^3, {pc}: {wall:.2f} s for {n_steps} steps, "
                f"{rec['iters_per_step_mean']:.1f} iterations per step")
            out.append(rec)
            prob.close()
        mesh.close()
        del T0d
        torch.cuda.empty_cache()
    return out


def grad_bytes(n_cells, n_faces, n_bfaces, n_bands=0, reordered=False, boundary_gradient=True):
    """Algorithmic bytes of one Gauss-gradient call.  Both paths: per cell T,
    V, the gradient (3 doubles) and the boundary-list start; per boundary face
    its list entry, T_b and its 32-byte record, and with boundary_gradient
    also snGrad_b and the boundary gradient (3 doubles).  Band path: one
    32-byte record per band slot (n_bands per cell).  Row path: the row length
    per cell and, per internal face, on each of its two rows a 32-byte record
    and a column index; a mesh kept in Morton order adds the field's copy into
    that order (label, read, write) and the label of each row's mesh cell (the
    gradient's round trip through a scratch array in the solver's order, 48 B
    per cell, is not counted)."""
    per_bface = 76 if boundary_gradient else 44
    if n_bands:
        return 44 * n_cells + 32 * n_bands * n_cells + per_bface * n_bfaces
    return 45 * n_cells + 72 * n_faces + per_bface * n_bfaces + (24 * n_cells if reordered else 0)


def run_grad(L, torch, p, label, launches=20):
    """The Gauss gradient on the config's box, skewed (non-orthogonal faces)."""
    import numpy as np
    import synth
    host = synth.affine(p.mesh, synth.SKEW)
    m = L.Mesh(host, gradient=True, non_orthogonal=True)
    reordered = bool(m.cell_order()[0])
    N, F, B = host.n_cells, host.n_faces, host.n_bfaces
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    T = dev(synth.initial_field(N, 61))
    Tb = dev(synth.initial_field(B, 62))
    snb = dev(400.0 * (synth.uniform01(63, B) - 0.5))
    del host
    g = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    bg = torch.empty((B, 3), dtype=torch.float64, device="cuda")
    for _ in range(3):
        L.lf_grad(m.h, T.data_ptr(), Tb.data_ptr(), snb.data_ptr(), g.data_ptr(), bg.data_ptr())
    torch.cuda.synchronize()
    # the mesh's stream is torch's current stream, so these events bracket the launches
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(launches):
        L.lf_grad(m.h, T.data_ptr(), Tb.data_ptr(), snb.data_ptr(), g.data_ptr(), bg.data_ptr())
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / launches
    K = m.n_bands
    # the same kernel as the corrected time step runs it: T and the gradient
    # in the solver's order, no boundary gradient (3 steps with per-kernel
    # timing; the step's other kernels are timed too)
    prob = L.Problem(m, p.bcs, p.DT, p.dt)
    prob.set_T(torch.from_numpy(p.T0).cuda())
    prob.step(1)
    prob.profile(True)
    prob.step(3)
    torch.cuda.synchronize()
    prof = prob.profile_read()
    prob.profile(False)
    prob.close()
    m.close()
    in_step = None
    if "grad" in prof:
        ms, cnt = prof["grad"]
        us_s = 1e3 * ms / cnt
        b_s = grad_bytes(N, F, B, K, False, boundary_gradient=False)
        g_s = b_s / (us_s * 1e-6) / 1e9
        in_step = {"kernel": (f"k_grad_band<{K}>" if K else "k_grad_rows") + " in the corrected step (solver order)",
                   "launches": cnt, "avg_us": us_s, "algorithmic_bytes": b_s, "achieved_GBps": g_s,
                   "frac": g_s / HBM_PEAK_GBS}
        if "nonorth" in prof:
            ms, cnt = prof["nonorth"]
            in_step["correction_divergence_avg_us"] = 1e3 * ms / cnt
    nbytes = grad_bytes(N, F, B, K, reordered)
    gbps = nbytes / (us * 1e-6) / 1e9
    kname = f"k_grad_band<{K}>" if K else "k_grad_rows"
    traffic = None
    tfile = GRAD_TRAFFIC_FILE if K else GRAD_ROWS_TRAFFIC_FILE
    if os.path.exists(tfile):
        with open(tfile) as f:
            tr = json.load(f)
        # counters taken on this kernel source and size only
        if (tr.get("source_sha256") == kernel_source_hash(GRAD_SOURCES) and tr.get("n_cells") == N
                and tr.get("kernel") == kname):
            traffic = tr["hbm_bytes_per_launch"]
    return {"workload": f"Gauss gradient, {label}",
            "kernel": kname, "launches": launches, "avg_us": us,
            "algorithmic_bytes": nbytes, "achieved_GBps": gbps, "peak_GBps": HBM_PEAK_GBS,
            "frac": gbps / HBM_PEAK_GBS, "traffic": traffic,
            "roofline": {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbps / HBM_PEAK_GBS, "traffic": traffic},
            "in_step": in_step}


def run_serving(L, torch, args):
    """512 parametric requests (side log-uniform in [16, 96], DT log-uniform in
    [1e-4, 1e-2], dt = 1e-3, 10 steps, snapshots of every step returned):
    first all arriving at once (saturated throughput), then Poisson arrivals
    at fractions of that rate.  Meshes are resident before the clock starts."""
    import synth
    from paper_2507_18268_amd import serve as S
    from paper_2507_18268_amd import autotune
    base = synth.request_stream(args.serve_requests, rate=1.0)
    host_meshes = {}

    def mesh_for_side(n):
        if n not in host_meshes:
            host_meshes[n] = synth.box_mesh(n, n, n)
        return host_meshes[n]

    def requests(rate):
        rs = synth.request_stream(args.serve_requests, rate=rate) if rate else base
        return [S.Request(rid=r.rid, n=r.n, DT=r.DT, dt=r.dt, steps=r.steps,
                          T0=synth.initial_field(r.n ** 3, r.seed), bcs=synth.fixed_x_bcs(),
                          arrival=(r.arrival if rate else 0.0)) for r in rs]

    tuning = autotune.load()
    lane = autotune.serving_params()
    tuned_lane = (autotune.load(form="serving") is not None and args.serve_direct_min < 0
                  and args.serve_group_iters < 0)
    if args.serve_direct_min < 0:
        args.serve_direct_min = lane["direct_min_side"]
    if args.serve_group_iters < 0:
        args.serve_group_iters = lane["group_iters"]
    out = {"workload": f"{args.serve_requests} requests, side log-uniform [16,96], DT log-uniform "
                       f"[1e-4,1e-2], dt 1e-3, 10 steps, snapshots returned, mixed FP32/FP64: "
                       f"batched kernel, large sides on the multi-kernel solver",
           "tuning": tuning["block_threads"] if tuning else None,
           "budget_GiB": args.serve_budget_gib, "slots": args.serve_slots,
           "direct_min_side": args.serve_direct_min or None, "direct_workers": args.serve_direct_workers,
           "direct_lane": "alone (lf_step_begin)" if args.serve_direct_alone else "group (lf_group)",
           "group_iters": args.serve_group_iters,
           "lane_source": "autotuned" if tuned_lane else "default"}
    sides = sorted({r.n for r in base})
    cells = sum(r.n ** 3 for r in base)

    # one long-running server for all legs (meshes resident, problem pools
    # warmed by the first leg), as a deployment would run it
    srv = S.Server(mesh_for_side, int(args.serve_budget_gib * 2 ** 30), n_slots=args.serve_slots,
                   slot_capacity=args.serve_capacity, max_steps=10, tuning=tuning,
                   direct_min_side=args.serve_direct_min or None,
                   direct_workers=args.serve_direct_workers,
                   direct_use_graph=not args.serve_direct_no_graph,
                   direct_group=not args.serve_direct_alone, group_iters=args.serve_group_iters,
                   direct_streams=args.serve_direct_streams)
    for n in sides:
        srv.preload_mesh(n)
    torch.cuda.synchronize()

    def one(rate, label):
        reqs = requests(rate)
        n_rej = len(srv.rejected)
        done = srv.run(reqs, poll_s=0.0,
                       progress=lambda k, t: log(f"[bench] serving {label}: {k}/{t} requests done"))
        summ = S.summarize(done)
        summ["rejected"] = len(srv.rejected) - n_rej
        summ["all_converged"] = all(all(s["converged"] == 1 for s in r.stats) for r in done)
        log(f"[bench] serving {label}: {summ.get('solves_per_s', 0):.1f} solves/s, "
            f"p50 {summ.get('p50_latency_s', 0) * 1e3:.1f} ms, p99 {summ.get('p99_latency_s', 0) * 1e3:.1f} ms")
        return summ

    one(None, "warm-up")
    sat = one(None, "saturated")
    sat["cell_steps_per_s"] = cells * 10 * sat["solves_per_s"] / len(base)
    out["saturated"] = sat
    rate_sat = sat["solves_per_s"]
    fracs = [0.5] if args.serve_quick else [0.25, 0.5, 1.0, 2.0, 4.0]
    out["poisson"] = []
    for f in fracs:
        summ = one(f * rate_sat, f"poisson {f}x")
        summ["offered_rate"] = f * rate_sat
        summ["fraction_of_saturated"] = f
        out["poisson"].append(summ)
    srv.close()
    if args.serve_small_budget_gib > 0:
        # a deliberately small HBM budget: meshes no longer all fit, so the
        # server evicts idle problems and meshes and rebuilds them on demand
        small = S.Server(mesh_for_side, int(args.serve_small_budget_gib * 2 ** 30),
                         n_slots=args.serve_slots, slot_capacity=args.serve_capacity, max_steps=10,
                         tuning=tuning, direct_min_side=args.serve_direct_min or None,
                         direct_workers=args.serve_direct_workers,
                         direct_use_graph=not args.serve_direct_no_graph,
                         direct_group=not args.serve_direct_alone, group_iters=args.serve_group_iters,
                   direct_streams=args.serve_direct_streams)
        srv = small
        summ = one(None, f"saturated, budget {args.serve_small_budget_gib} GiB")
        summ["budget_GiB"] = args.serve_small_budget_gib
        summ["mesh_builds"] = small.mesh_builds
        summ["evictions"] = small.evictions
        out["small_budget"] = summ
        small.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="graded_256")
    ap.add_argument("--n", type=int, default=None, help="override the cube side (testing only)")
    ap.add_argument("--precond", choices=["config", "diagonal", "dic", "amg"], default="config",
                    help="the main leg's preconditioner (default: the config's; for profiling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-roofline-pass", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--accuracy-steps", type=int, default=20)
    ap.add_argument("--inner-tol", type=float, default=0.0, help="mixed: inner reduction (0 = default)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--grad-only", action="store_true",
                    help="only the Gauss-gradient leg (for profiling it alone)")
    ap.add_argument("--paper-sweep", action="store_true",
                    help="the paper's four box sizes, 500 steps of 0.2 s each (about a minute)")
    ap.add_argument("--skewed-only", action="store_true",
                    help="only the config's box skewed, --steps corrected time steps (for profiling)")
    ap.add_argument("--no-extra-configs", action="store_true")
    ap.add_argument("--no-paper-shapes", action="store_true",
                    help="skip the bounded run of the paper's four box sizes")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--serve-quick", action="store_true",
                    help="one Poisson rate (0.5x of saturated) instead of 0.25x..4x")
    ap.add_argument("--serve-small-budget-gib", type=float, default=1.0,
                    help="also serve the stream under this HBM budget (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-capacity", type=int, default=64)
    ap.add_argument("--serve-direct-min", type=int, default=-1,
                    help="requests with at least this cube side run on the multi-kernel solver "
                         "(0 = never, -1 = the autotuned threshold)")
    ap.add_argument("--serve-direct-workers", type=int, default=32)
    ap.add_argument("--serve-direct-no-graph", action="store_true")
    ap.add_argument("--serve-direct-alone", action="store_true",
                    help="direct lane without the group: each request alone (lf_step_begin/poll)")
    ap.add_argument("--serve-direct-streams", type=int, default=4,
                    help="streams of the grouped direct lane's own work (assembly, pass turns)")
    ap.add_argument("--serve-group-iters", type=int, default=-1,
                    help="inner iterations per group block (0: the library default, -1: autotuned)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = 64 << 20                      # 64 Mi doubles = 512 MiB each way
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "launches": 5}))
        return

    import synth
    from paper_2507_18268_amd import lapfoam as L

    if args.serve_only:
        print(json.dumps({"serving": run_serving(L, torch, args)}), flush=True)
        return
    if args.paper_sweep:
        print(json.dumps({"paper_sweep": run_paper_sweep(L, torch, preconds=("diagonal", "amg"))}), flush=True)
        return

    t = time.perf_counter()
    p = synth.build_config(args.config, n=args.n)
    N, F = p.mesh.n_cells, p.mesh.n_faces
    log(f"[bench] {args.config}: {N} cells, {F} faces, mesh generated in {time.perf_counter() - t:.1f} s")
    if args.grad_only:
        print(json.dumps({"grad": run_grad(L, torch, p, GRAD_LABEL)}), flush=True)
        return
    if args.skewed_only:
        print(json.dumps({"skewed": run_config_leg(L, torch, args.config, args.steps, skew=True)}), flush=True)
        return
    pc_name = p.precond if args.precond == "config" else args.precond
    precond = {"dic": L.LF_PC_DIC, "amg": L.LF_PC_AMG}.get(pc_name, L.LF_PC_DIAGONAL)
    precision = L.LF_PREC_MIXED if p.precision == "mixed" else L.LF_PREC_FP64
    opts = L.make_opts(tol=synth.TOL, rel_tol=synth.REL_TOL, max_iter=synth.MAX_ITER,
                       precond=precond, precision=precision)
    t = time.perf_counter()
    mesh = L.Mesh(p.mesh)
    prob = L.Problem(mesh, p.bcs, p.DT, p.dt, opts)
    T0 = torch.from_numpy(p.T0).cuda()
    torch.cuda.synchronize()
    layout_name = "bands" if prob.layout() == L.LF_LAYOUT_BANDS else "rows"
    walk = prob.amul_form()
    amul_form = {0: "one row per thread", 1: "row walk", 2: "block walk of the box",
                 3: "two red-black pairs per lane",
                 4: "block walk of the box (solve on the Jacobi-scaled matrix)"}[walk]
    log(f"[bench] device mesh + problem ready in {time.perf_counter() - t:.1f} s "
        f"(workspaces {mesh.ws_bytes / 2**30:.2f} + {prob.ws_bytes / 2**30:.2f} GiB, {layout_name} layout{', Amul by the ' + amul_form if walk else ''})")

    prob.set_T(T0)
    if args.warmup > 0:
        prob.step(args.warmup)
    prob.set_T(T0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, _ = prob.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} steps in {wall:.3f} s")

    iters = [s["n_iter"] for s in stats]
    total_iters = sum(iters)
    value = N * total_iters / wall
    solve_s = sum(s["solve_ms"] for s in stats) / 1e3
    step_ms = [s["assemble_ms"] + s["solve_ms"] for s in stats]
    ok = all(s["converged"] == 1 for s in stats)

    out = {
        "metric": METRIC, "value": value, "unit": "cell-PCG-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision == L.LF_PREC_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {round(N ** (1 / 3))}^3 box, z expansion ratio "
                               f"{synth.CONFIGS[args.config]['z_ratio']}, DT={p.DT}, dt={p.dt}, "
                               f"implicit Euler, PCG {pc_name}, tol {synth.TOL}",
                   "n_cells": N, "n_faces": F, "precision": p.precision, "layout": layout_name,
                   "amul": amul_form},
        "iters_per_step_mean": total_iters / len(stats),
        "solver_only_cell_iters_per_s": N * total_iters / solve_s if solve_s > 0 else None,
        "assemble_ms_mean": sum(s["assemble_ms"] for s in stats) / len(stats),
        "p50_step_ms": percentile(step_ms, 50), "p99_step_ms": percentile(step_ms, 99),
        "all_converged": ok,
    }

    if not args.no_roofline_pass:
        prob.set_T(T0)
        prob.profile(True)
        prob.step(args.steps)
        torch.cuda.synchronize()
        prof = prob.profile_read()
        prob.profile(False)
        kernels = {k: {"avg_us": 1e3 * ms / n, "launches": n} for k, (ms, n) in prof.items()}
        out["kernel_avg_us"] = kernels
        dom = max(prof, key=lambda k: prof[k][0])
        ka = kernels["amul_dot"]
        us = ka["avg_us"]
        # algorithmic bytes of the product as it runs: the band layout's
        # neighbours are implicit (c + d_k), so no face addresses
        unit = walk == 4
        per_launch = amul_bytes(N, F, addressed=(layout_name != "bands"), unit_diag=unit)
        achieved = per_launch / (us * 1e-6) / 1e9
        kname = {0: "k_amul_dot", 1: "k_amul_dot_walk", 2: "k_amul_dot_box", 3: "k_amul_dot_rb2",
                 4: "k_amul_dot_box_scaled"}[walk]
        what = "q~ = (S A S) p~" if unit else "q = A p"
        roof = {"kernel": f"{kname} ({what} with p.q partials)", "bound": "hbm",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes_per_launch": per_launch,
                "algorithmic_bytes": ("16 B/cell (p, q; unit diagonal)" if unit else "24 B/cell (p, diag, q)")
                                     + " + 8 B/face (coefficient)"
                                     + ("" if layout_name == "bands" else " + 8 B/face (two int32 addresses)"),
                "avg_launch_us": us, "largest_total_time_kernel": dom}
        face_addr = amul_bytes(N, F, addressed=True, unit_diag=unit)
        roof["face_addressed_bytes_per_launch"] = face_addr
        roof["face_addressed_frac"] = face_addr / (us * 1e-6) / 1e9 / HBM_PEAK_GBS
        lb = layout_bytes(p.mesh, layout_name, unit_diag=unit)
        roof["layout"] = layout_name
        roof["layout_bytes_per_launch"] = lb
        roof["layout_GBps"] = lb / (us * 1e-6) / 1e9
        roof["layout_frac"] = roof["layout_GBps"] / HBM_PEAK_GBS
        if os.path.exists(TRAFFIC_FILE):
            with open(TRAFFIC_FILE) as f:
                tr = json.load(f)
            if (tr.get("source_sha256") == kernel_source_hash() and tr.get("n_cells") == N
                    and tr.get("kernel") == kname):
                roof["traffic"] = tr["hbm_bytes_per_launch"]
                roof["traffic_GBps"] = roof["traffic"] / (us * 1e-6) / 1e9
                roof["traffic_frac"] = roof["traffic_GBps"] / HBM_PEAK_GBS
        out["roofline"] = roof
        # whole-iteration view: the three kernels of one PCG iteration
        it_us = sum(kernels[k]["avg_us"] for k in ("amul_dot", "update", "direction") if k in kernels)
        out["pcg_iteration_us"] = it_us

    if not args.no_mixed and precision == L.LF_PREC_FP64 and precond == L.LF_PC_DIAGONAL:
        out["mixed"] = run_mixed(L, torch, p, mesh, prob, T0, args)
        out["mixed"]["speedup_vs_fp64_time_to_tol"] = out["ms_per_step"] / out["mixed"]["ms_per_step"]

    if not args.no_extra_configs:
        # the other configs of the workload family (parity cases elsewhere),
        # timed the same way: 32^3 (launch-latency bound), 192^3 permuted (row
        # layout, random-neighbour gathers), 256^3 red-black DIC
        out["other_configs"] = {name: run_config_leg(L, torch, name, steps)
                                for name, steps in (("plain_32", 20), ("permuted_192", 30),
                                                    ("graded_256_dic", 50))}
        # the same 256^3 box skewed: the corrected Laplacian (gradient, correction
        # fluxes and their divergence before each assembly)
        out["other_configs"]["graded_256_skewed"] = run_config_leg(L, torch, "graded_256", 50, skew=True)
        # the same box with the aggregation multigrid preconditioner
        out["other_configs"]["graded_256_amg"] = run_config_leg(L, torch, "graded_256", 50, precond="amg")

    if not args.no_grad and args.n is None:
        log("[bench] Gauss gradient ...")
        out["grad"] = run_grad(L, torch, p, GRAD_LABEL)
        if not args.no_extra_configs:
            # the row path: the randomly numbered 192^3 box, skewed (kept in Morton order)
            out["grad_rows"] = run_grad(L, torch, synth.build_config("permuted_192"),
                                        "192^3 box graded in z, randomly numbered and skewed")

    if not args.no_serve:
        out["serving"] = run_serving(L, torch, args)

    if not args.no_paper_shapes and args.n is None:
        # the paper's evaluation boxes (100^3 .. 400^3, dt 0.2 s), bounded steps
        out["paper_shapes"] = {
            "workload": "uniform unit boxes 100^3, 200^3, 300^3, 400^3 (the paper's Mesh-S..XL), "
                        f"DT={PAPER_DIFFUSIVITY}, dt={PAPER_DT}, implicit Euler, PCG diagonal, "
                        f"tol {synth.TOL}, FP64; steps per side {PAPER_BOUNDED_STEPS}",
            "runs": run_paper_sweep(L, torch, steps=PAPER_BOUNDED_STEPS, preconds=("diagonal", "amg"))}

    if not args.no_cpu_baseline:
        log("[bench] oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_budget)

    prob.close()
    mesh.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
