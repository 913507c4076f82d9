#!/usr/bin/env python3
"""Benchmark: staggered phase-field fracture on one MI355X.

Metric: time per load step / load history and GDOF-updates/s of the
fixed-stress S1 scheme in mixed precision (FP32 inner CG, FP64 outer loops),
against the plain FP64 standard scheme on the same GPU.

Workload (default): 512 x 512 Q1 single-edge-notched tension panel (unit
square, notch y = 0.5, x <= 0.5 as Dirichlet d = 1), E = 210 GPa, nu = 0.3,
Gc = 2.7 N/mm, l = 0.004 mm, eta = 1e-6, volumetric-deviatoric split, top
edge u_y ramped by 6e-5 mm per step.  A "step" is one load step of that
history: the staggered iterations until ||R_d||/||b|| <= 1e-5, each with the
QP update, the S1 trial solve and predictor, the phase solve, the Newton
displacement solve (PCG with fused reductions) and the reaction force.
Both schemes use Jacobi-Chebyshev preconditioning (degree 3 for the FP32
inner solves, 5 for FP64), start their displacement solves from the
projection onto the last four solutions (--guess-vectors), and use the work
decomposition measured fastest for each on this mesh: LDS tiles for S1
mixed, column marching with 2 rows for ST FP64 (--tune-reps N lets the
autotuner choose instead).
The timed window ends in load step 91, the step in which the crack runs
through the ligament (the longest steps of the history, where the schemes
differ most): load steps 1..91-K-W run first with S1 mixed, untimed, and
both schemes start from that committed state; W warmup steps follow
untimed, then K load steps are timed (--window-end moves the window,
--full-history times all 100 steps from the initial state).  Each scheme
stops a step at max_stag = 500 staggered iterations; the line lists the
steps that ended there and gives the speedup over the whole window and over
the steps both schemes converged.

value = GDOF-updates/s of S1 mixed over the timed steps (sum over all CG
solves of free DOFs x iterations, divided by the wall time between two
device synchronisations).  Inputs are resident in HBM before timing.

Two further modes print their own single JSON line:
  --workload sweep64     the seeded 64-instance tension sweep (mesh sizes
                         128..512, Gc, l and notch drawn per instance), S1
                         mixed, column marching with 4 rows per wave (one
                         shared launch per operator kind): load steps W+1..W+K
                         of every instance, batched with shared CG launches
                         (value), batched on concurrent streams, and one by
                         one;
  --workload apply-sizes the FP32 fused tangent apply and the CG vector
                         update at 512^2 .. 4096^2 (one displacement solve of
                         a notched panel, CG capped), against the HBM peak;
  --workload trial-readings  ST and S1/S3 under the four readings of the
                         trial solve (floored or unfloored block, predict ->
                         correct or trial-only), FP64, over the whole load
                         history of --trial-problem (64^2 by default):
                         staggered counts, convergence and force curves;
  --workload slab3d      the 3-D load step (pf3d_load_step, FP64, Jacobi PCG)
                         on the 64^2 tension panel extruded into a slab of
                         two element layers, S1 and ST over --steps load
                         steps after --warmup: time per step, GDOF-updates/s
                         and staggered counts;
  --workload apply3d     the 3-D operators (node-gather kernels, FP64) on
                         cubes of 32^3..96^3 elements: time per launch and
                         algorithmic GB/s of the internal force, tangent
                         apply and phase apply;
  --workload oracle-history  the CPU baseline over a whole load history: the
                         oracle (FP64, direct solves) on the 64^2
                         configuration for ST and S1, with the cap of
                         --max-stag (no GPU needed), for comparison with the
                         GPU times of trial-readings on the same history.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time per load history and GDOF-updates/s, S1 mixed vs std FP64, 1 MI355X"
GUESS_VECTORS = 0   # --guess-vectors: starting guesses of the displacement solves (timed runs)
KIND = {"tension512": "notched tension panel", "tension64": "notched tension panel",
        "shear1024": "notched shear panel (spectral split)",
        "lshape2048": "L-shaped panel (masked quadrant)"}
HBM_PEAK_GBS = 8000.0
# The load step of the 512^2 tension history in which the crack runs through
# the ligament (both schemes; the longest steps of the history).
NUCLEATION_STEP_512 = 91


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fused_apply_bytes_per_node():
    """Algorithmic bytes per node of the FP32 fused elasticity CG apply
    (k_cg_apply, used by the FP32 inner solves): read z (2 comps), p_old (2),
    d (1), node flag (1 B), element flag (1 B per element ~ node); write
    p_new (2), q (2)."""
    return (2 + 2 + 1 + 2 + 2) * 4 + 1 + 1


def cheb_step_bytes_per_node():
    """Algorithmic bytes per node of an FP32 Jacobi-Chebyshev step on the
    tangent (k_march<OpCheb<OpTangent<float>>>, not the last step): read
    d_{k-1}, z, res, D^-1 (2 comps each), d, node flag, element flag (1 B per
    element ~ node); write d_k, z, res (2 comps each)."""
    return (2 + 2 + 2 + 2 + 1 + 2 + 2 + 2) * 4 + 1 + 1


def updcheb_bytes_per_node():
    """Algorithmic bytes per node of the FP32 CG update fused with the first
    Chebyshev step on the tangent (k_cg_updcheb<OpUpdCheb<OpTangent<float>>>):
    read r, q, D^-1, x, p (2 comps each), d, node flag, element flag; write
    x, r, d_1, z, res (2 comps each)."""
    return (2 * 5 + 1 + 2 * 5) * 4 + 1 + 1


def updcheb2_bytes_per_node(last=True):
    """Algorithmic bytes per node of the FP32 CG update fused with the first
    two Chebyshev steps on the tangent (k_cg_updcheb2<OpTangent<float>>, LDS
    tiles): read r, q, D^-1, x, p (2 comps each), d, node flag, element flag;
    write x, r, z (2 comps each) and, when more steps follow, d_2 and res_2."""
    return (2 * 5 + 1 + 2 * (3 if last else 5)) * 4 + 1 + 1


def update_bytes_per_node():
    """Algorithmic bytes per node of the FP32 CG vector update (k_cg_update):
    per DOF read x, p, q, r, D^-1 and write x, r, z, two DOFs per node."""
    return 2 * (5 + 3) * 4


def measured_traffic(kname):
    """Per-launch HBM bytes of the dominant kernel from the committed counter
    runs (profiles/hbm_traffic_tension512.json) and a note naming that
    source, or (None, None) when the kernel source has changed since the
    counters were taken or they were taken on another kernel."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_tension512.json")
    src = os.path.join(ROOT, "paper_2209_07969_amd", "csrc", "pf_kernels.hip")
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernel_source_sha256") != sha or rec.get("kernel") != kname:
        return None, None
    return rec["traffic_bytes_per_launch"], (
        f"profiles/hbm_traffic_tension512.json: rocprofv3 FETCH_SIZE and WRITE_SIZE runs of "
        f"this kernel, taken on pf_kernels.hip sha256 {sha[:16]} (the source built here)")


def load_step_logged(ctx, problem, lam, every=25):
    """One load step driven through pf_staggered_iterate / pf_commit_step
    (the loop pf_load_step runs), printing a progress line every `every`
    staggered iterations so that long crack-propagation steps report."""
    t0 = time.perf_counter()
    st = ctx.staggered_iterate(lam)
    while st["r_stag"] > problem.tol_stag and st["n_stag"] < ctx.opts.max_stag:
        st = ctx.staggered_iterate(lam)
        if st["n_stag"] % every == 0:
            log(f"    ... {st['n_stag']} staggered iterations, r_stag={st['r_stag']:.2e}")
    ctx.commit_step()
    st["force"] = list(ctx.reaction_force(problem.load_group))
    st["converged"] = int(st["r_stag"] <= problem.tol_stag)
    st["time_ms"] = (time.perf_counter() - t0) * 1e3
    return st


STEP_FIELDS = ("n_stag", "n_newton", "n_trial", "n_dsolve", "n_cg_u", "n_cg_d", "n_cg_trial",
               "gated_max", "floor_hits", "r_stag", "force", "time_ms", "time_u_ms",
               "time_d_ms", "dof_updates", "converged", "cg_not_converged")


def step_record(label, step, timed, st):
    """One JSON-lines record of a load step's statistics."""
    rec = {"run": label, "step": step, "timed": timed}
    for k in STEP_FIELDS:
        v = st.get(k)
        rec[k] = list(v) if isinstance(v, (tuple, list)) else v
    return json.dumps(rec)


def run_steps(pf, problem, scheme, precision, warmup, steps, profile=False, degree=None,
              tune_reps=0, rows=0, jsonl=None, label="", start=0, state=None):
    """Run load steps start+1..start+warmup untimed and the next `steps`
    timed.  state: (u, d, H) committed after load step `start` (None: the
    initial state, start = 0).  degree: Jacobi-Chebyshev degree (None = plain
    Jacobi); rows: work decomposition (march_rows); tune_reps > 0: let the
    autotuner pick it; jsonl: an open file that receives one record per load
    step."""
    import torch
    opts = {} if degree is None else {"precond": 1, "cheb_degree": degree}
    if GUESS_VECTORS:
        opts["guess_vectors"] = GUESS_VECTORS
    ctx = pf.Context(problem, scheme=scheme, precision=precision, march_rows=rows, **opts)
    if state is not None:
        ctx.set_state(*state)
    ctx.chosen_rows = ctx.autotune(tune_reps) if tune_reps > 0 else rows
    if profile:
        ctx.set_profiling(True)
    for n in range(start, start + warmup):
        st = load_step_logged(ctx, problem, float(problem.loads[n]))
        if jsonl:
            jsonl.write(step_record(label, n + 1, False, st) + "\n")
        log(f"  warmup step {n+1}: n_stag={st['n_stag']} cg_u={st['n_cg_u']} "
            f"cg_d={st['n_cg_d']} cg_trial={st['n_cg_trial']} {st['time_ms']:.0f} ms")
    if profile:
        ctx.set_profiling(True)     # reset counters: only timed steps count
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rows = []
    for n in range(start + warmup, start + warmup + steps):
        st = load_step_logged(ctx, problem, float(problem.loads[n]))
        st["step"] = n + 1
        rows.append(st)
        if jsonl:
            jsonl.write(step_record(label, n + 1, True, st) + "\n")
            jsonl.flush()
        log(f"  timed step {n+1}: n_stag={st['n_stag']} conv={st['converged']} "
            f"newton={st['n_newton']} cg_u={st['n_cg_u']} cg_d={st['n_cg_d']} "
            f"cg_trial={st['n_cg_trial']} gated={st['gated_max']} F={st['force'][1]:.4f} "
            f"{st['time_ms']:.0f} ms (u {st['time_u_ms']:.0f}, d {st['time_d_ms']:.0f})")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return ctx, rows, t1 - t0


def prefix_state(pf, problem, n_steps, degree, rows):
    """The committed state after load steps 1..n_steps of S1 mixed: the
    common starting point of both timed runs (input preparation, untimed)."""
    if n_steps <= 0:
        return None
    opts = {} if degree is None else {"precond": 1, "cheb_degree": degree}
    ctx = pf.Context(problem, scheme=pf.S1, precision=pf.MIXED, march_rows=rows, **opts)
    t0 = time.perf_counter()
    for n in range(n_steps):
        st = ctx.load_step(float(problem.loads[n]))
        if (n + 1) % 10 == 0 or n + 1 == n_steps:
            log(f"  prefix step {n + 1}: n_stag={st['n_stag']} F={st['force'][1]:.4f} "
                f"({time.perf_counter() - t0:.1f} s)")
    state = ctx.get_state()
    ctx.close()
    return state


def step_table(rows):
    """Per-step record of a timed run for the JSON line."""
    return [{"step": r["step"], "n_stag": r["n_stag"], "converged": int(r["converged"]),
             "n_newton": r["n_newton"], "n_cg_u": r["n_cg_u"], "n_cg_d": r["n_cg_d"],
             "n_cg_trial": r["n_cg_trial"], "time_ms": round(r["time_ms"], 1),
             "time_u_ms": round(r["time_u_ms"], 1), "time_d_ms": round(r["time_d_ms"], 1)}
            for r in rows]


def copy_bandwidth():
    """Measured device-to-device copy rate (GB/s, bytes read + written) of a
    1 GiB buffer: the GPU's practical HBM ceiling beside the 8 TB/s peak."""
    import torch
    n = 256 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2 * 4 * n / sec / 1e9


def cpu_baseline(pf, problem, st_steps=None):
    """The oracle (FP64, assembled CSR + SuperLU), untuned, on a bounded
    sample of the workload: the k = 0 displacement solve of load step 1
    limited to one Newton iteration (assemble R_u and K_t, one sparse direct
    solve, the line-search residual), then the QP update and the staggered
    residual.  value: its wall time in seconds.  The GPU runs the same sample
    (ST FP64, one Newton iteration: pf_staggered_iterate opening step 1) in a
    second fresh context after a first one has warmed the library up; its
    time is reported beside the oracle's.  cores: the process's CPU time over
    the oracle's wall time (all threads, so a multithreaded library call
    would show), rounded, at least 1.  After the sample, one phase solve
    (assembled K_dd(H), SuperLU) is timed on its own; with st_steps (the ST
    FP64 run's per-step records) the line adds an estimate of the oracle's
    time for that run's window: Newton iterations x the sample time plus
    staggered iterations x the phase-solve time."""
    import dataclasses

    import numpy as np
    import torch

    import oracle
    p1 = dataclasses.replace(problem, max_newton=1)
    lam = float(p1.loads[0])
    for rep in range(2):
        ctx = pf.Context(p1, scheme=pf.ST, precision=pf.FP64, max_newton=1)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        ctx.staggered_iterate(lam)
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - tg
        ctx.close()
    orc = oracle.Oracle(p1, 0)
    t0, c0 = time.perf_counter(), time.process_time()
    u = orc.u.copy()
    u[orc.u_fixed] = lam * orc.u_unit[orc.u_fixed]
    R0 = np.linalg.norm(orc.residual_u(u, orc.d)[orc.u_free])
    u, nit, _ = orc.newton(u, orc.d, R0 if R0 > 0 else 1.0)
    parts = orc.energies(u, orc.d)
    H = np.maximum(orc.H, parts["psi_plus"])
    orc.stag_residual(orc.d, H)
    t, cpu_s = time.perf_counter() - t0, time.process_time() - c0
    cores = max(1, round(cpu_s / t))
    tp = time.perf_counter()
    orc.solve_phase(H, orc.d)
    t_phase = time.perf_counter() - tp
    est = None
    if st_steps:
        est = {"seconds": sum(r["n_newton"] * t + r["n_stag"] * t_phase for r in st_steps),
               "gpu_st_fp64_seconds": sum(r["time_ms"] for r in st_steps) / 1e3,
               "steps": [r["step"] for r in st_steps],
               "method": ("extrapolated: the ST FP64 run's Newton iterations x the sample time "
                          "plus its staggered iterations x the phase-solve time")}
    return {
        "value": t,
        "unit": "s per sample (one Newton iteration of the k = 0 displacement solve of load "
                "step 1, QP update and staggered residual)",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{problem.name} ({2 * (problem.nx + 1) * (problem.ny + 1)} displacement "
                   f"DOF): load step 1, k = 0 displacement solve with one Newton iteration "
                   f"(assembled CSR + SuperLU), {t:.1f} s wall, {cpu_s:.1f} s CPU "
                   f"({cores} host core{'s' if cores > 1 else ''}); the GPU's ST FP64 run of "
                   f"the same sample took {t_gpu * 1e3:.1f} ms"),
        "gpu_same_sample_s": t_gpu,
        "oracle_over_gpu": t / t_gpu,
        "phase_solve_s": t_phase,
        "window_estimate": est,
    }


def run_oracle_history(args):
    """The oracle over the whole 64^2 load history, ST and S1, on one host
    process: total time, staggered iterations per step, forces."""
    import dataclasses

    import oracle
    import workloads as W
    base = W.config_tension64()
    if args.max_stag > 0:
        base = dataclasses.replace(base, max_stag=args.max_stag)
    out = []
    for scheme in (0, 1):
        orc = oracle.Oracle(base, scheme)
        t0, c0 = time.perf_counter(), time.process_time()
        rows = []
        for lam in base.loads:
            st = orc.load_step(float(lam))
            rows.append({"n_stag": st.n_stag, "converged": bool(st.converged),
                         "force": st.force})
        secs, cpu_s = time.perf_counter() - t0, time.process_time() - c0
        out.append({"scheme": ["ST", "S1"][scheme], "seconds": secs, "cpu_seconds": cpu_s,
                    "cores": max(1, round(cpu_s / secs)),
                    "n_stag_total": sum(r["n_stag"] for r in rows), "steps": rows})
        log(f"  oracle {out[-1]['scheme']}: {secs:.1f} s, N_stag {out[-1]['n_stag_total']}")
    return {
        "metric": "oracle time per load history (CPU baseline), ST and S1 FP64",
        "value": out[1]["seconds"], "unit": "s", "n_gpus": 0, "steps": len(base.loads),
        "warmup": 0, "ms_per_step": out[1]["seconds"] * 1e3 / len(base.loads),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"oracle-history: {base.name} ({base.nx}x{base.ny}, "
                               f"{len(base.loads)} load steps), max_stag {base.max_stag}"},
        "cpu_baseline": {"kind": "oracle", "runs": out},
    }


# Algorithmic bytes per node of the 3-D operators (FP64): internal force
# reads u (3 comps) and d, writes R (3); tangent apply reads u, d and p (3),
# writes q (3); phase apply reads the 8 point coefficients of one element
# per node, p and writes q.
BYTES_3D = {"internal_force": (3 + 1 + 3) * 8, "tangent_apply": (3 + 1 + 3 + 3) * 8,
            "phase_apply": (8 + 1 + 1) * 8}


def run_apply3d(pf, args):
    """Time per launch of the 3-D operators over cube sizes."""
    import types

    import torch

    import workloads as W
    out = []
    for n in (32, 64, 96):
        box = types.SimpleNamespace(nx=n, ny=n, nz=n, lx=1.0, ly=1.0, lz=1.0,
                                    material=W.Material())
        ops = pf.Hex3DOps(box)
        N, E = ops.N, ops.E
        g = torch.Generator(device="cuda").manual_seed(n)
        u = torch.rand(3 * N, dtype=torch.float64, device="cuda", generator=g) * 1e-3
        d = torch.rand(N, dtype=torch.float64, device="cuda", generator=g)
        pvec = torch.rand(3 * N, dtype=torch.float64, device="cuda", generator=g)
        coef = torch.rand(8 * E, dtype=torch.float64, device="cuda", generator=g) + 1.0
        q3 = torch.empty(3 * N, dtype=torch.float64, device="cuda")
        q1 = torch.empty(N, dtype=torch.float64, device="cuda")
        calls = {"internal_force": lambda: ops.internal_force(u, d, q3),
                 "tangent_apply": lambda: ops.tangent_apply(u, d, pvec, q3),
                 "phase_apply": lambda: ops.phase_apply(coef, d, q1)}
        for name, fn in calls.items():
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 20
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            gbs = BYTES_3D[name] * N / (us * 1e-6) / 1e9
            out.append({"mesh": f"{n}^3", "kernel": name, "nodes": N, "us": us, "GBs": gbs,
                        "frac_hbm": gbs / HBM_PEAK_GBS})
            log(f"  {n}^3 {name}: {us:.1f} us, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS * 100:.1f} %)")
    big = [r for r in out if r["mesh"] == "96^3" and r["kernel"] == "tangent_apply"][0]
    return {
        "metric": "3-D tangent apply GB/s vs mesh size, 1 MI355X", "value": big["GBs"],
        "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": big["us"] / 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "apply3d: unit cubes of 32^3, 64^3 and 96^3 trilinear "
                               "hexahedra, random fields, VD split"},
        "roofline": {"bound": "alu", "achieved": big["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": big["frac_hbm"], "traffic": None,
                     "note": "node-gather kernels re-evaluate each element per node; the "
                             "fraction is of the HBM peak they cannot reach"},
        "sizes": out,
    }


def run_slab3d(pf, args):
    """S1 and ST through the 3-D load step on the extruded 64^2 panel."""
    import torch

    import workloads as W
    p = W.slab_from_panel(W.config_tension64(), nz=2, lz=2.0 / 64)
    if args.warmup + args.steps > len(p.loads):
        raise SystemExit("warmup + steps exceeds the load history")
    runs = {}
    for name, scheme in (("S1", pf.S1), ("ST", pf.ST)):
        ctx = pf.Hex3DContext(p, scheme=scheme)
        for n in range(args.warmup):
            ctx.load_step(float(p.loads[n]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows = [ctx.load_step(float(p.loads[n]))
                for n in range(args.warmup, args.warmup + args.steps)]
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        ctx.close()
        runs[name] = {"seconds": secs, "ms_per_step": secs * 1e3 / args.steps,
                      "gdof_updates_per_s": sum(r["dof_updates"] for r in rows) / secs / 1e9,
                      "n_stag": [r["n_stag"] for r in rows],
                      "force_y": [r["force"][1] for r in rows]}
        log(f"  3-D {name}: {secs:.2f} s, N_stag {runs[name]['n_stag']}")
    s1 = runs["S1"]
    return {
        "metric": "time per load step, 3-D slab, S1 vs ST FP64, 1 MI355X",
        "value": s1["gdof_updates_per_s"], "unit": "GDOF-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": s1["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"slab3d: {p.nx}x{p.ny}x{p.nz} hexahedra (the {p.nx}^2 notched "
                               f"tension panel extruded, u_z = 0 on both faces), load steps "
                               f"{args.warmup + 1}..{args.warmup + args.steps}"},
        "s1_fp64": s1, "st_fp64": runs["ST"],
        "speedup_s1_vs_st": runs["ST"]["seconds"] / s1["seconds"],
    }


def run_sweep(pf, args):
    """Batched vs one-by-one throughput of the 64-instance sweep.  Modes
    (--sweep-modes): shared CG launches, concurrent streams, one by one;
    value is the first listed mode's GDOF-updates/s.  Each mode runs load
    steps 1..W untimed, then W+1..W+K timed, of every instance."""
    import torch

    import workloads as W
    probs = W.batch_instances()
    # --sweep-part K/M: the instances i with i % M == K (a long history split
    # over several jobs)
    part_k, part_m = (int(v) for v in args.sweep_part.split("/"))
    if not (part_m >= 1 and 0 <= part_k < part_m):
        raise SystemExit("--sweep-part: K/M with 0 <= K < M")
    index = [i for i in range(len(probs)) if i % part_m == part_k]
    probs = [probs[i] for i in index]
    steps, warm = args.steps, args.warmup
    if warm + steps > min(len(p.loads) for p in probs):
        raise SystemExit("warmup + steps exceeds the instances' load history")
    modes = [m.strip() for m in args.sweep_modes.split(",") if m.strip()]
    if not modes or any(m not in ("shared", "streams", "one") for m in modes):
        raise SystemExit("--sweep-modes: a comma list of shared, streams, one")
    chosen = [args.sweep_rows] * len(probs)
    if args.sweep_rows == 0:
        for i, p in enumerate(probs):
            ctx = pf.Context(p, scheme=pf.S1, precision=pf.MIXED, march_rows=0)
            chosen[i] = ctx.autotune(10)
            ctx.close()
    res = {}

    def one_by_one():
        t, upd, forces, rows_all = 0.0, 0.0, [], []
        for i, p in enumerate(probs):
            ctx = pf.Context(p, scheme=pf.S1, precision=pf.MIXED, march_rows=chosen[i])
            for n in range(warm):
                ctx.load_step(float(p.loads[n]))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rows = [ctx.load_step(float(p.loads[n])) for n in range(warm, warm + steps)]
            torch.cuda.synchronize()
            t += time.perf_counter() - t0
            upd += sum(r["dof_updates"] for r in rows)
            forces.append([r["force"] for r in rows])
            rows_all.append(rows)
            ctx.close()
            if (i + 1) % 16 == 0:
                log(f"  one by one: {i + 1}/{len(probs)} instances, {t:.1f} s timed")
        return t, upd, forces, rows_all

    def batched(shared):
        streams = [torch.cuda.Stream() for _ in probs]
        ctxs = [pf.Context(p, scheme=pf.S1, precision=pf.MIXED, stream=st.cuda_stream,
                           march_rows=ch) for p, st, ch in zip(probs, streams, chosen)]
        B = pf.Batch(ctxs, workers=args.workers, shared=shared)
        for n in range(warm):
            B.load_step([float(p.loads[n]) for p in probs])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows = []
        jl = open(args.stats_jsonl, "a") if args.stats_jsonl else None
        for n in range(warm, warm + steps):
            rows.append(B.load_step([float(p.loads[n]) for p in probs]))
            if jl:
                jl.write(json.dumps({
                    "mode": "shared" if shared else "streams", "step": n + 1,
                    "seconds": time.perf_counter() - t0, "instances": index,
                    "force": [r["force"] for r in rows[-1]],
                    "n_stag": [r["n_stag"] for r in rows[-1]],
                    "converged": [int(r["converged"]) for r in rows[-1]],
                    "dof_updates": sum(r["dof_updates"] for r in rows[-1])}) + "\n")
                jl.flush()
            if (n + 1) % 5 == 0:
                log(f"  {'shared launches' if shared else 'concurrent streams'}: load step "
                    f"{n + 1}, {time.perf_counter() - t0:.1f} s, max N_stag "
                    f"{max(r['n_stag'] for r in rows[-1])}")
        if jl:
            jl.close()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        B.close()
        for c in ctxs:
            c.close()
        upd = sum(r["dof_updates"] for rr in rows for r in rr)
        forces = [[rows[k][i]["force"] for k in range(steps)] for i in range(len(probs))]
        rows_t = [[rows[k][i] for k in range(steps)] for i in range(len(probs))]
        return t, upd, forces, rows_t

    for m in modes:
        if m == "one":
            res[m] = one_by_one()
        else:
            res[m] = batched(m == "shared")
        log(f"  {m}: {res[m][0]:.2f} s, {res[m][1] / res[m][0] / 1e9:.1f} GDOF-updates/s")
    ref = res[modes[0]]
    same = {m: res[m][2] == ref[2] for m in modes[1:]}
    rows_ref = ref[3]
    n_stag = [sum(r["n_stag"] for r in rr) for rr in rows_ref]
    capped = sum(1 for rr in rows_ref for r in rr if not r["converged"])
    sizes = [p.nx for p in probs]
    names = {"shared": "shared_launches", "streams": "concurrent_streams", "one": "one_by_one"}
    out = {
        "metric": "GDOF-updates/s, 64-instance S1 mixed sweep, batched vs one by one, 1 MI355X",
        "value": ref[1] / ref[0] / 1e9, "unit": "GDOF-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": ref[0] * 1e3 / steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": (f"sweep64: {len(probs)} of the 64 seeded notched tension "
                                f"instances (index % {part_m} == {part_k}), meshes "
                                f"{min(sizes)}^2..{max(sizes)}^2 (sum {sum(s * s for s in sizes)} "
                                f"elements), load steps {warm + 1}..{warm + steps} of 50"),
                   "scheme": "S1", "precision": "mixed", "workers": args.workers,
                   "march_rows": sorted(set(chosen)), "mode": names[modes[0]]},
        "staggered_iterations_per_instance": n_stag,
        "steps_at_max_stag": capped,
    }
    for m in modes:
        t, upd = res[m][0], res[m][1]
        out[names[m]] = {"value": upd / t / 1e9, "seconds": t,
                         "identical_forces_to_first_mode": same.get(m, True)}
    if "one" in res and modes[0] != "one":
        out["speedup_vs_one_by_one"] = res["one"][0] / ref[0]
    return out


def run_apply_sizes(pf, args):
    """Fused FP32 tangent apply and CG vector update over mesh sizes and
    work-item heights (march_rows 0 = the library's own choice)."""
    import workloads as W
    out = []
    for n in (512, 1024, 2048, 4096):
        p = W.tension_panel(n=n, l=4.0 / n, du=6e-5, steps=1)
        for ch in (0, 1, 2, 4, 8):
            ctx = pf.Context(p, scheme=pf.ST, precision=pf.MIXED, max_stag=1, max_newton=1,
                             max_cg=args.apply_iters, march_rows=ch)
            ctx.set_profiling(True)
            ctx.load_step(float(p.loads[0]))
            la, ms_a, nodes = ctx.kernel_time(0)
            lu, ms_u, _ = ctx.kernel_time(2)
            ctx.close()
            ta, tu = ms_a / max(la, 1), ms_u / max(lu, 1)
            ba = fused_apply_bytes_per_node() * nodes
            bu = update_bytes_per_node() * nodes
            out.append({
                "mesh": f"{n}x{n}", "march_rows": ch, "nodes": nodes,
                "apply_us": ta * 1e3, "apply_GBs": ba / (ta * 1e-3) / 1e9,
                "apply_frac": ba / (ta * 1e-3) / 1e9 / HBM_PEAK_GBS, "apply_launches": la,
                "update_us_with_events": tu * 1e3,
            })
            log(f"  {n}^2 rows={ch}: apply {ta * 1e3:.1f} us {out[-1]['apply_GBs']:.0f} GB/s "
                f"({out[-1]['apply_frac'] * 100:.1f} %)")
    big = [r for r in out if r["mesh"] == "4096x4096" and r["march_rows"] == 0][0]
    return {
        "metric": "fused FP32 tangent apply GB/s vs mesh size, 1 MI355X",
        "value": big["apply_GBs"], "unit": "GB/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "apply-sizes: notched tension panels 512^2..4096^2, one "
                               f"displacement solve capped at {args.apply_iters} CG iterations"},
        "roofline": {"bound": "hbm", "achieved": big["apply_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": big["apply_frac"], "traffic": None},
        "sizes": out,
    }


def run_trial_readings(pf, args):
    """The readings of the trial solve on one problem (FP64): the floored
    block with predict -> correct (the default), the unfloored block by
    MINRES, the trial-only update, both literal readings together, and ST
    for reference.  Per step: staggered iterations, convergence, trial
    solves and their iterations, floor candidates and the reaction force."""
    import dataclasses
    import workloads as W
    base = {"tension64": W.config_tension64, "tension512": W.config_tension512}[
        args.trial_problem]()
    if args.max_stag > 0:
        base = dataclasses.replace(base, max_stag=args.max_stag)
    if args.trial_steps > 0:
        base = dataclasses.replace(base, loads=base.loads[:args.trial_steps])
    readings = [("ST", "st", 0, 0, 0)]
    for scheme in (1, 3):
        for name, key, op, upd in (("floored, predict-correct", "floored-pc", 0, 0),
                                   ("unfloored (MINRES), predict-correct", "unfloored-pc", 1, 0),
                                   ("floored, trial-only", "floored-only", 0, 1),
                                   ("unfloored (MINRES), trial-only", "unfloored-only", 1, 1)):
            readings.append((f"S{scheme} {name}", f"s{scheme}-{key}", scheme, op, upd))
    if args.trial_reading != "all":
        readings = [r for r in readings if r[1] == args.trial_reading]
    out = []
    ref_force = None
    for label, _, scheme, op, upd in readings:
        p = dataclasses.replace(base, trial_operator=op, trial_update=upd)
        ctx = pf.Context(p, scheme=scheme, precision=pf.FP64)
        torch_sync()
        t0 = time.perf_counter()
        rows = []
        for lam in p.loads:
            st = ctx.load_step(float(lam))
            rows.append({"n_stag": st["n_stag"], "converged": st["converged"],
                         "n_trial": st["n_trial"], "n_it_trial": st["n_cg_trial"],
                         "floor_candidates": st["floor_hits"],
                         "force": st["force"][p.load_comp]})
            if st["n_stag"] >= 50:
                log(f"    {label} step {len(rows)}: n_stag {st['n_stag']} "
                    f"converged {st['converged']}")
        torch_sync()
        secs = time.perf_counter() - t0
        ctx.close()
        F = [r["force"] for r in rows]
        if ref_force is None:
            ref_force = F
        peak = max(abs(f) for f in ref_force)
        dev = max(abs(a - b) for a, b in zip(F, ref_force)) / peak
        out.append({"reading": label, "seconds": secs,
                    "n_stag_total": sum(r["n_stag"] for r in rows),
                    "steps_not_converged": sum(1 for r in rows if not r["converged"]),
                    "trial_iterations": sum(r["n_it_trial"] for r in rows),
                    "force_dev_vs_st": dev, "steps": rows})
        log(f"  {label}: {secs:.2f} s, N_stag {out[-1]['n_stag_total']}, "
            f"not converged {out[-1]['steps_not_converged']}, force dev {dev:.3e}")
    lit = ([r for r in out if r["reading"] == "S1 unfloored (MINRES), predict-correct"]
           or out)[0]
    return {
        "metric": "staggered iterations per load history under the trial readings, 1 MI355X",
        "value": lit["n_stag_total"], "unit": "staggered iterations", "n_gpus": 1,
        "steps": len(base.loads), "warmup": 0, "ms_per_step": lit["seconds"] * 1e3 / len(base.loads),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"trial-readings: {base.name} ({base.nx}x{base.ny}, "
                               f"{len(base.loads)} load steps), FP64, max_stag {base.max_stag}"},
        "readings": out,
    }


def torch_sync():
    import torch
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="tension512",
                    choices=["tension512", "tension64", "shear1024", "lshape2048", "sweep64",
                             "apply-sizes", "trial-readings", "oracle-history", "slab3d",
                             "apply3d"])
    ap.add_argument("--trial-problem", default="tension64", choices=["tension64", "tension512"],
                    help="problem of the trial-readings mode (its whole load history)")
    ap.add_argument("--trial-reading", default="all",
                    choices=["all", "st"] + [f"s{k}-{r}" for k in (1, 3) for r in
                                             ("floored-pc", "unfloored-pc", "floored-only",
                                              "unfloored-only")],
                    help="run only this reading in the trial-readings mode")
    ap.add_argument("--trial-steps", type=int, default=0,
                    help="first load steps of the trial-readings problem (0: all)")
    ap.add_argument("--max-stag", type=int, default=0,
                    help="staggered iteration cap of the trial-readings and oracle-history "
                         "modes (0: the problem's)")
    ap.add_argument("--workers", type=int, default=16, help="host workers of the sweep batch")
    ap.add_argument("--sweep-modes", default="shared,streams,one",
                    help="sweep64: comma list of modes to run (shared launches, concurrent "
                         "streams, one by one); value is the first mode's throughput")
    ap.add_argument("--schemes", default="",
                    help="comma list of further fixed-stress schemes (S2, S3) run in mixed "
                         "precision on the same window as S1 mixed, reported beside it")
    ap.add_argument("--jacobi", action="store_true",
                    help="plain Jacobi instead of Jacobi-Chebyshev for both schemes")
    ap.add_argument("--s1-degree", type=int, default=3, help="Chebyshev degree, S1 mixed")
    ap.add_argument("--st-degree", type=int, default=5, help="Chebyshev degree, ST FP64")
    ap.add_argument("--rows", type=int, default=-1,
                    help="work decomposition of the S1 mixed run (march_rows: 0 library "
                         "choice, 1 LDS tiles, 2/4/8 column marching); default: LDS tiles at "
                         "512^2, library choice else")
    ap.add_argument("--st-rows", type=int, default=-1,
                    help="work decomposition of the ST FP64 run; default: column marching with "
                         "2 rows at 512^2, library choice else")
    ap.add_argument("--tune-reps", type=int, default=0,
                    help="autotuner launches per candidate (0: keep --rows)")
    ap.add_argument("--sweep-part", default="0/1",
                    help="sweep64: K/M runs the instances whose index is K modulo M")
    ap.add_argument("--sweep-rows", type=int, default=4,
                    help="work decomposition of every sweep instance (0: autotune each)")
    ap.add_argument("--apply-iters", type=int, default=512,
                    help="CG iterations per size in the apply-sizes mode")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--stats-jsonl", default="",
                    help="write one JSON line of statistics per load step of the S1 mixed and "
                         "ST FP64 runs to this file")
    ap.add_argument("--no-st", action="store_true", help="skip the ST FP64 comparison run")
    ap.add_argument("--st-only", action="store_true",
                    help="time only the ST FP64 run (long histories in separate jobs)")
    ap.add_argument("--full-history", action="store_true",
                    help="time the whole load history (warmup 0, all steps) for both schemes")
    ap.add_argument("--window-end", type=int, default=-1,
                    help="last timed load step: load steps 1..end-steps-warmup run first "
                         "(S1 mixed, untimed) and both schemes start from that state; default "
                         "91 on tension512 (the step in which the crack runs through the "
                         "ligament), else warmup + steps from the initial state")
    ap.add_argument("--at1", action="store_true",
                    help="AT1 with penalised irreversibility instead of AT2 with the history "
                         "field, for both schemes")
    ap.add_argument("--guess-vectors", type=int, default=4,
                    help="start the displacement solves of the timed runs (both schemes) from "
                         "the projection onto this many earlier solutions (0..4; 0 = from "
                         "zero)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (for HBM counter scaling)")
    args = ap.parse_args()

    global GUESS_VECTORS
    GUESS_VECTORS = args.guess_vectors
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    if args.workload == "oracle-history":
        print(json.dumps(run_oracle_history(args)))
        return

    import torch

    import paper_2209_07969_amd as pf
    import workloads as W

    pf.require_device()
    if args.workload == "sweep64":
        print(json.dumps(run_sweep(pf, args)))
        return
    if args.workload == "apply-sizes":
        print(json.dumps(run_apply_sizes(pf, args)))
        return
    if args.workload == "trial-readings":
        print(json.dumps(run_trial_readings(pf, args)))
        return
    if args.workload == "slab3d":
        print(json.dumps(run_slab3d(pf, args)))
        return
    if args.workload == "apply3d":
        print(json.dumps(run_apply3d(pf, args)))
        return
    if args.rows < 0:
        args.rows = 1 if args.workload == "tension512" else 0
    if args.st_rows < 0:
        args.st_rows = 2 if args.workload == "tension512" else 0
    problem = {"tension512": W.config_tension512, "tension64": W.config_tension64,
               "shear1024": W.config_shear1024,
               "lshape2048": W.config_lshape2048}[args.workload]()
    if args.at1:
        import dataclasses
        problem = dataclasses.replace(problem, phase_model=1)
    if args.full_history:
        args.warmup, args.steps = 0, len(problem.loads)
        args.window_end = len(problem.loads)
    if args.window_end < 0:
        args.window_end = (NUCLEATION_STEP_512 if args.workload == "tension512"
                           else args.warmup + args.steps)
    start = args.window_end - args.steps - args.warmup
    if start < 0 or args.window_end > len(problem.loads):
        raise SystemExit("the window (warmup + steps ending at --window-end) does not fit the "
                         "load history")
    if args.copy_calibration:
        # plain elementwise kernels of known size for counter scaling: a fill
        # (256 MiB written) and a scale-copy (256 MiB read + 256 MiB written)
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    s1_deg, st_deg = (None, None) if args.jacobi else (args.s1_degree, args.st_degree)
    jsonl = open(args.stats_jsonl, "w") if args.stats_jsonl else None
    if args.st_only:
        log(f"ST FP64 on {problem.name}")
        state = prefix_state(pf, problem, start, s1_deg, args.rows)
        ctx2, rows2, secs2 = run_steps(pf, problem, pf.ST, pf.FP64, args.warmup, args.steps,
                                       degree=st_deg, tune_reps=args.tune_reps, rows=args.st_rows,
                                       jsonl=jsonl, label="st_fp64", start=start, state=state)
        print(json.dumps({
            "metric": "time per load step, ST FP64 (comparison run)",
            "value": secs2 * 1e3 / args.steps, "unit": "ms/step", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": secs2 * 1e3 / args.steps,
            "higher_is_better": False, "seconds": secs2,
            "gdof_updates_per_s": sum(r["dof_updates"] for r in rows2) / secs2 / 1e9,
            "max_stag": problem.max_stag, "steps_table": step_table(rows2),
            "precond": "jacobi" if st_deg is None else f"jacobi-chebyshev degree {st_deg}",
            "march_rows": ctx2.chosen_rows, "guess_vectors": GUESS_VECTORS, "dtype": "f64",
            "data": "synthetic"}))
        ctx2.close()
        if jsonl:
            jsonl.close()
        return
    log(f"{problem.name}: load steps 1..{start} (S1 mixed, untimed) give both runs their "
        f"starting state")
    state = prefix_state(pf, problem, start, s1_deg, args.rows)
    log(f"S1 mixed on {problem.name}")
    ctx, rows, secs = run_steps(pf, problem, pf.S1, pf.MIXED, args.warmup, args.steps,
                                profile=True, degree=s1_deg, tune_reps=args.tune_reps,
                                rows=args.rows, jsonl=jsonl, label="s1_mixed", start=start,
                                state=state)
    updates = sum(r["dof_updates"] for r in rows)
    value = updates / secs / 1e9
    ms_per_step = secs * 1e3 / args.steps
    rows_s1 = ctx.chosen_rows if ctx.chosen_rows is not None else ctx.opts.march_rows
    # dominant kernel per CG iteration of the displacement solves: the fused
    # apply (one launch), the update fused with the first Chebyshev step
    # (one launch, degree >= 2) or the further Chebyshev steps (degree - 2)
    la, ma, nodes = ctx.kernel_time(0)
    lf, mf, _ = ctx.kernel_time(2)
    lc, mc, _ = ctx.kernel_time(3)
    # template argument of the kernel names: the work-item height, which the
    # library picks from the mesh size when rows is 0 (column marching)
    ch = "CH" if rows_s1 == 0 else rows_s1
    cands = [(ma / max(la, 1), la, ma / max(la, 1), fused_apply_bytes_per_node(),
              f"k_cg_apply<{ch}, OpTangent<float>> (fused CG direction update + "
              f"tangent apply)")]
    two = rows_s1 == 1 and s1_deg is not None and s1_deg >= 3   # tiles: two steps fused
    if s1_deg and s1_deg >= 2 and lf:
        if two:
            cands.append((mf / lf, lf, mf / lf, updcheb2_bytes_per_node(s1_deg == 3),
                          "k_cg_updcheb2<OpTangent<float>> (CG update fused with the first two "
                          "Chebyshev steps)"))
        else:
            cands.append((mf / lf, lf, mf / lf, updcheb_bytes_per_node(),
                          f"k_cg_updcheb<{ch}, OpUpdCheb<OpTangent<float>>> (CG update "
                          f"fused with the first Chebyshev step)"))
    further = (s1_deg - 3) if two else ((s1_deg - 2) if s1_deg else 0)
    if further > 0 and lc:
        cands.append((further * mc / lc, lc, mc / lc, cheb_step_bytes_per_node(),
                      f"k_march<{ch}, OpCheb<OpTangent<float>>> (Jacobi-Chebyshev step)"))
    _, launches, avg_ms, bpn, kname = max(cands, key=lambda c: c[0])
    alg_bytes = bpn * nodes
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    ctx.close()

    extra = {}
    for name in [x.strip().upper() for x in args.schemes.split(",") if x.strip()]:
        if name not in ("S2", "S3"):
            raise SystemExit(f"--schemes: unknown scheme {name}")
        log(f"{name} mixed on {problem.name}")
        ctx3, rows3, secs3 = run_steps(pf, problem, {"S2": pf.S2, "S3": pf.S3}[name], pf.MIXED,
                                       args.warmup, args.steps, degree=s1_deg,
                                       tune_reps=args.tune_reps, rows=args.rows, jsonl=jsonl,
                                       label=f"{name.lower()}_mixed", start=start, state=state)
        extra[f"{name.lower()}_mixed"] = {
            "seconds": secs3, "ms_per_step": secs3 * 1e3 / args.steps,
            "gdof_updates_per_s": sum(r["dof_updates"] for r in rows3) / secs3 / 1e9,
            "steps": step_table(rows3)}
        ctx3.close()

    st_res = None
    if not args.no_st:
        log(f"ST FP64 on {problem.name}")
        ctx2, rows2, secs2 = run_steps(pf, problem, pf.ST, pf.FP64, args.warmup, args.steps,
                                       degree=st_deg, tune_reps=args.tune_reps, rows=args.st_rows,
                                       jsonl=jsonl, label="st_fp64", start=start, state=state)
        upd2 = sum(r["dof_updates"] for r in rows2)
        st_res = {
            "seconds": secs2,
            "ms_per_step": secs2 * 1e3 / args.steps,
            "gdof_updates_per_s": upd2 / secs2 / 1e9,
            "precond": "jacobi" if st_deg is None else f"jacobi-chebyshev degree {st_deg}",
            "march_rows": ctx2.chosen_rows,
            "steps": step_table(rows2),
        }
        ctx2.close()

    # speedup over the whole window and over the steps both runs converged
    conv = None
    if st_res:
        both = [(a, b) for a, b in zip(rows, rows2) if a["converged"] and b["converged"]]
        t_s1 = sum(a["time_ms"] for a, _ in both)
        t_st = sum(b["time_ms"] for _, b in both)
        conv = {"steps": [a["step"] for a, _ in both],
                "s1_mixed_ms": t_s1, "st_fp64_ms": t_st,
                "speedup": (t_st / t_s1) if t_s1 > 0 else None}
    capped = {"s1_mixed": [r["step"] for r in rows if not r["converged"]],
              "st_fp64": [r["step"] for r in rows2 if not r["converged"]] if st_res else None}
    copy_gbs = copy_bandwidth()
    log(f"device copy (1 GiB): {copy_gbs:.0f} GB/s")

    cpu = None
    if not args.no_cpu:
        log("oracle CPU baseline sample")
        cpu = cpu_baseline(pf, problem, rows2 if st_res else None)

    traffic, traffic_src = measured_traffic(kname)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GDOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{problem.name}: {problem.nx}x{problem.ny} Q1 {KIND[args.workload]}, "
                         f"l={problem.material.l} mm, load steps {start + args.warmup + 1}.."
                         f"{start + args.warmup + args.steps} of {len(problem.loads)} x "
                         f"{problem.loads[0]:.2g} mm"
                         + (f" (both runs from the S1 mixed state after step {start}, then "
                            f"{args.warmup} untimed steps)" if start > 0 else "")
                         + (" ending in the step where the crack runs through the ligament"
                            if args.workload == "tension512"
                            and args.window_end == NUCLEATION_STEP_512 else "")),
            "max_stag": problem.max_stag,
            "scheme": "S1", "precision": "mixed (FP32 inner CG, FP64 outer)",
            "precond": "jacobi" if s1_deg is None else f"jacobi-chebyshev degree {s1_deg}",
            "march_rows": rows_s1,
            "tol_stag": problem.tol_stag, "tol_pcg": problem.tol_pcg,
            "phase_model": ("AT1 with penalised irreversibility" if args.at1
                            else "AT2 with history field"),
            "guess_vectors": GUESS_VECTORS,
        },
        "s1_mixed": {"seconds": secs, "steps": step_table(rows)},
        "st_fp64": st_res,
        "speedup_s1_mixed_vs_st_fp64": (st_res["ms_per_step"] / ms_per_step) if st_res else None,
        "speedup_converged_steps": conv,
        **extra,
        "steps_at_max_stag": capped,
        "roofline": {
            "kernel": kname,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_source": traffic_src,
            "avg_launch_us": avg_ms * 1e3,
            "sampled_launches": launches,
            "bytes_per_launch": alg_bytes,
            "copy_GBs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
        "cpu_baseline": cpu,
    }
    if jsonl:
        jsonl.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
