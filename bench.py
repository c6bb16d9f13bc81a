"""Throughput benchmark of the LBM-RANS step on one MI355X.

Workload (default): single seeded airfoil-like body, FP32, Re_c = 6e6,
Mach 0.15, 10 degrees incidence, 40-chord square domain, 8 levels from c/8 to
c/1024 with distance-band refinement (about 2.0M fluid cells, 1.25e8 cell
updates per coarse step).  A step is one coarse (level-0) step, i.e. the
whole recursive multilevel cycle in which level l takes 2^l sub-steps.

Prints one JSON line:  MLUPS = sum_l N_l 2^l per coarse step * steps / seconds.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM peak, D2Q9 LBM-RANS step; FP16-store vs FP32 at equal Cf error"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell update, as the method defines the work: populations
# read + write (18 x storage), nu-tilde read + write (2 x its precision), the
# wall distance in FP64, one flag byte
ALG_BYTES = {"f32": 18 * 4 + 8 + 8 + 1, "f16": 18 * 2 + 8 + 8 + 1, "bf16": 18 * 2 + 8 + 8 + 1,
             "f64": 18 * 8 + 16 + 8 + 1}
# what the step kernel moves per cell update by design: the algorithmic arrays with
# the wall distance in the arithmetic precision (4 B in FP32 arithmetic), plus the
# stored rho, u (written, 3 x CT) and the u of the SA stencil (read, 2 x CT)
IMPL_BYTES = {"f32": 18 * 4 + 8 + 4 + 1 + 20, "f16": 18 * 2 + 8 + 4 + 1 + 20,
              "bf16": 18 * 2 + 8 + 4 + 1 + 20, "f64": 18 * 8 + 16 + 8 + 1 + 40}
TARGET_FRAC = 0.60
DTYPE = {"f32": "f32", "f16": "f16-store/f32", "bf16": "bf16-store/f32", "f64": "f64",
         "mixed": "f32-store on the two finest levels, f16-store below/f32",
         "f16s": "f16-store (free-stream shift)/f32", "bf16s": "bf16-store (free-stream shift)/f32",
         "mixeds": "f32-store on the two finest levels, f16-store (free-stream shift) below/f32"}


def lup_bytes(storage, level, n_levels, table=None):
    """Algorithmic bytes of one cell update on a level (mixed storage: FP32 on the
    two finest levels, FP16 below); table=IMPL_BYTES for the kernel's own."""
    table = table or ALG_BYTES
    storage = {"f16s": "f16", "bf16s": "bf16", "mixeds": "mixed"}.get(storage, storage)
    if storage == "mixed":
        return table["f32"] if level >= n_levels - 2 else table["f16"]
    return table[storage]


def step_bytes(storage, sim, n_levels, repeat=1, table=None):
    """Algorithmic bytes of one coarse step of a solver (times repeat)."""
    return repeat * sum(lup_bytes(storage, l, n_levels, table) * sim.level_info(l)["n_fluid"] * 2 ** l
                        for l in range(n_levels))


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_airfoil_2M_traffic.txt")
THREE_ELEMENT_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_batch_three_element_19M_traffic.txt")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2601_18443_amd", "csrc", f) for f in ("lbr_kernels.hip", "lbr_host.cpp")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the code (comments and whitespace stripped) of the kernels and of
    the host code that lays out their launches; the same as the profile
    summaries record."""
    from paper_2601_18443_amd.prof_summary import kernel_source_hash as h
    return h()


def measured_traffic(storage, path=None):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter summary
    (default: the benchmark airfoil's), or None when the summary is missing or the
    kernel changed since."""
    path = path or TRAFFIC_FILE
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash() or vals.get("storage") != storage:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(case, min_seconds=10.0, max_steps=4):
    """The FP64 oracle on the same workload: build the same grid, then time whole coarse
    steps until about min_seconds of work (at most max_steps)."""
    import oracle
    t0 = time.perf_counter()
    sim = oracle.Sim(case)
    tb = time.perf_counter() - t0
    lups = sim.lups_per_coarse_step()
    steps, dt = 0, 0.0
    while steps < max_steps and (steps == 0 or dt < min_seconds):
        t0 = time.perf_counter()
        sim.advance(1)
        dt += time.perf_counter() - t0
        steps += 1
    log(f"oracle: build {tb:.1f} s, {steps} coarse steps in {dt:.1f} s")
    return {"value": lups * steps / dt / 1e6, "unit": "MLUPS", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{steps} coarse steps ({lups * steps} cell updates) of the same 8-level airfoil "
                      f"grid from the uniform initial state, FP64, OpenMP; grid build ({tb:.0f} s) untimed"}


def equal_cf(case, steps):
    """Storage precision at the converged state of the workload: FP32, FP16 and
    mixed storage (both with the free-stream shift) each run the same coarse
    steps from the same start (graph replay) and their surface data are compared
    with the FP64 path's, which is itself within 1e-10 of the FP64 oracle (the
    oracle would need hours for these steps).  The Cf bound is the one the FP32
    path is held to: max |Cf - Cf_FP64| <= 1 % of max |Cf_FP64|."""
    import paper_2601_18443_amd as P

    def run(st):
        s = P.Solver(case, storage=st)
        s.use_graph(True)
        s.advance(steps)
        s.synchronize()
        cp, cf = s.surface(0)
        f = s.forces()
        s.residual()
        s.advance(100)
        r = s.residual()
        s.close()
        log(f"equal-Cf check: {st} after {steps} coarse steps, residual {r:.1e}")
        return cp, cf, f, r

    ref = run("f64")
    out = {"coarse_steps": steps, "reference": "f64 path (within 1e-10 of the FP64 oracle)",
           "cf_bound": "max |dCf| <= 0.01 max |Cf|", "f64_residual": ref[3],
           "f64_forces": {"C_Df": ref[2][0], "C_D": ref[2][2], "C_L": ref[2][3]}}
    for st in ("f32", "f16s", "mixeds"):
        cp, cf, f, r = run(st)
        cf_err = float(np.max(np.abs(cf - ref[1])) / np.max(np.abs(ref[1])))
        out[st] = {"cp_max_abs": float(np.max(np.abs(cp - ref[0]))), "cf_max_abs_over_max_cf": cf_err,
                   "cd_rel": float(abs(f[2] - ref[2][2]) / abs(ref[2][2])),
                   "cl_rel": float(abs(f[3] - ref[2][3]) / abs(ref[2][3])),
                   "residual": r, "meets_cf_bound": bool(cf_err <= 0.01)}
    return out


def three_element_roofline(steps=10, tune=False):
    """The FP32 step on the 19.5M-cell three-element case, whose working set
    (about 5 GB) is far beyond the 256 MB Infinity Cache: the HBM fraction of the
    step without cache help.  The start-up ramp is shortened to one coarse step,
    since only the kernel durations are measured here."""
    import torch
    import lbr_inputs as LI
    import paper_2601_18443_amd as P
    case = LI.case_three_element()
    case.update(ramp_steps=1.0)
    t0 = time.perf_counter()
    s = P.Solver(case, storage="f32")
    s.synchronize()
    log(f"three-element grid built in {time.perf_counter() - t0:.1f} s")
    rows = s.tune(trials=3) if tune else [4] * case["n_levels"]
    s.use_graph(True)
    s.advance(3)
    s.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(steps)
    s.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    s.profile(True)
    s.advance(steps)
    s.synchronize()
    kt = s.profile(False)
    L = case["n_levels"]
    lups = s.lups_per_coarse_step()
    launches = kt[3] if kt[3] > 0 else 2 ** L - 1
    bpl = step_bytes("f32", s, L) / launches
    achieved = bpl / (kt[0] * 1e-6) / 1e9
    traffic = measured_traffic("f32", THREE_ELEMENT_TRAFFIC_FILE)
    out = {"workload": "three-element high-lift-like case, 8 levels c/32..c/4096, FP32",
           "cells": int(sum(s.level_info(l)["n_fluid"] for l in range(L))), "lups_per_step": lups,
           "ms_per_step": round(1000 * dt / steps, 3), "mlups": round(lups * steps / dt / 1e6, 1),
           "tile_rows": rows, "avg_launch_us": round(kt[0], 3), "launches_per_step": round(launches, 2),
           "alg_bytes_per_launch": round(bpl, 0), "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": None if traffic is None else round(traffic, 0)}
    if traffic is not None:
        out["hbm_GBps"] = round(traffic / (kt[0] * 1e-6) / 1e9, 1)
        out["hbm_frac_measured"] = round(out["hbm_GBps"] / HBM_PEAK_GBS, 4)
    s.close()
    log(f"three-element FP32: {out['ms_per_step']} ms per step, frac {out['frac']}")
    return out


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "dispatches": 3}))


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Read + write GB/s of a plain device copy (torch copy_) of nbytes: what this
    part sustains for a pure stream, the reference for the kernel's HBM rate."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbps


def run_sweep(args):
    """Batched angle-of-attack sweep: 16 seeded cases (alpha -4..16 deg, 3-5 levels,
    finest c/512, 0.5M-3.4M cells each, 27M in all) advanced by shared launches, one
    super step taking case k through 2^(5 - L_k) coarse steps; against the same cases
    advanced one after another with the same number of steps each."""
    import torch
    import lbr_inputs as LI
    import paper_2601_18443_amd as P

    cases = [LI.case_sweep(k) for k in range(16)]
    log("building the 16 sweep grids on the GPU")
    t0 = time.perf_counter()
    sims = [P.Solver(c, storage=args.storage) for c in cases]
    for s in sims:
        s.synchronize()
    log(f"build {time.perf_counter() - t0:.1f} s")
    n_cells = int(sum(s.level_info(l)["n_fluid"] for s, c in zip(sims, cases) for l in range(c["n_levels"])))
    batch = P.Batch(sims)
    rows = batch.tune(trials=3) if args.tune else None
    if rows:
        log(f"tile heights per virtual level (tuned): {rows}")
    per = [batch.steps_per_super_step(k) for k in range(len(cases))]
    lups = batch.lups_per_super_step()
    lmax = max(c["n_levels"] for c in cases)
    if args.graph:
        batch.use_graph(True)
    log(f"{n_cells} cells, {lups} cell updates per super step; warmup {args.warmup}")
    batch.advance(args.warmup)
    batch.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.advance(args.steps)
    batch.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    batch.profile(True)
    batch.advance(args.steps)
    batch.synchronize()
    kt = batch.profile(False)
    # the same super steps as one cooperative grid per two super steps, with
    # grid-wide barriers in place of the launch boundaries (one format only)
    persistent = None
    if args.persistent and args.storage not in ("mixed", "mixeds"):
        batch.use_persistent(True)
        batch.advance(2)
        batch.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.advance(args.steps)
        batch.synchronize()
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        batch.use_persistent(False)
        persistent = {"value": round(batch.lups_per_super_step() * args.steps / dtp / 1e6, 1), "unit": "MLUPS",
                      "ms_per_step": round(1000 * dtp / args.steps, 4),
                      "launches_over_persistent": round(dtp / dt, 3), "tile_rows": 4}
        log(f"persistent grid: {args.steps} super steps in {dtp:.3f} s ({dtp / dt:.3f} x the launches)")
    batch.close()
    launches = kt[3] if kt[3] > 0 else 2 ** lmax - 1            # per super step
    log(f"batched: {args.steps} super steps in {dt:.3f} s; k_step_batch {kt[0]:.2f} us/launch, "
        f"finest {kt[1]:.2f}, level 0 {kt[2]:.2f}, {launches:.0f} launches per super step")
    finite = all(np.all(np.isfinite(s.forces())) for s in sims)
    bytes_per_launch = sum(step_bytes(args.storage, s, c["n_levels"], p)
                           for s, c, p in zip(sims, cases, per)) / launches

    def one_after_another(solvers):
        """The same cases advanced one after another, each with its own graph and
        tuned tile heights, the same coarse steps per case."""
        total = 0.0
        for s, p in zip(solvers, per):
            if args.tune:
                s.tune(trials=3)
            if args.graph:
                s.use_graph(True)
            s.advance(2 * p)
            s.synchronize()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.advance(args.steps * p)
            s.synchronize()
            torch.cuda.synchronize()
            total += time.perf_counter() - t0
        return total

    seq = one_after_another(sims)
    log(f"one after another ({args.storage}): {seq:.3f} s")
    seq32 = None
    if args.storage != "f32":
        # the baseline of the sweep: the same cases one after another in plain FP32
        for s in sims:
            s.close()
        sims32 = [P.Solver(c, storage="f32") for c in cases]
        seq32 = one_after_another(sims32)
        log(f"one after another (f32): {seq32:.3f} s")
        finite = finite and all(np.all(np.isfinite(s.forces())) for s in sims32)
        for s in sims32:
            s.close()
    mlups = lups * args.steps / dt / 1e6
    roof = None
    if kt[0] > 0:
        achieved = bytes_per_launch / (kt[0] * 1e-6) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_step_batch (all virtual levels)", "avg_launch_us": round(kt[0], 3),
                "launches_per_step": round(launches, 2),
                "finest_level_avg_launch_us": round(kt[1], 3), "level0_avg_launch_us": round(kt[2], 3),
                "alg_bytes_per_launch": round(bytes_per_launch, 0)}
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1000 * dt / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic (seeded airfoil-like polylines)",
        "config": {"workload": "batched sweep: 16 airfoil-like cases, AoA -4..16 deg, 3-5 levels to c/512, "
                               "Re 6e6, M 0.15; a step is one super step (2^(5 - L_k) coarse steps of case k)",
                   "cells": n_cells, "lups_per_step": lups, "coarse_steps_per_super_step": per,
                   "storage": args.storage, "graph": bool(args.graph), "tile_rows": rows},
        "roofline": roof, "cpu_baseline": None,
        "one_after_another": {"value": round(lups * args.steps / seq / 1e6, 1), "unit": "MLUPS",
                              "ms_per_step": round(1000 * seq / args.steps, 4)},
        "batched_over_one_after_another": round(seq / dt, 3),
        "persistent": persistent,
        "one_after_another_f32": None if seq32 is None else
        {"value": round(lups * args.steps / seq32 / 1e6, 1), "unit": "MLUPS",
         "ms_per_step": round(1000 * seq32 / args.steps, 4)},
        "batched_over_one_after_another_f32": None if seq32 is None else round(seq32 / dt, 3),
        "finite": bool(finite),
    }
    print(json.dumps(out), flush=True)


def run_sweep_steady(args):
    """The 16-case sweep run to steady state: batched (converged cases leave the
    launches) against the same cases one after another, each to the same
    tolerance with the same check interval in coarse steps.  The line's value is
    the batched wall time to solution."""
    import torch
    import lbr_inputs as LI
    import paper_2601_18443_amd as P

    tol, max_super, every = args.tol, args.max_super_steps, 100
    cases = [LI.case_sweep(k) for k in range(16)]
    sims = [P.Solver(c, storage=args.storage) for c in cases]
    batch = P.Batch(sims)
    rows = batch.tune(trials=3) if args.tune else None
    batch.use_graph(True)
    lmax = max(c["n_levels"] for c in cases)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps, res = batch.run_to_steady(tol, max_super, every)
    batch.synchronize()
    dt = time.perf_counter() - t0
    log(f"batched ({args.storage}): all 16 cases to residual < {tol:g} in {dt:.1f} s")
    per_case = []
    for k, (c, sim) in enumerate(zip(cases, sims)):
        f = sim.forces()
        per_case.append({"alpha_deg": c["alpha_deg"], "levels": c["n_levels"], "coarse_steps": steps[k],
                         "residual": res[k], "C_L": float(f[3]), "C_D": float(f[2]), "C_Df": float(f[0])})
    batch.close()
    for sim in sims:
        sim.close()
    seq = 0.0
    alone = []
    for k, c in enumerate(cases):
        sim = P.Solver(c, storage="f32")
        if args.tune:
            sim.tune(trials=3)
        sim.use_graph(True)
        per = 2 ** (lmax - c["n_levels"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        n, r = sim.run_to_steady(tol, max_super * per, every * per)
        sim.synchronize()
        seq += time.perf_counter() - t1
        alone.append({"coarse_steps": n, "residual": r, "C_L": float(sim.forces()[3])})
        sim.close()
        log(f"alone (f32) case {k}: {n} coarse steps, residual {r:.1e}")
    log(f"one after another (f32): {seq:.1f} s")
    line = {
        "metric": "wall time to steady state of the 16-case sweep", "value": round(dt, 2), "unit": "s",
        "n_gpus": 1, "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.storage],
        "data": "synthetic (seeded airfoil-like polylines)",
        "config": {"workload": "batched sweep to steady state: 16 airfoil-like cases, AoA -4..16 deg, 3-5 levels "
                               "to c/512, Re 6e6, M 0.15; residual checked every 100 super steps",
                   "tol": tol, "storage": args.storage, "tile_rows": rows},
        "roofline": None, "cpu_baseline": None,
        "one_after_another_f32_s": round(seq, 2), "batched_speedup": round(seq / dt, 3),
        "cases": per_case, "alone_f32": alone,
    }
    print(json.dumps(line), flush=True)


def run_precision(args):
    """Storage precision at the converged state of the 8-level airfoil: every
    storage runs the same number of coarse steps from the same start (graph
    replay, default tile heights), and its surface data are compared with
    those of the FP64 path (itself pinned to the FP64 oracle).  The Cf bound is
    the one the FP32 path is held to: max |Cf - Cf_FP64| <= 1 % of max |Cf_FP64|."""
    import torch
    import lbr_inputs as LI
    import paper_2601_18443_amd as P

    case = LI.case_airfoil_2M()
    steps = args.converge_steps

    def run(st):
        s = P.Solver(case, storage=st)
        s.use_graph(True)
        s.advance(1)
        s.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(steps - 1)
        s.synchronize()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cp, cf = s.surface(0)
        f = s.forces()
        s.residual()
        s.advance(100)
        r = s.residual()
        lups = s.lups_per_coarse_step()
        s.close()
        log(f"{st}: {steps} coarse steps in {dt:.1f} s, residual {r:.1e}")
        return cp, cf, f, r, lups * (steps - 1) / dt / 1e6

    ref = run("f64")
    out = {}
    for st in ("f32", "f16", "f16s", "mixed", "mixeds", "bf16", "bf16s"):
        cp, cf, f, r, mlups = run(st)
        cf_err = float(np.max(np.abs(cf - ref[1])) / np.max(np.abs(ref[1])))
        out[st] = {"cp_max_abs": float(np.max(np.abs(cp - ref[0]))), "cf_max_abs_over_max_cf": cf_err,
                   "cd_rel": float(abs(f[2] - ref[2][2]) / abs(ref[2][2])),
                   "cl_rel": float(abs(f[3] - ref[2][3]) / abs(ref[2][3])),
                   "residual": r, "meets_cf_bound": bool(cf_err <= 0.01), "mlups": round(mlups, 1)}
    ok = [st for st in out if out[st]["meets_cf_bound"]]
    best = max(ok, key=lambda st: out[st]["mlups"]) if ok else None
    line = {
        "metric": METRIC, "value": None if best is None else out[best]["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": steps, "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": None if best is None else DTYPE[best],
        "data": "synthetic (seeded airfoil-like polylines)",
        "config": {"workload": "precision at the converged state: single airfoil-like body, 8 levels "
                               "c/8..c/1024, Re 6e6, M 0.15, AoA 10 deg; every storage against the FP64 path",
                   "coarse_steps": steps, "fastest_within_cf_bound": best,
                   "fp64_forces": [float(v) for v in ref[2]], "fp64_residual": ref[3]},
        "roofline": None, "cpu_baseline": None,
        "storages": out,
    }
    print(json.dumps(line), flush=True)


def make_parser():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "f64", "mixed", "f16s", "bf16s", "mixeds"])
    ap.add_argument("--graph", type=int, default=1, help="replay the coarse step from a HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP16 / BF16 storage runs reported beside the main line")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--persistent", type=int, default=1,
                    help="sweep: also time the persistent mode (one cooperative grid per launch table)")
    ap.add_argument("--tune", type=int, default=0,
                    help="choose each level's tile height with the library's tuner before the warm-up (default: "
                         "the library's 64 x 4 tiles; the tuner times each level's sub-step alone and has picked "
                         "heights that are slower in the merged schedule)")
    ap.add_argument("--workload", default="airfoil",
                    choices=["airfoil", "three_element", "sweep", "sweep_steady", "precision"],
                    help="airfoil: the benchmark line (8 levels, 2.0M cells); three_element: the "
                         "19.4M-cell high-lift case (cycle time per step, run past its start-up ramp); "
                         "sweep: 16 cases in shared launches against the same cases one after another; "
                         "sweep_steady: the sweep run to steady state, batched against one after another; "
                         "precision: surface data of every storage at the converged airfoil state "
                         "against the FP64 path, and which storages meet the FP32 Cf bound")
    ap.add_argument("--tol", type=float, default=1e-6, help="residual tolerance of sweep_steady")
    ap.add_argument("--max-super-steps", type=int, default=6000, help="cap of sweep_steady")
    ap.add_argument("--converge-steps", type=int, default=5000,
                    help="coarse steps of every storage in the precision workload")
    ap.add_argument("--equal-cf-steps", type=int, default=3000,
                    help="coarse steps of the equal-Cf check of the default line (0: skip it)")
    ap.add_argument("--no-three-element", action="store_true",
                    help="skip the three-element FP32 roofline record of the default line")
    return ap


def main():
    args = make_parser().parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: running the step over several GPUs is not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "sweep":
        run_sweep(args)
        return
    if args.workload == "precision":
        run_precision(args)
        return
    if args.workload == "sweep_steady":
        run_sweep_steady(args)
        return

    import torch
    import lbr_inputs as LI
    import paper_2601_18443_amd as P

    if args.workload == "three_element":
        case = LI.case_three_element()
        args.warmup = max(args.warmup, int(case["ramp_steps"]) + 10)
        args.no_cpu_baseline = True
    else:
        case = LI.case_airfoil_2M()
    log(f"building the {case['n_levels']}-level {args.workload} grid on the GPU")
    t0 = time.perf_counter()
    sim = P.Solver(case, storage=args.storage)
    sim.synchronize()
    log(f"build {time.perf_counter() - t0:.1f} s")
    lups = sim.lups_per_coarse_step()
    finest = sim.level_info(case["n_levels"] - 1)
    rows = [4] * case["n_levels"]                    # the library's default tile height
    if args.tune:
        rows = sim.tune(trials=5)
        log(f"tile heights per level (tuned): {rows}")
    if args.graph:
        sim.use_graph(True)
    log(f"{lups} cell updates per coarse step; warmup {args.warmup}")
    sim.advance(args.warmup)
    sim.synchronize()

    # timed region
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.advance(args.steps)
    sim.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} coarse steps in {dt:.3f} s")
    # kernel durations: start / stop HIP events attached to every dispatch on the
    # library's streams (hipExtLaunchKernelGGL), over a window of the same length run
    # with direct launches right after the timed region
    sim.profile(True)
    sim.advance(args.steps)
    sim.synchronize()
    kt = sim.profile(False)
    log(f"event-timed kernels (us/launch): all launches {kt[0]:.2f}, finest {kt[1]:.2f}, "
        f"level 0 {kt[2]:.2f}; {kt[3]:.1f} launches per coarse step")
    mlups = lups * args.steps / dt / 1e6
    f = sim.forces()
    n_cells = int(sum(sim.level_info(l)["n_fluid"] for l in range(case["n_levels"])))
    if not np.all(np.isfinite(f)):
        log("warning: non-finite force coefficients")

    # roofline of the dominant kernel (k_step, all levels): algorithmic bytes per
    # launch = ALG_BYTES x cell updates per launch; duration from the HIP events
    n_levels = case["n_levels"]
    launches_per_step = kt[3] if kt[3] > 0 else sum(2 ** l for l in range(n_levels))
    bytes_per_launch = step_bytes(args.storage, sim, n_levels) / launches_per_step
    roof = None
    if kt[0] > 0:
        achieved = bytes_per_launch / (kt[0] * 1e-6) / 1e9
        traffic = measured_traffic(args.storage)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic, 0),
                "kernel": "k_step_batch (merged schedule, all levels)", "avg_launch_us": round(kt[0], 3),
                "launches_per_step": round(launches_per_step, 2),
                "finest_level_avg_launch_us": round(kt[1], 3),
                "level0_avg_launch_us": round(kt[2], 3),
                "alg_bytes_per_launch": round(bytes_per_launch, 0),
                "alg_bytes_per_lup": round(step_bytes(args.storage, sim, n_levels) / lups, 2),
                "impl_bytes_per_lup": round(step_bytes(args.storage, sim, n_levels, table=IMPL_BYTES) / lups, 2),
                "target_frac": TARGET_FRAC, "gap_to_target": round(TARGET_FRAC - achieved / HBM_PEAK_GBS, 4)}
        # context: the measured HBM rate of the kernel against a plain device copy
        copy = copy_bandwidth()
        roof["copy_GBps"] = round(copy, 1)
        if traffic is not None:
            hbm = traffic / (kt[0] * 1e-6) / 1e9
            roof["hbm_GBps"] = round(hbm, 1)
            # the counted (L2-miss) traffic against the peak: an upper bound on the
            # DRAM fraction here, since part of it may be served by the Infinity Cache
            roof["hbm_frac_measured"] = round(hbm / HBM_PEAK_GBS, 4)
            roof["hbm_over_copy"] = round(hbm / copy, 4)
        log(f"device copy {copy:.0f} GB/s")
    # the same workload with 16-bit population storage (FP32 arithmetic), same timing
    variants = {}
    if not args.no_variants and args.storage == "f32":
        sim.close()
        del sim
        for st in ("f16", "bf16", "mixed", "f16s", "bf16s", "mixeds"):
            v = P.Solver(case, storage=st)
            if args.tune:
                v.tune(trials=5)
            if args.graph:
                v.use_graph(True)
            v.advance(args.warmup)
            v.synchronize()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v.advance(args.steps)
            v.synchronize()
            torch.cuda.synchronize()
            dtv = time.perf_counter() - t0
            v.profile(True)
            v.advance(args.steps)
            v.synchronize()
            ktv = v.profile(False)
            per_lup = step_bytes(st, v, n_levels) / lups
            lv = ktv[3] if ktv[3] > 0 else launches_per_step
            ach = per_lup * lups / lv / (ktv[0] * 1e-6) / 1e9 if ktv[0] > 0 else None
            variants[st] = {"value": round(lups * args.steps / dtv / 1e6, 1), "unit": "MLUPS",
                            "ms_per_step": round(1000 * dtv / args.steps, 4),
                            "k_step_avg_launch_us": round(ktv[0], 3), "launches_per_step": round(lv, 2),
                            "achieved_GBps": None if ach is None else round(ach, 1),
                            "frac": None if ach is None else round(ach / HBM_PEAK_GBS, 4),
                            "alg_bytes_per_lup": round(per_lup, 2)}
            log(f"{st} storage: {variants[st]['value']} MLUPS, k_step {ktv[0]:.2f} us")
            v.close()
            del v
    eq = None
    if args.workload == "airfoil" and args.storage == "f32" and args.equal_cf_steps > 0:
        if "sim" in locals():
            sim.close()
            del sim
        eq = equal_cf(case, args.equal_cf_steps)
        mlups_of = {"f32": round(mlups, 1)}
        mlups_of.update({k: v["value"] for k, v in variants.items()})
        for st in ("f32", "f16s", "mixeds"):
            eq[st]["mlups"] = mlups_of.get(st)
        ok = [st for st in ("f32", "f16s", "mixeds") if eq[st]["meets_cf_bound"] and eq[st]["mlups"]]
        best = max(ok, key=lambda st: eq[st]["mlups"]) if ok else None
        eq["fastest_within_cf_bound"] = best
        eq["speedup_over_f32_at_equal_cf"] = (None if best is None or not eq["f32"]["mlups"]
                                              else round(eq[best]["mlups"] / eq["f32"]["mlups"], 3))
    te = None
    if args.workload == "airfoil" and args.storage == "f32" and not args.no_three_element:
        te = three_element_roofline(tune=bool(args.tune))
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the same workload")
        cpu = cpu_baseline(case)
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1000 * dt / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic (seeded airfoil-like polylines)",
        "config": {"workload": ("single airfoil-like body, 8 levels c/8..c/1024, 40c domain, "
                                "Re 6e6, M 0.15, AoA 10 deg") if args.workload == "airfoil" else
                               ("three-element high-lift-like configuration (slat, main, flap; "
                                "30 deg deflections), 8 levels c/32..c/4096, 40c domain, Re 9e6, "
                                "M 0.2, AoA 8 deg, after the start-up ramp"),
                   "cells": n_cells,
                   "finest_cells": finest["n_fluid"], "lups_per_step": lups,
                   "storage": args.storage, "graph": bool(args.graph), "tile_rows": rows},
        "roofline": roof, "cpu_baseline": cpu,
        "storage_variants": variants or None,
        "equal_cf": eq,
        "three_element_fp32": te,
        "forces": {"C_Df": f[0], "C_Dp": f[1], "C_D": f[2], "C_L": f[3]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
