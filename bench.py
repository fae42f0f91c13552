#!/usr/bin/env python3
"""Throughput of the full projection time step on one MI355X.

Default workload: the hall, 1024 x 512 x 256 cells (134M; 40 x 20 x 10 m,
dx = 3.9 cm), 2-cell solid walls, a ceiling slab with a 16-cell return plenum,
4 forced inlet vents blowing 1 m/s down, 2 outlet vents, 64 seeded obstacles,
CO2 1000 ppm in the hall and 400 ppm supply, CFL 0.3, sixth-order filter on,
four immersed-boundary FFT pressure iterations per step; FP64 (the headline),
then the same workload in the FP32 form with FP64 refinement.  A step is the
whole hot path: dt, momentum RK4, divergence, 4 x (IB right-hand side + 3D
real FFT + spectral solve + inverse FFT), correction, scalar RK4, filter, FP64
diagnostics.

Prints one JSON line.  ``value`` is Gcell-steps/s with all inputs resident in
HBM.  ``roofline`` prices the dominant kernel's algorithmic bytes per launch
against its average launch time, measured with HIP events recorded by the
library on the stream each launch goes to.  ``cpu_baseline`` times the FP64
CPU oracle on whole steps of the same workload on this host, in a child
process that runs beside the GPU measurements.  ``serving`` runs the request
stream of 64 room scenarios x 2000 steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published


def near_solid_cells(sc):
    """Cells with a solid face neighbour (where the IB term can be nonzero)."""
    b = sc.beta == 0
    near = np.zeros_like(b)
    for ax in range(3):
        near |= np.roll(b, 1, axis=ax) | np.roll(b, -1, axis=ax)
    return int(near.sum())


def kernel_bytes(sc, esz=8):
    """Algorithmic (compulsory) HBM bytes per launch of each kernel, for the
    step sequence of the library (stage-averaged where a kernel has modes)."""
    n = sc.ncells
    m = sc.nx // 2
    spec = 2 * esz * (m + 1) * sc.ny * sc.nz          # complex half spectrum
    nib = near_solid_cells(sc)
    return {
        # RK4 momentum: fields touched per stage 9, 15, 15, 9 (x esz) + mask byte
        "mom_stage": n * ((9 + 15 + 15 + 9) / 4 * esz + 1),
        # two stages per pass: u^n in, acc and u2 out (9 fields); u2, u^n, acc in, u* out (12)
        "mom_pair": n * ((9 + 12) / 2 * esz + 1),
        # the same for the scalar: c^n, u, v, w in, acc and c2 out (6); c2, c^n, acc, u, v, w in, c* out (7)
        "scalar_pair": n * ((6 + 7) / 2 * esz + 1),
        # RK4 scalar: 6, 8, 8, 6 fields + mask byte
        "scalar_stage": n * ((6 + 8 + 8 + 6) / 4 * esz + 1),
        "ib_rhs": nib * (4 + 1 + 3 * esz),             # list entry, saved r0, r, p centre
        "fft_x_fwd": n * esz + spec,                  # r in, spectrum out
        "fft_y": 2 * spec,
        "fft_z": 2 * spec,
        "fft_yz": 2 * spec,                           # fused y/z pass: one read, one write
        "fft_x_inv": spec + n * esz,
        "filter": n * (6 * esz + 1),                  # velocity: 3 fields in, 3 out
        "filter_c": n * (2 * esz + 1),                # CO2
        # FP64: u* and p in, u out; FP32 form: u*, p_n, dp in, u and p out (FP64 arithmetic)
        "correct": n * (7 * esz + 1) if esz == 8 else n * (9 * esz + 1),
        "div": n * 4 * esz,
        "refine_res": n * (5 * esz + 1),              # u*, p_n in (p_{n-1} only next to solids), res out
    }


def step_bytes(sc, esz=8, per_stage=False, fused_yz=False, mom_pairs=False, sca_pairs=False):
    """Pass-model bytes of one whole step (launch counts of the step sequence;
    fused_yz: the y/z passes of a solve run as one fused pass; mom_pairs,
    sca_pairs: the RK4 stages run two per pass)."""
    kb = kernel_bytes(sc, esz)
    it = sc.n_piter if (sc.beta == 0).any() else min(sc.n_piter, 1)
    y_passes = 2 if sc.ny > 1 else 0
    yz = kb["fft_yz"] if fused_yz else y_passes * kb["fft_y"] + kb["fft_z"]
    poisson = kb["fft_x_fwd"] + yz + kb["fft_x_inv"]
    ib = kb["ib_rhs"] if (sc.beta == 0).any() else 0
    projection = kb["div"] + it * (poisson + ib) + kb["correct"]
    if esz == 4 and it > 0:
        projection += kb["refine_res"] + poisson      # FP64 residual and one correction solve
    mom = 2 * kb["mom_pair"] if mom_pairs else 4 * kb["mom_stage"]
    sca = 2 * kb["scalar_pair"] if sca_pairs else 4 * kb["scalar_stage"]
    total = (mom + (4 if per_stage else 1) * projection + sca + (kb["filter"] + kb["filter_c"] if sc.filter else 0))
    return total


WORKLOADS = {
    "room": "ventilated room 256x128x96 (10x5x3.75 m), 8 seeded boxes, 1 m/s duct, CFL 0.3, filter on, "
            "4 IB pressure iterations",
    "large": "large room 512x256x192 (10x5x3.75 m), 8 seeded boxes, 1 m/s duct, CFL 0.3, filter on, "
             "4 IB pressure iterations",
    "hall": "hall 1024x512x256 (40x20x10 m), ceiling plenum, 4 forced inlets, 2 outlets, 64 seeded boxes, "
            "1 m/s, CFL 0.3, filter on, 4 IB pressure iterations",
}
# Smaller rooms (the grid sizes of the serving stream), where the y/z passes of
# each solve run as one fused pass: 10 m long, 4 seeded boxes, otherwise as the room.
SMALL_ROOMS = {"room64": (64, 64, 64), "room128": (128, 64, 64), "room192": (192, 96, 64)}
for _k, _g in SMALL_ROOMS.items():
    WORKLOADS[_k] = (f"room {_g[0]}x{_g[1]}x{_g[2]} (10 m long), 4 seeded boxes, 1 m/s duct, CFL 0.3, "
                     "filter on, 4 IB pressure iterations")


def workload(name="room"):
    import scenarios
    if name == "room":
        return scenarios.room()
    if name == "large":
        return scenarios.room(512, 256, 192, dx=10.0 / 512)
    if name == "hall":
        return scenarios.hall()
    if name in SMALL_ROOMS:
        g = SMALL_ROOMS[name]
        return scenarios.room(*g, dx=10.0 / g[0], n_boxes=4)
    raise ValueError(name)


def cpu_baseline_child(workload_name, steps):
    """Run in a child process (``bench.py --cpu-oracle WORKLOAD STEPS``): time
    the oracle (plain numpy FP64) on whole steps of the workload from its
    initial state and print one JSON line.  Set-up (scenario generation,
    dense forcing arrays) is not timed."""
    from oracle.step import Oracle
    sc = workload(workload_name)
    O = Oracle.from_scenario(sc)
    st = Oracle.state_from_scenario(sc)
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        st, _ = O.step(st)
        times.append(time.perf_counter() - t0)
        print(f"[cpu-oracle] {workload_name} step {len(times)}/{steps}: {times[-1]:.1f} s", file=sys.stderr,
              flush=True)
    el = sum(times)
    try:
        import resource
        rss_gb = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss / 1e6
    except Exception:
        rss_gb = None
    print(json.dumps({"cells": sc.ncells, "steps": steps, "seconds": el, "step_s": times, "rss_GB": rss_gb}),
          flush=True)


def start_cpu_baseline(workload_name, steps):
    """Start the oracle timing in a child process (before this process touches
    the GPU); returns the Popen."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-oracle", workload_name, str(steps)],
                            stdout=subprocess.PIPE, stderr=None, env=env, cwd=ROOT)


def finish_cpu_baseline(proc, workload_name, timeout_s):
    """Collect the child's timing (waiting at most timeout_s); None if it did
    not finish in time or failed."""
    import subprocess
    try:
        out, _ = proc.communicate(timeout=max(1.0, timeout_s))
    except subprocess.TimeoutExpired:
        proc.kill()
        proc.communicate()
        print("[bench] the CPU oracle did not finish in time; no cpu_baseline", file=sys.stderr, flush=True)
        return None
    if proc.returncode != 0:
        print(f"[bench] the CPU oracle failed (exit {proc.returncode}); no cpu_baseline", file=sys.stderr, flush=True)
        return None
    r = json.loads(out.decode().strip().splitlines()[-1])
    el = r["seconds"]
    return {
        "value": r["cells"] * r["steps"] / el / 1e9,
        "unit": "Gcell-steps/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{r['steps']} full step(s) of the same workload ({WORKLOADS[workload_name]}, FP64) from its "
                  f"initial state, {el:.1f} s wall in a child process on 1 of {os.cpu_count()} host cores (numpy "
                  f"elementwise and pocketfft run single-threaded), beside the GPU measurements; peak host "
                  f"memory {r['rss_GB']:.1f} GB",
    }


def particle_bench(S, sc, esz, n=1 << 20, steps=100, seed=5):
    """Lagrangian particles (Section 2.3) in the solver's current velocity: n
    particles of 1-100 um spread over the room, `steps` implicit-Euler steps.
    Algorithmic bytes per particle-step: position, velocity (read and write)
    and diameter (13 x 8 B) plus the 24 interpolation gathers (24 x esz)."""
    import torch
    rng = np.random.default_rng(seed)
    dev = S.device
    box = (sc.lx, sc.ly, sc.lz)
    pos = torch.as_tensor(np.stack([rng.uniform(0, box[a], n) for a in range(3)]), device=dev).contiguous()
    vel = torch.zeros((3, n), dtype=torch.float64, device=dev)
    diam = torch.as_tensor(rng.uniform(1e-6, 100e-6, n), device=dev)
    S.particles_step(pos, vel, diam, dt=1e-3)
    torch.cuda.synchronize()
    S.profile("particles")
    t0 = time.perf_counter()
    for _ in range(steps):
        S.particles_step(pos, vel, diam, dt=1e-3)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, nl = S.profile_read()
    S.profile(None)
    per = 1e-3 * ms / max(nl, 1)
    # the same particles sorted by cell once (their gathers then coalesce)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.particles_sort(pos, vel, diam)
    torch.cuda.synchronize()
    sort_s = time.perf_counter() - t1
    S.profile("particles")
    t0 = time.perf_counter()
    for _ in range(steps):
        S.particles_step(pos, vel, diam, dt=1e-3)
    torch.cuda.synchronize()
    el_s = time.perf_counter() - t0
    ms_s, nl_s = S.profile_read()
    S.profile(None)
    per_s = 1e-3 * ms_s / max(nl_s, 1)
    b = n * (13 * 8 + 24 * esz)
    return {"particles": n, "steps": steps, "Mparticle_steps_per_s": n * steps / el / 1e6,
            "kernel_avg_us": 1e6 * per, "algorithmic_GBs": b / per / 1e9, "bytes_per_particle_step": 13 * 8 + 24 * esz,
            "sorted": {"sort_ms": 1e3 * sort_s, "Mparticle_steps_per_s": n * steps / el_s / 1e6,
                       "kernel_avg_us": 1e6 * per_s, "algorithmic_GBs": b / per_s / 1e9}}


SERVING_POLICIES = ("pool_fp32_refine", "pool_fp64", "fifo_fp64")


def serving_bench(n_req, n_steps, budget_gib, mean_gap=0.5, seed=7, log=None,
                  policies=("pool_fp32_refine", "fifo_fp64")):
    """The serving stream: Poisson arrivals of room scenarios of four grid
    sizes, served with continuous batching in the pool (FP32 with FP64
    refinement, or FP64; HBM budget deliberately small so admission binds)
    and FIFO with the plain per-scenario FP64 loop.  Returns the summaries."""
    import scenarios
    from paper_2204_02107_amd import serving, FP32_REFINE, FP64
    reqs = scenarios.serving_requests(n_req, seed=seed, mean_gap=mean_gap, n_steps=n_steps)
    cases = {r["id"]: scenarios.serving_scenario(r) for r in reqs}
    out = {"requests": n_req, "steps_each": n_steps, "mean_gap_s": mean_gap, "hbm_budget_GiB": budget_gib,
           "stream_seed": seed, "cells_total": int(sum(c.ncells for c in cases.values()))}
    budget = int(budget_gib * (1 << 30))
    for pol in policies:
        if pol == "pool_fp32_refine":
            rec = serving.serve(reqs, cases, budget, FP32_REFINE, log=log)
        elif pol == "pool_fp64":
            rec = serving.serve(reqs, cases, budget, FP64, log=log)
        elif pol == "fifo_fp64":
            rec = serving.fifo(reqs, cases, FP64, log=log)
        else:
            raise ValueError(pol)
        out[pol] = serving.summarize(rec)
        if log:
            log(f"{pol}: " + json.dumps(out[pol]))
    return out


# Obstacle in the channel (Section 3.1.1, Table 2): the paper's St and C_D
# per obstacle resolution.
CUBE_PAPER = {30: {"St": 0.2097, "C_D": 3.12}, 60: {"St": 0.2094, "C_D": 3.05}}


def cube_bench(n_h, t_end, every=20, precision="fp64", chunk=512, cfl=0.3, per_stage=False):
    """Run the obstacle-in-channel case to t_end (units of h / U_b), sampling
    the obstacle force every ``every`` steps at CFL 0.3 (proportionally more
    steps at a smaller CFL, so that the samples stay equally spaced in time)
    on the device, and report the step throughput with the drag coefficient
    and Strouhal number over the second half of the run."""
    import torch
    import scenarios
    import paper_2204_02107_amd as m
    from paper_2204_02107_amd import postproc
    sc = scenarios.cube_channel(n_h, cfl=cfl)
    # the forcing relaxation time stays that of CFL 0.3, so that only the time step changes
    sc.tau_f = 2.0 * 0.3 * (sc.lx / sc.nx) / sc.meta["u_max"]
    every = max(1, int(round(every * 0.3 / cfl)))
    h, u_b = sc.meta["h"], sc.meta["u_b"]
    prec = m.FP64 if precision == "fp64" else m.FP32_REFINE
    S = m.Solver(sc, precision=prec, project_each_stage=per_stage)
    i0, i1, j0, j1, _, _ = sc.meta["obstacle_cells"]
    box = (i0 - 1, i1 + 1, j0 - 1, j1 + 1, 0, 1)
    buf = torch.zeros((chunk, 8), dtype=torch.float64, device=S.device)
    recs = []
    steps = 0
    t_stop = t_end * h / u_b
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while True:
        for r in range(chunk):
            S.step(every, diag=False)
            S.body_force(box, buf, r)
        steps += every * chunk
        part = buf.cpu().numpy()
        recs.append(part)
        t_sim = part[-1, 6]
        print(f"[cube] n_h={n_h} steps={steps} t={t_sim * u_b / h:.1f} h/U_b "
              f"F=({part[-1, 0] + part[-1, 3]:.4e}, {part[-1, 1] + part[-1, 4]:.4e}) "
              f"wall={time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        if not np.isfinite(part).all() or t_sim >= t_stop:
            break
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    S.close()
    rec = np.concatenate(recs)
    coef = postproc.obstacle_coefficients(rec, h, u_b, sc.lz)
    return {"workload": f"obstacle in channel, {n_h} cells per edge, {sc.nx}x{sc.ny}, Re_ob 84", "cells": sc.ncells,
            "precision": precision, "cfl": cfl, "projection": "every RK4 stage" if per_stage else "once per step",
            "steps": steps, "t_end_h_over_Ub": float(rec[-1, 6] * u_b / h),
            "wall_s": el, "Gcell_steps_s": sc.ncells * steps / el / 1e9, **coef,
            "paper_DNSLABIB": CUBE_PAPER.get(n_h)}


def consistency_run(workload_name="room", steps=2000, chunk=400):
    """The workload run `steps` steps in FP64 and in the FP32 form with FP64
    refinement: the room-mean CO2, its fitted decay rate (ACH) and the kinetic
    energy of both, and their differences (the accuracy statement of the FP32
    form over a long horizon)."""
    import torch
    import paper_2204_02107_amd as m
    from paper_2204_02107_amd import postproc
    sc = workload(workload_name)
    out = {"workload": WORKLOADS[workload_name], "steps": steps}
    for name, prec in (("fp64", m.FP64), ("fp32_refine", m.FP32_REFINE)):
        S = m.Solver(sc, precision=prec)
        diags = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(chunk, steps - done)
            S.step(k, diag=False)
            diags += S.read_diags(k)
            done += k
            print(f"[consistency] {name} steps={done} t={diags[-1]['t']:.3f}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        S.close()
        d = diags[-1]
        out[name] = {"t_end_s": d["t"], "wall_s": el, "Gcell_steps_s": sc.ncells * steps / el / 1e9, "ke": d["ke"],
                     "co2_room_mean_end": d["co2_room_mean"], "ach_fit_per_h": postproc.fitted_ach(diags[steps // 10:], c_out=400.0),
                     "div_l2_end": d["div_l2"]}
    a, b = out["fp64"], out["fp32_refine"]
    out["ach_rel_diff"] = abs(b["ach_fit_per_h"] - a["ach_fit_per_h"]) / abs(a["ach_fit_per_h"])
    out["co2_mean_diff_ppm"] = b["co2_room_mean_end"] - a["co2_room_mean_end"]
    out["ke_rel_diff"] = abs(b["ke"] - a["ke"]) / abs(a["ke"])
    return out


# Kernel symbol (as rocprofv3 prints it) -> name in kernel_bytes.
def kernel_key(sym):
    import re
    m = re.search(r"k_(\w+?)(_b)?(<([^>]*)>)?\(", sym)
    if not m:
        return None
    base, targs = m.group(1), (m.group(4) or "")
    if base == "mom_stage":
        return "mom_stage"
    if base == "mom_pair":
        return "mom_pair"
    if base == "sca_pair":
        return "scalar_pair"
    if base == "sca_stage":
        return "scalar_stage"
    if base in ("filter", "filter_lds", "filter_ring"):
        return "filter" if targs.endswith("3") else "filter_c"
    if base == "fft_cols":
        parts = [x.strip() for x in targs.split(",")]
        return "fft_z" if len(parts) > 1 and parts[1] == "2" else "fft_y"
    if base == "fft_yz":
        return "fft_yz"
    if base in ("correct", "refine_correct", "correct_ring", "refine_correct_ring"):
        return "correct"
    if base in ("div", "fft_x_fwd", "fft_x_inv", "ib_rhs", "refine_res", "refine_res_ib"):
        return base
    return None


def copy_probe(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of nbytes, reps times: the reference for
    scaling rocprofv3's FETCH_SIZE and WRITE_SIZE counters to bytes."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "reps": reps}), flush=True)


def pmc_per_kernel(csv_path, counter):
    """Mean counter value (KiB per dispatch) per kernel symbol from a
    rocprofv3 --pmc counter_collection.csv."""
    import csv
    acc = {}
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] != counter:
                continue
            k = row["Kernel_Name"]
            s, n = acc.get(k, (0.0, 0))
            acc[k] = (s + float(row["Counter_Value"]), n + 1)
    return {k: s / n for k, (s, n) in acc.items()}


def traffic_table(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes=1 << 30):
    """Calibrated HBM bytes per launch of each kernel: FETCH_SIZE and
    WRITE_SIZE scaled by what they read for the plain copy of copy_bytes."""
    cf = max(pmc_per_kernel(copy_fetch_csv, "FETCH_SIZE").items(), key=lambda kv: kv[1])[1]
    cw = max(pmc_per_kernel(copy_write_csv, "WRITE_SIZE").items(), key=lambda kv: kv[1])[1]
    f_scale, w_scale = copy_bytes / (1024 * cf), copy_bytes / (1024 * cw)
    out = {}
    for counter, path, scale in (("FETCH_SIZE", fetch_csv, f_scale), ("WRITE_SIZE", write_csv, w_scale)):
        sums = {}
        for sym, v in pmc_per_kernel(path, counter).items():
            key = kernel_key(sym)
            if key is None:
                continue
            s, n = sums.get(key, (0.0, 0))
            sums[key] = (s + v * 1024 * scale, n + 1)
        for key, (s, n) in sums.items():
            out.setdefault(key, {})["fetch_bytes" if counter == "FETCH_SIZE" else "write_bytes"] = s / n
    for key, d in out.items():
        d["bytes"] = d.get("fetch_bytes", 0.0) + d.get("write_bytes", 0.0)
    return {"fetch_scale": f_scale, "write_scale": w_scale, "kernels": out}


def measure(sc, prec, args, label):
    """Time args.steps whole steps (after args.warmup) of one workload in one
    precision, then each kernel's launches with HIP events: once in the step's
    own two-stream schedule, once with every launch alone on one stream."""
    import torch
    import paper_2204_02107_amd as m
    esz = 8 if prec == m.FP64 else 4
    dev = torch.device("cuda:0")
    S = m.Solver(sc, precision=prec, device=dev, project_each_stage=args.per_stage)
    S.set_stage_pairs(args.stage_pairs)
    S.set_fft_pipeline(args.fft_pipeline)
    if args.no_overlap:
        S.set_overlap(False)
    print(f"[bench] {label}: workload {sc.name} cells={sc.ncells} warmup={args.warmup}", file=sys.stderr, flush=True)
    S.step(args.warmup, diag=False)
    torch.cuda.synchronize()
    # timed region: exactly K steps, bracketed by synchronisation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(args.steps, diag=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hist = S.read_diags(1)[0]
    value = sc.ncells * args.steps / el / 1e9
    print(f"[bench] {label}: {args.steps} steps in {el:.3f} s -> {value:.3f} Gcell-steps/s; "
          f"t={hist['t']:.4f} ke={hist['ke']:.4e} co2_mean={hist['co2_room_mean']:.4f}",
          file=sys.stderr, flush=True)
    kb = kernel_bytes(sc, esz)

    def per_kernel():
        per = {}
        for name in kb:
            if name == "refine_res" and prec == m.FP64:
                continue
            S.profile(name)
            S.step(args.profile_steps, diag=False)
            ms, nl = S.profile_read()
            S.profile(None)
            if nl:
                per[name] = {"avg_us": 1e3 * ms / nl, "launches_per_step": nl / args.profile_steps,
                             "ms_per_step": ms / args.profile_steps, "GBs": kb[name] / (1e-3 * ms / nl) / 1e9}
        return per

    per = per_kernel()
    S.set_overlap(False)
    alone = per_kernel()
    S.set_overlap(not args.no_overlap)
    S.close()
    del S
    torch.cuda.empty_cache()
    # the dominant kernel and its roofline from the launches timed alone (the
    # second stream idle): in the step's own schedule the scalar half shares
    # the memory system with the momentum pairs on large grids
    dom = max(alone, key=lambda k: alone[k]["ms_per_step"])
    print(f"[bench] {label} per-kernel: " + json.dumps({k: {kk: round(vv, 3) for kk, vv in v.items()}
                                                       for k, v in per.items()}), file=sys.stderr, flush=True)
    sbytes = step_bytes(sc, esz, args.per_stage, fused_yz="fft_yz" in per, mom_pairs="mom_pair" in per,
                        sca_pairs="scalar_pair" in per)
    rnd = lambda d: {k: {"avg_us": round(v["avg_us"], 2), "GBs": round(v["GBs"], 1),
                         "frac": round(v["GBs"] / HBM_PEAK_GBS, 3), "launches_per_step": v["launches_per_step"]}
                     for k, v in d.items()}
    return {
        "value": value, "ms_per_step": 1e3 * el / args.steps, "steps": args.steps,
        "step_bytes_per_cell": sbytes / sc.ncells,
        "hbm_frac_end_to_end": sbytes * (value * 1e9 / sc.ncells) / (HBM_PEAK_GBS * 1e9),
        "dominant": dom, "dominant_GBs": alone[dom]["GBs"], "dominant_avg_us": alone[dom]["avg_us"],
        "kernels": rnd(per), "kernels_alone": rnd(alone),
    }


def traffic_of(workload_name, precision, kernel):
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(tfile):
        return None
    try:
        with open(tfile) as f:
            tr = json.load(f)
        return tr.get(f"{workload_name}/{precision}", {}).get(kernel)
    except (OSError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=1, help="whole oracle steps timed for cpu_baseline")
    ap.add_argument("--cpu-oracle", nargs=2, metavar=("WORKLOAD", "STEPS"), help=argparse.SUPPRESS)
    ap.add_argument("--profile-steps", type=int, default=10)
    ap.add_argument("--workload", default="hall", choices=list(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="precision of the headline value (the other form is measured too unless --one-form)")
    ap.add_argument("--one-form", action="store_true", help="measure only the headline precision")
    ap.add_argument("--per-stage", action="store_true",
                    help="the per-stage projection variant (a projection after every RK4 stage)")
    ap.add_argument("--no-particles", action="store_true")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run every launch of a step in order on one stream (for kernel traces whose durations "
                         "are those of each kernel alone)")
    ap.add_argument("--stage-pairs", type=int, default=-1, choices=[-1, 0, 1],
                    help="RK4 stages two per pass: -1 by grid size (default), 0 never, 1 wherever the tile divides the grid")
    ap.add_argument("--fft-pipeline", type=int, default=-1, choices=[-1, 0, 1],
                    help="pipelined FFT column passes: -1 by tile count (default), 0 never, 1 wherever they apply")
    ap.add_argument("--serving", default="config4", choices=["none", "short", "config4", "config4-all"],
                    help="serving stream: config4 = 64 requests x 2000 steps, pool FP32 form vs FIFO FP64; "
                         "config4-all adds the pool in FP64; short = 16 x 300")
    ap.add_argument("--serving-seeds", type=int, nargs="*", default=[7], help="stream seeds of the serving leg")
    ap.add_argument("--cube", type=int, nargs="*", metavar="N_H",
                    help="only run the obstacle-in-channel validation at these resolutions (cells per obstacle edge)")
    ap.add_argument("--cube-t-end", type=float, default=300.0, help="simulated time in units of h / U_b")
    ap.add_argument("--cube-cfl", type=float, default=0.3, help="maximum Courant number of the obstacle case")
    ap.add_argument("--consistency", type=int, metavar="STEPS",
                    help="only run the workload STEPS steps in FP64 and in the FP32 form and compare them")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run the plain 1 GiB device copy used to calibrate the PMC byte counters")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="fold rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE outputs of this benchmark and of --copy-probe "
                         "into profiles/traffic.json under <workload>/<precision> (no GPU needed)")
    args = ap.parse_args()
    if args.cpu_oracle:
        cpu_baseline_child(args.cpu_oracle[0], int(args.cpu_oracle[1]))
        return
    if args.traffic:
        tfile = os.path.join(ROOT, "profiles", "traffic.json")
        tab = {}
        if os.path.exists(tfile):
            with open(tfile) as f:
                tab = json.load(f)
        t = traffic_table(*args.traffic)
        tab[f"{args.workload}/{args.precision}"] = {k: v["bytes"] for k, v in t["kernels"].items()}
        tab[f"{args.workload}/{args.precision}/detail"] = t
        os.makedirs(os.path.dirname(tfile), exist_ok=True)
        with open(tfile, "w") as f:
            json.dump(tab, f, indent=1, sort_keys=True)
        print(json.dumps(t, indent=1))
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.consistency:
        print(json.dumps(consistency_run(args.workload, args.consistency)), flush=True)
        return
    if args.cube is not None:
        for n_h in args.cube or [30]:
            print(json.dumps(cube_bench(n_h, args.cube_t_end, precision=args.precision, cfl=args.cube_cfl,
                                        per_stage=args.per_stage)), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the step runs on a single MI355X and this build has "
              "no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    t_start = time.perf_counter()
    # the oracle's timing starts first, in a child process, before this
    # process touches the GPU; it runs beside the GPU measurements
    cpu_proc = None if args.no_cpu else start_cpu_baseline(args.workload, args.cpu_steps)

    import torch
    import paper_2204_02107_amd as m

    sc = workload(args.workload)
    forms = [args.precision] + ([] if args.one_form else [("fp32" if args.precision == "fp64" else "fp64")])
    res = {}
    for form in forms:
        res[form] = measure(sc, m.FP64 if form == "fp64" else m.FP32_REFINE, args, form)
    head = res[args.precision]
    dom = head["dominant"]
    achieved = head["dominant_GBs"]
    out = {
        "metric": "Gcell-steps/s (full step incl. FFT Poisson)",
        "value": head["value"],
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 (FP64 refinement and reductions)",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.workload] + (", FP64" if args.precision == "fp64" else ", FP32 + FP64 refinement")
                        + (", projection after every RK4 stage" if args.per_stage else ""),
            "cells": sc.ncells,
            "forced_cells": int(len(sc.forced_idx)),
        },
        "step_bytes_per_cell": head["step_bytes_per_cell"],
        "hbm_frac_end_to_end": head["hbm_frac_end_to_end"],
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_of(args.workload, args.precision, dom),
            "avg_us": head["dominant_avg_us"],
            "schedule": "every launch alone on one stream (dnslab_set_overlap 0), HIP events around each launch",
        },
        "kernels": head["kernels"],
        "kernels_alone": head["kernels_alone"],
    }
    for form in forms[1:]:
        r = res[form]
        out["fp32_refine" if form == "fp32" else "fp64"] = {
            "value": r["value"], "unit": "Gcell-steps/s", "ms_per_step": r["ms_per_step"],
            "step_bytes_per_cell": r["step_bytes_per_cell"], "hbm_frac_end_to_end": r["hbm_frac_end_to_end"],
            "roofline": {"kernel": r["dominant"], "achieved": r["dominant_GBs"],
                         "frac": r["dominant_GBs"] / HBM_PEAK_GBS, "avg_us": r["dominant_avg_us"],
                         "traffic": traffic_of(args.workload, form, r["dominant"])},
            "kernels": r["kernels"], "kernels_alone": r["kernels_alone"],
        }
    if not args.no_particles:
        S = m.Solver(sc, precision=m.FP64 if args.precision == "fp64" else m.FP32_REFINE)
        S.step(args.warmup, diag=False)
        out["particles"] = particle_bench(S, sc, 8 if args.precision == "fp64" else 4)
        S.close()
        del S
        torch.cuda.empty_cache()
        print("[bench] particles: " + json.dumps(out["particles"]), file=sys.stderr, flush=True)
    if args.serving != "none":
        n_req, n_steps = (16, 300) if args.serving == "short" else (64, 2000)
        pols = SERVING_POLICIES if args.serving == "config4-all" else ("pool_fp32_refine", "fifo_fp64")
        runs = []
        for seed in args.serving_seeds:
            print(f"[bench] serving stream {n_req} x {n_steps}, seed {seed} ...", file=sys.stderr, flush=True)
            runs.append(serving_bench(n_req, n_steps, budget_gib=1.0, seed=seed, policies=pols,
                                      log=lambda msg: print("[serving] " + msg, file=sys.stderr, flush=True)))
        out["serving"] = runs[0] if len(runs) == 1 else runs
    if cpu_proc is not None:
        print("[bench] waiting for the CPU oracle ...", file=sys.stderr, flush=True)
        # bounded: the whole run stays within about 9 minutes
        cb = finish_cpu_baseline(cpu_proc, args.workload, 540.0 - (time.perf_counter() - t_start))
        if cb is not None:
            out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
