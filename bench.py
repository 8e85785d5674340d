#!/usr/bin/env python3
"""Benchmark of the fused MD + MDLG coarse-graining step on one MI355X.

Workload: 2D Lennard-Jones gas, N = 1,048,576 particles at area fraction
0.0784 and kT = 20 (box L = sqrt(N pi / (4 phi)) = 3241.06 sigma), FP64,
dt = 1e-4, MDLG lattice 1024 x 1024 (dx = 3.165 sigma), coarse step of 50 MD
steps, D2Q49 counts.  Inputs are synthetic (jittered grid, Maxwellian
velocities; seed 0).

One benchmark step = one coarse time step: s_cg MD steps, each one fused
force + velocity-Verlet kernel, the last one also evaluating the coarse-
graining event, plus the cell-list rebuilds on their schedule, replayed from
captured HIP graphs: one cell-list interval in every SAMPLE_EVERY (8) as three
graphs with HIP events between them (the kernel times of the same run), the
others as one graph each (a graph boundary costs the device ~15 us, so
splitting every interval would cost the job ~5%).  `value` is particle-steps/s
of the whole job, with the state resident in HBM.

Prints one JSON line.  --gpus above 1 is not supported (one GPU per box).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MD particle-steps/s + MDLG cell-updates/s (1M LJ, φ=0.0784), f_eq err vs FP64"
HBM_PEAK_GBS = 8000.0
STEP_BYTES = 64.0        # read + write x, v (FP64) per particle-step
CG_BYTES = 40.0          # snapshot read + write (32) + one counter read-modify-write (8) per particle-event


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed coarse steps per repetition")
    ap.add_argument("--warmup", type=int, default=3, help="untimed coarse steps (before the timed warm-up)")
    ap.add_argument("--warmup-seconds", type=float, default=0.5, help="sustained stepping before timing")
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions (the median is reported)")
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--phi", type=float, default=0.0784)
    ap.add_argument("--kT", type=float, default=20.0)
    ap.add_argument("--lx", type=int, default=1024)
    ap.add_argument("--s-cg", type=int, default=50)
    ap.add_argument("--force-bits", type=int, default=64, choices=(64, 32))
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--skin", type=float, default=0.0)
    ap.add_argument("--step-kernel", type=int, default=0)
    ap.add_argument("--gather-batch", type=int, default=0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--coarse-sweep", type=int, default=1, help="also time coarse steps of 10 and 200 MD steps")
    ap.add_argument("--cpu-baseline-steps", type=int, default=500,
                    help="MD steps of the oracle sample (0 disables the CPU baseline)")
    ap.add_argument("--workload", default="single", choices=("single", "batched", "precision", "surrogate", "paper", "neq"),
                    help="single: the 1M box; batched: 256 uneven replicas in one launch per step; "
                         "precision: FP32 pair forces against FP64 on the 4M box")
    ap.add_argument("--seeds", type=int, default=4, help="precision: seeds")
    ap.add_argument("--precision-steps", type=int, default=10000, help="precision: MD steps per run")
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--train-steps", type=int, default=200000, help="surrogate: Adam steps")
    ap.add_argument("--train-batch", type=int, default=2048, help="surrogate: minibatch")
    ap.add_argument("--groups", type=int, default=4, help="surrogate: replica groups (80 replicas each)")
    ap.add_argument("--paper-replicas", type=int, default=4, help="paper: independent systems of 99,856 particles")
    ap.add_argument("--events", type=int, default=20, help="paper: coarse-graining events per Table 1 row (2000 in the paper)")
    ap.add_argument("--equil", type=int, default=1000000, help="paper: MD steps discarded before the sweep")
    ap.add_argument("--rows", default="", help="paper: comma-separated Table 1 rows (0-11); default all")
    ap.add_argument("--paper-rc", type=float, default=2.5,
                    help="paper: LJ cutoff in sigma (energy-shifted); 2^(1/6) gives the purely repulsive WCA potential")
    ap.add_argument("--stop-at", type=int, default=0, help="paper: stop the sweep before this MD step (0: run to the end)")
    ap.add_argument("--checkpoint", default="", help="paper: write state and accumulators here when stopping early")
    ap.add_argument("--resume", default="", help="paper: continue the sweep from a checkpoint")
    ap.add_argument("--crosscheck", type=int, default=1, help="paper: one coarse step of row 0 by the oracle too")
    ap.add_argument("--neq-replicas", type=int, default=256, help="neq: ensemble size")
    ap.add_argument("--neq-events", type=int, default=100, help="neq: coarse steps recorded")
    ap.add_argument("--pdf-out", default="", help="paper: write the binned displacement PDFs and K(X_i) here (JSON)")
    ap.add_argument("--autotune", action="store_true", help="batched: tune the launch first (lj_md_autotune)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (bandwidth and counter calibration)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_fused3_1M_phi0.0784.traffic.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2101_01160_amd", "csrc", "md.hip")


def source_sha256():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(n, spl):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    same counter reads for a plain copy of known size), or None when the
    summary is missing, for another workload or kernel, or older than the
    kernel source."""
    try:
        kv = {}
        for ln in open(TRAFFIC_FILE):
            if ":" in ln and not ln.startswith("#"):
                k, v = ln.split(":", 1)
                kv[k.strip()] = v.strip()
        if (kv.get("source_sha256") != source_sha256() or int(kv.get("n", -1)) != n
                or int(kv.get("steps_per_launch", -1)) != spl):
            return None
        fetch = float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"]) * 1024.0
        write = float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"]) * 1024.0
        return fetch + write
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration(mib):
    import torch
    a = torch.empty(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_mib": mib, "read_bytes": mib << 20, "write_bytes": mib << 20, "us_per_copy": ms * 1e3,
                      "gb_per_s_read_plus_write": 2 * (mib << 20) / (ms * 1e-3) / 1e9}), flush=True)


def host_cpu():
    """CPU model and the number of cores this process may use."""
    model = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, int(os.cpu_count() or 1), int(usable)


def _oracle_sample(job):
    """One oracle run (single-threaded FP64 C) on its own seeded sample; returns
    (seconds, counts, events).  Runs in a worker process for the all-cores leg."""
    n, phi, kT, lx, s_cg, seed, steps = job
    import mdlg_inputs as mi
    from oracle import md as omd
    pos, vel, L = mi.initial_state(n, phi, kT, seed)
    acc = omd.CGAccum(lx)
    t0 = time.perf_counter()
    omd.md_run(pos, vel, np.zeros((n, 2), np.int64), L, steps, cg=acc, s_cg=s_cg)
    return time.perf_counter() - t0, acc.counts.copy(), acc.events


def cpu_baseline(n, phi, kT, lx, s_cg, seed, steps, all_core_steps=None, max_procs=16):
    """The oracle (single-threaded FP64 C, as it stands) on bounded samples of the
    same workload: one core on the benchmark's seed, then one independent sample
    per usable host core (seeds seed+1 ..) in parallel processes.  `value` is
    the all-cores aggregate.  Also returns the one-core run's counts, the
    reference of the f_eq comparison."""
    import multiprocessing as mp
    model, nproc, usable = host_cpu()
    dt1, counts, events = _oracle_sample((n, phi, kT, lx, s_cg, seed, steps))
    one = {"value": n * steps / dt1, "unit": "particle-steps/s", "cores": 1,
           "sample": f"{n} particles x {steps} MD steps with {events} coarse-graining events "
                     f"(s_cg={s_cg}, lx={lx}), {dt1:.1f} s on one host core"}
    procs = max(1, min(max_procs, usable))
    steps_all = all_core_steps or max(s_cg, steps // 2)
    jobs = [(n, phi, kT, lx, s_cg, seed + 1 + i, steps_all) for i in range(procs)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_oracle_sample, jobs)
    wall = time.perf_counter() - t0
    busy = max(r[0] for r in res)
    out = {"value": procs * n * steps_all / busy, "unit": "particle-steps/s", "cores": procs, "kind": "oracle",
           "sample": f"{procs} processes, each {n} particles x {steps_all} MD steps (s_cg={s_cg}, lx={lx}) on its own "
                     f"seed; slowest {busy:.1f} s, wall {wall:.1f} s",
           "one_core": one, "cpu_model": model, "nproc": nproc, "usable_cores": usable}
    return out, counts, events


def gpu_feq_vs_oracle(m, torch, pos0, vel0, L, lx, s_cg, steps, force_bits, ocounts, oevents):
    """Measured f_eq of the GPU run against the oracle's from the same initial
    state over the same steps: max_i |g_i(GPU) - g_i(oracle)| and whether the
    integer counts are identical."""
    n = pos0.shape[0]
    sysm = m.LJSystem(torch.from_numpy(pos0).cuda(), torch.from_numpy(vel0).cuda(), box_l=L, force_bits=force_bits)
    acc = sysm.attach_cg(lx, s_cg)
    sysm.step(steps)
    sysm.check()
    counts = acc.counts.cpu().numpy()[0]
    events = acc.events
    sysm.close()
    g, _ = m.mdlg_feq_measured(counts, n, events)
    go, _ = m.mdlg_feq_measured(ocounts, n, oevents)
    return {"max_abs_dg": float(np.max(np.abs(g - go))), "counts_identical": bool(np.array_equal(counts, ocounts)),
            "events": int(events), "md_steps": int(steps),
            "reference": "the oracle (FP64 CPU) from the same initial state"}


SAMPLE_EVERY = 8  # cell-list intervals per timed sample (split into three graphs)


def sample_every(units):
    return max(1, min(SAMPLE_EVERY, units // 3))


def timed_reps(sysm, units, reps, torch):
    """`reps` repetitions of `units` cell-list intervals, each bracketed by HIP
    events on the launch stream (every sample_every(units)-th interval split
    into three graphs for the kernel times); returns [(ms, kernel ms [3],
    launches [3])]."""
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        kms, kcnt = sysm.step_timed(units, sample_every(units))
        e1.record()
        torch.cuda.synchronize()
        out.append((e0.elapsed_time(e1), [float(x) for x in kms], [int(x) for x in kcnt]))
    return out


def warm(sysm, units, seconds, torch):
    """Replay intervals until `seconds` of sustained stepping have passed (the
    clocks of a loaded GPU settle below those of a short burst)."""
    t0 = time.perf_counter()
    while True:
        sysm.step_timed(units, sample_every(units))
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            return time.perf_counter() - t0


def median_rep(rows):
    order = sorted(range(len(rows)), key=lambda i: rows[i][0])
    return rows[order[len(order) // 2]]


def bench_single(args):
    """The headline workload (see the module docstring)."""
    n, phi, kT, lx, s_cg = args.n, args.phi, args.kT, args.lx, args.s_cg
    import mdlg_inputs as mi
    pos0, vel0, L = mi.initial_state(n, phi, kT, args.seed)
    dxl = L / lx
    base = None
    if args.cpu_baseline_steps > 0:
        # host-only work first, before this process touches the GPU
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        base, ocounts, oevents = cpu_baseline(n, phi, kT, lx, s_cg, args.seed, args.cpu_baseline_steps)
        print(f"# cpu baseline: {base['value']:.3e} particle-steps/s on {base['cores']} cores", file=sys.stderr,
              flush=True)

    import torch

    import paper_2101_01160_amd as m
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    kw = dict(force_bits=args.force_bits, block_size=args.block_size, skin=args.skin,
              step_kernel=args.step_kernel, gather_batch=args.gather_batch)
    sysm = m.LJSystem(torch.from_numpy(pos0).to(dev), torch.from_numpy(vel0).to(dev), box_l=L, **kw)
    acc = sysm.attach_cg(lx, s_cg)
    info = sysm.info()
    K = info["rebuild_every"]
    print(f"# init done: n={n} L={L:.3f} lx={lx} s_cg={s_cg} cells/side={info['cells_per_side']} "
          f"rebuild_every={K} block={info['block_size']}", file=sys.stderr, flush=True)
    # warm-up: W coarse steps of captured intervals (every graph variant), then
    # sustained stepping; the accumulators restart afterwards, so that the f_eq
    # statistics come from the timed repetitions, long after the grid start
    units = max(3, math.ceil(args.steps * s_cg / K))
    sysm.step_timed(max(4, math.ceil(args.warmup * s_cg / K)))
    warm_s = warm(sysm, units, args.warmup_seconds, torch)
    acc.counts.zero_()
    acc.moments.zero_()
    ev0 = acc.events
    steps_before = sysm.info()["steps_done"]
    reps = timed_reps(sysm, units, args.reps, torch)
    sysm.check()
    events = acc.events - ev0
    md_steps = units * K
    ms, kms, kcnt = median_rep(reps)
    value = n * md_steps / (ms * 1e-3)
    print(f"# timed {args.reps} x {md_steps} MD steps after {warm_s:.2f} s of warm-up: median {ms:.2f} ms "
          f"(all: {', '.join(f'{r[0]:.2f}' for r in reps)})", file=sys.stderr, flush=True)
    t_step, t_cg, t_rebuild = kms
    spl = int(info.get("steps_per_launch", 1)) or 1
    launch_ms = spl * t_step
    launch_bytes = spl * STEP_BYTES * n
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(n, spl) if args.force_bits == 64 and args.step_kernel in (0, 3) else None

    counts = acc.counts.cpu().numpy()[0]
    moments = acc.moments.cpu().numpy()[0]
    g, ovf = m.mdlg_feq_measured(counts, n, events)
    mu2, mu4, a2 = m.mdlg_moments(moments, dxl)
    lam, r = m.mdlg_lambda_from_moments(mu2, mu4, 2)
    gG = m.mdlg_feq_gauss(a2)
    gW = m.mdlg_feq_wsg(a2, lam)
    sysm.close()

    # the coarse-graining's share: the same intervals (same rebuild interval)
    # without coarse-graining, and with the per-cell field n_i(x) accumulated
    print("# reference runs: no coarse-graining; per-cell field", file=sys.stderr, flush=True)
    ref = m.LJSystem(torch.from_numpy(pos0).to(dev), torch.from_numpy(vel0).to(dev), box_l=L, rebuild_every=K, **kw)
    ref.step_timed(4)
    warm(ref, units, args.warmup_seconds, torch)
    ms_plain = median_rep(timed_reps(ref, units, args.reps, torch))[0]
    cacc = ref.attach_cg(lx, s_cg, cell_acc=True)
    ref.step_timed(4)
    ev1 = cacc.events
    ms_cell = median_rep(timed_reps(ref, units, args.reps, torch))[0]
    ev_cell = (cacc.events - ev1) // args.reps
    ref.check()
    ref.close()
    ev_rep = events // args.reps
    over_ev = (ms - ms_plain) / max(ev_rep, 1)         # ms per coarse-graining event (counts and moments)
    over_cell = (ms_cell - ms_plain) / max(ev_cell, 1)  # ms per event with the per-cell field written

    # the other coarse steps of the workload (10 and 200 MD steps), same system size
    other = {}
    for sc in (10, 200):
        if sc == s_cg or not args.coarse_sweep:
            continue
        print(f"# coarse step {sc}", file=sys.stderr, flush=True)
        o = m.LJSystem(torch.from_numpy(pos0).to(dev), torch.from_numpy(vel0).to(dev), box_l=L, **kw)
        o.attach_cg(lx, sc)
        Ks = o.info()["rebuild_every"]
        u = max(3, math.ceil(args.steps * s_cg / Ks))
        o.step_timed(max(4, math.ceil(2 * sc / Ks)))
        warm(o, u, 0.5 * args.warmup_seconds, torch)
        mo, km, _ = median_rep(timed_reps(o, u, args.reps, torch))
        o.check()
        o.close()
        other[str(sc)] = {"particle_steps_per_s": n * u * Ks / (mo * 1e-3), "us_per_md_step": mo * 1e3 / (u * Ks),
                          "rebuild_every": Ks, "kernel_ms": {"step": km[0], "step_with_cg_event": km[1],
                                                             "rebuild": km[2]}}

    feq_err = None
    if base is not None:
        print("# f_eq against the oracle's run", file=sys.stderr, flush=True)
        feq_err = gpu_feq_vs_oracle(m, torch, pos0, vel0, L, lx, s_cg, args.cpu_baseline_steps, args.force_bits,
                                    ocounts, oevents)

    launch_s = launch_ms * 1e-3
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms * s_cg / md_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.force_bits == 64 else "f64 state, f32 pair forces",
        "data": "synthetic (jittered-grid positions, Maxwellian velocities, seed %d)" % args.seed,
        "config": {"workload": f"2D LJ gas N={n}, phi={phi}, kT={kT}, L={L:.3f}, dt=1e-4, "
                               f"lattice {lx}x{lx}, coarse step {s_cg} MD steps, D2Q49 counts",
                   "n": n, "phi": phi, "kT": kT, "box_l": L, "lx": lx, "s_cg": s_cg,
                   "md_steps_per_step": s_cg, "force_bits": args.force_bits,
                   "cells_per_side": info["cells_per_side"], "rebuild_every": K,
                   "block_size": info["block_size"]},
        "timing": {"repetitions": args.reps, "md_steps_per_repetition": md_steps,
                   "ms_per_repetition": [r_[0] for r_ in reps], "value_from": "median repetition",
                   "split_interval_every": sample_every(units),
                   "warmup_s": warm_s, "steps_before_timing": int(steps_before)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "frac_kind": ("algorithmic-equivalent: 64 B per particle-step (x, v read and written) times the "
                                   "steps of one launch over the launch time; a launch that advances several steps "
                                   "keeps the steps between its first load and last store on chip, so this figure "
                                   "is not bounded by 1"),
                     "kernel": (f"MD step kernel, {spl} ordinary steps per launch" if spl > 1 else
                                "MD step kernel (no coarse-graining event)"),
                     "kernel_ms": launch_ms, "bytes_per_launch": launch_bytes, "steps_per_launch": spl,
                     "hbm_counter_gbs": (traffic / launch_s / 1e9) if traffic else None,
                     "hbm_counter_frac": (traffic / launch_s / 1e9 / HBM_PEAK_GBS) if traffic else None,
                     "hbm_counter_bytes_per_particle_step": (traffic / (spl * n)) if traffic else None},
        "us_per_md_step": ms * 1e3 / md_steps,
        "kernel_ms": {"step": t_step, "step_with_cg_event": t_cg, "rebuild": t_rebuild, "launches": kcnt,
                      "meaning": "step: per ordinary MD step; step_with_cg_event: per coarse-graining event, the "
                                 "graph holding it less its ordinary steps at the per-step rate; rebuild: per "
                                 "cell-list interval"},
        "coarse_graining": {
            "events_per_repetition": ev_rep,
            "us_per_event": over_ev * 1e3,
            "us_per_event_with_cell_field": over_cell * 1e3,
            "particles_binned_per_s": n / (over_ev * 1e-3) if over_ev > 0 else None,
            "cell_updates_per_s": lx * lx / (over_cell * 1e-3) if over_cell > 0 else None,
            "method": ("time of the same intervals with the coarse-graining attached minus without it (same rebuild "
                       "interval), per event; cell updates: every one of the lx^2 cells gets its n_i(x) added to "
                       "the per-cell field (cell_acc) at each event")},
        "other_coarse_steps": other,
        "feq": {"events": int(events), "a2": a2, "r": r, "lambda2": lam, "overflow": ovf,
                "g0": float(g[0]), "max_abs_meas_minus_gauss": float(np.max(np.abs(g - gG))),
                "max_abs_meas_minus_wsg": float(np.max(np.abs(g - gW))),
                "statistics_from": (f"the timed repetitions only, after {int(steps_before)} MD steps from the grid "
                                    f"start (whose spacing equals the lattice cell)"),
                "feq_err_vs_fp64_oracle": feq_err["max_abs_dg"] if feq_err else None,
                "feq_err_check": feq_err},
    }
    if base is not None:
        line["cpu_baseline"] = base
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described, not built)"}))
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "precision":
        bench_precision(args)
        return
    if args.workload == "surrogate":
        bench_surrogate(args)
        return
    if args.workload == "paper":
        bench_paper(args)
        return
    if args.workload == "neq":
        bench_neq(args)
        return
    bench_single(args)


def bench_precision(args):
    """FP32 pair arithmetic (FP64 state, integration, wrap and sums) against the
    all-FP64 run from the same initial state: energy and momentum drift, the
    measured f_eq difference, and throughput, over several seeds."""
    import torch

    import mdlg_inputs as mi
    import paper_2101_01160_amd as m

    n = 1 << 22 if args.n == (1 << 20) else args.n
    lx = 2048 if args.lx == 1024 else args.lx
    s_cg, md_steps = args.s_cg, args.precision_steps
    dev = torch.device("cuda:0")
    rows = []
    for seed in range(args.seeds):
        pos0, vel0, L = mi.initial_state(n, args.phi, args.kT, seed)
        res = {}
        for bits in (64, 32):
            sysm = m.LJSystem(torch.from_numpy(pos0).to(dev), torch.from_numpy(vel0).to(dev), box_l=L,
                              force_bits=bits, block_size=args.block_size, skin=args.skin,
                              step_kernel=args.step_kernel)
            e_start = sysm.energy()[0]
            acc = sysm.attach_cg(lx, s_cg)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            sysm.step(md_steps)
            e1.record()
            torch.cuda.synchronize()
            sysm.check()
            ms = e0.elapsed_time(e1)
            e_end = sysm.energy()[0]
            g, _ = m.mdlg_feq_measured(acc.counts.cpu().numpy()[0], n, acc.events)
            res[bits] = {"rate": n * md_steps / (ms * 1e-3), "g": g,
                         "energy_drift": ((e_end[0] + e_end[1]) - (e_start[0] + e_start[1])) / e_start[0],
                         "momentum_drift": float(np.hypot(e_end[2] - e_start[2], e_end[3] - e_start[3]))}
            sysm.close()
        rows.append(res)
        print(f"# seed {seed}: fp64 {res[64]['rate']:.3e}, fp32 {res[32]['rate']:.3e} particle-steps/s, "
              f"max|dg| {np.max(np.abs(res[32]['g'] - res[64]['g'])):.2e}", file=sys.stderr, flush=True)
    dg = np.array([np.max(np.abs(r[32]["g"] - r[64]["g"])) for r in rows])
    g64 = np.array([r[64]["g"] for r in rows])
    se_seed = float(np.max(np.std(g64, axis=0, ddof=1) / np.sqrt(len(rows)))) if len(rows) > 1 else None
    out = {
        "metric": "FP32 pair forces vs FP64: particle-steps/s and f_eq difference", "unit": "particle-steps/s",
        "value": float(np.mean([r[32]["rate"] for r in rows])),
        "fp64_value": float(np.mean([r[64]["rate"] for r in rows])),
        "n_gpus": 1, "steps": md_steps, "warmup": 0, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 state, f32 pair forces", "data": "synthetic",
        "config": {"workload": f"2D LJ gas N={n}, phi={args.phi}, kT={args.kT}, {md_steps} MD steps, lattice "
                               f"{lx}x{lx}, coarse step {s_cg}, seeds 0..{args.seeds - 1}"},
        "feq_max_abs_fp32_minus_fp64": {"per_seed": dg.tolist(), "mean": float(dg.mean())},
        "feq_seed_standard_error_max": se_seed,
        "energy_drift_rel": {"fp64": [r[64]["energy_drift"] for r in rows], "fp32": [r[32]["energy_drift"] for r in rows]},
        "momentum_drift_abs": {"fp64": [r[64]["momentum_drift"] for r in rows],
                               "fp32": [r[32]["momentum_drift"] for r in rows]},
    }
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """Replica sweep: R systems of uneven size stepped together (one kernel per
    MD step over all of them, one graph per cell-list interval), against the
    same systems run one after another."""
    import torch

    import mdlg_inputs as mi
    import paper_2101_01160_amd as m

    s_cg = args.s_cg
    specs = mi.replica_sweep(args.replicas)
    states = [mi.initial_state(sp.n, sp.phi, sp.kT, sp.seed) for sp in specs]
    pos = np.concatenate([st[0] for st in states])
    vel = np.concatenate([st[1] for st in states])
    ntot = int(pos.shape[0])
    kw = dict(force_bits=args.force_bits, block_size=args.block_size, skin=args.skin,
              step_kernel=args.step_kernel, gather_batch=args.gather_batch)
    params = [m.lj_params(sp.n, sp.L, **kw) for sp in specs]
    dev = torch.device("cuda:0")
    tpos, tvel = torch.from_numpy(pos).to(dev), torch.from_numpy(vel).to(dev)
    tuned = None
    bparams = params
    if args.autotune:
        lats = [m.Lattice(lx=sp.lx, reserved=0) for sp in specs]
        t0 = time.perf_counter()
        bparams, us = m.lj_md_autotune(params, tpos, tvel, s_cg, lats, use_cache=False)
        tuned = {"seconds": time.perf_counter() - t0, "best_us_per_md_step": us,
                 "step_kernel": bparams[0].step_kernel, "block_size": bparams[0].block_size,
                 "skins": sorted({round(p.skin, 3) for p in bparams})}
        print(f"# autotune: {tuned}", file=sys.stderr, flush=True)
    batch = m.LJSystem(tpos, tvel, params=bparams)
    acc = batch.attach_cg([sp.lx for sp in specs], s_cg)
    info = batch.info()
    print(f"# batch: {len(specs)} replicas, {ntot} particles, rebuild_every={info['rebuild_every']}",
          file=sys.stderr, flush=True)
    batch.step(args.warmup * s_cg)
    torch.cuda.synchronize()
    md_steps = args.steps * s_cg
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    batch.step(md_steps)
    e1.record()
    torch.cuda.synchronize()
    batch.check()
    ms_batch = e0.elapsed_time(e1)
    bcounts = acc.counts.cpu().numpy()
    batch.close()
    # the same replicas one by one, same steps
    ms_seq = 0.0
    max_dg = 0.0
    for r, (sp, st) in enumerate(zip(specs, states)):
        single = m.LJSystem(torch.from_numpy(st[0]).to(dev), torch.from_numpy(st[1]).to(dev), params=[params[r]])
        sacc = single.attach_cg(sp.lx, s_cg)
        single.step(args.warmup * s_cg)
        torch.cuda.synchronize()
        e0.record()
        single.step(md_steps)
        e1.record()
        torch.cuda.synchronize()
        single.check()
        ms_seq += e0.elapsed_time(e1)
        ev = sacc.events
        g1, _ = m.mdlg_feq_measured(bcounts[r], sp.n, ev)
        g2, _ = m.mdlg_feq_measured(sacc.counts.cpu().numpy()[0], sp.n, ev)
        max_dg = max(max_dg, float(np.max(np.abs(g1 - g2))))  # 0 when the launch matches
        single.close()
    rate_b = ntot * md_steps / (ms_batch * 1e-3)
    rate_s = ntot * md_steps / (ms_seq * 1e-3)
    print(json.dumps({
        "metric": "batched replicas: aggregate particle-steps/s", "value": rate_b, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batch / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.force_bits == 64 else "f64 state, f32 pair forces", "data": "synthetic",
        "config": {"workload": f"{len(specs)} replicas, N log-uniform in [4096, 262144] (total {ntot}), "
                               f"phi in (0.0784, 0.2, 0.4) x kT in (1, 5, 20), lattice cell ~2 sigma, "
                               f"coarse step {s_cg}", "md_steps_per_step": s_cg,
                   "rebuild_every": info["rebuild_every"]},
        "one_by_one": {"value": rate_s, "ms_total": ms_seq, "speedup_of_batch": rate_b / rate_s,
                       "path": "each replica alone, default FP64 launch"},
        "autotune": tuned,
        "feq_max_abs_batch_minus_single": max_dg}), flush=True)


MLP_FLOP_PER_SAMPLE = 2.0 * (6 * 256 + 256 * 256 * 2 + 256 * 49)  # forward products


def bench_surrogate(args):
    """Surrogate f_eq: GPU-generated MDLG data (batched MD + trajectory
    coarse-graining), training on the GPU, held-out errors against measured
    f_eq and the WSG closed form, inference throughput on the matrix cores,
    and the cost of the same f_eq values by molecular dynamics."""
    import torch

    import paper_2101_01160_amd as m
    from paper_2101_01160_amd import surrogate as S

    log = lambda s: print("# " + s, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    data = S.generate(n_groups=args.groups, reps_per_group=80, n=65536, n_snap=201, equil=2000, log=log)
    t_gen = time.perf_counter() - t0
    tr, va, te = S.split_by_replica(data)
    net, hist = S.train(data, tr, steps=args.train_steps, batch=args.train_batch, val_idx=va,
                        val_every=max(1, args.train_steps // 8), log=log, average_tail=0.3)
    table = S.moment_table(data, tr, box=S.parameter_box(data))
    res = S.evaluate(net, data, te, with_guard=True, table=table)
    log(f"held-out: {res}")
    # the guard without a trajectory through the C entry point on a sample of
    # held-out points: same rule as the batched evaluation
    sample = te[:: max(1, len(te) // 64)]
    agree = 0
    t_guard = time.perf_counter()
    for i in sample:
        g, fb, err, _, _ = net.feq_table(data.X[i], table, tol=1e-3)
        agree += int(fb == (err > 1e-3))
    us_guard = (time.perf_counter() - t_guard) / len(sample) * 1e6
    # inference throughput: one launch sequence for a large batch, HIP events
    B = 65536
    big = m.SurrogateMLP(net.params(), B)
    xb = torch.from_numpy(np.resize(data.X[te], (B, 6)).astype(np.float32)).cuda()
    out = torch.empty((B, 49), dtype=torch.float32, device="cuda")
    for _ in range(3):
        m.mdlg_mlp_forward(big.handle, xb, out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = max(1, args.steps // 5)
    e0.record()
    for _ in range(reps):
        m.mdlg_mlp_forward(big.handle, xb, out)
    e1.record()
    torch.cuda.synchronize()
    ms_inf = e0.elapsed_time(e1) / reps
    tflops = MLP_FLOP_PER_SAMPLE * B / (ms_inf * 1e-3) / 1e12
    # training step time (GPU work plus launch overhead), fixed batch
    x4 = torch.from_numpy(data.X[tr[:args.train_batch]].astype(np.float32)).cuda()
    r4 = torch.from_numpy(data.G[tr[:args.train_batch]].astype(np.float32)).cuda()
    lbuf = torch.zeros(1, dtype=torch.float32, device="cuda")
    probe = m.SurrogateMLP(net.params(), args.train_batch)
    for _ in range(3):
        probe.train_step(x4, r4, 1e-6, lbuf)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(50):
        probe.train_step(x4, r4, 1e-6, lbuf)
    e1.record()
    torch.cuda.synchronize()
    us_train = e0.elapsed_time(e1) / 50 * 1e3
    # MD route to the same f_eq values: particle-steps per sample of the generator
    steps_per_sample = data.timing["particle_steps"] / len(data)
    sec_md_per_sample = (data.timing["md_s"] + data.timing["cg_s"]) / len(data)
    sec_nn_per_sample = ms_inf * 1e-3 / B
    rate = B / (ms_inf * 1e-3)
    print(json.dumps({
        "metric": "surrogate f_eq evaluations/s (6 -> 256x3 -> 49, BF16 MFMA)", "value": rate,
        "unit": "f_eq/s", "n_gpus": 1, "steps": reps, "warmup": 3, "ms_per_step": ms_inf,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16 (fp32 accumulate)",
        "data": "synthetic (GPU MD of random-init LJ gases)",
        "config": {"workload": f"{len(data)} samples: {args.groups * 80} replicas x 65536 particles, "
                               f"phi~U(0.05,0.4), kT~U(1,20), 10 coarse times 10..200 MD steps, 16 drifts |u|<=0.2; "
                               f"inference batch {B}", "train_steps": args.train_steps,
                   "train_batch": args.train_batch},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": tflops / 2500.0, "traffic": None},
        "heldout": res, "guard_agreement": agree / len(sample), "guard_call_us": us_guard,
        "timing": {"generate_s": t_gen, "md_s": data.timing["md_s"], "coarse_grain_s": data.timing["cg_s"],
                   "train_s": hist["train_s"], "train_step_us": us_train, "inference_us_per_batch": ms_inf * 1e3},
        "gain": {"md_particle_steps_per_feq": steps_per_sample, "md_seconds_per_feq": sec_md_per_sample,
                 "surrogate_seconds_per_feq": sec_nn_per_sample,
                 "speedup": sec_md_per_sample / sec_nn_per_sample,
                 "equivalent_particle_steps_per_s": steps_per_sample * rate}}), flush=True)


# Table 1: coarse-grained time step dt_cg (tau), lattice spacing dx (sigma), lattice points lx, MD output
# frequency (MD steps of 1e-4 tau per coarse step).  The 5.5 / 180 row is taken as printed; the lattice
# always has lx cells over L, so its spacing is L / lx.
TABLE1 = [(0.3911, 4.0, 250, 3911), (0.5000, 5.0, 200, 5000), (0.5626, 5.5, 180, 5626),
          (0.6927, 20.0 / 3.0, 150, 6927), (0.9009, 25.0 / 3.0, 120, 9009), (1.1261, 10.0, 100, 11261),
          (1.4994, 12.5, 80, 14994), (1.6342, 40.0 / 3.0, 75, 16342), (2.0338, 15.625, 64, 20338),
          (2.9280, 20.0, 50, 29280), (4.1821, 25.0, 40, 41821), (6.1751, 31.25, 32, 61751)]
PAPER_N, PAPER_L, PAPER_KT, PAPER_A2 = 99856, 1000.0, 20.0, 0.1611
# D2Q25 sets of the Results section and the outer ring of D2Q49
SHELLS = {"f0": [0], "f1-4": [1, 2, 3, 4], "f5-8": [5, 6, 7, 8], "f9-12": [9, 10, 11, 12],
          "f13-20": list(range(13, 21)), "f21-24": [21, 22, 23, 24], "f25-48": list(range(25, 49))}


def _row_results(m, R, L, E_done, rows_state, t_t, c_t, n_bin):
    """Per Table 1 row: a^2, r, lambda, measured f_eq against G and WSG per
    D2Q25 set, and the KL divergences of the binned displacement PDF."""
    out_rows, pdfs = [], []
    for ri in sorted(rows_state):
        st = rows_state[ri]
        dt_cg, dx_print, lx, freq = TABLE1[ri]
        dxl = L / lx
        events = int(st["events"])
        if events == 0:
            continue
        counts, moments, hist = st["counts"], st["moments"], st["hist"]
        ntot = R * PAPER_N
        c = counts.sum(axis=0)
        g, ovf = m.mdlg_feq_measured(c, ntot, events, symmetrize=True)
        mu2, mu4, a2 = m.mdlg_moments(moments.sum(axis=0), dxl)
        lam, r = m.mdlg_lambda_from_moments(mu2, mu4, 2)
        gG, gW = m.mdlg_feq_gauss(a2), m.mdlg_feq_wsg(a2, lam)
        shells = {}
        for name, idx in SHELLS.items():
            cnt = float(c[idx].sum())
            gm, gg, gw = float(g[idx].mean()), float(gG[idx].mean()), float(gW[idx].mean())
            shells[name] = {"meas": gm, "G": gg, "WSG": gw, "meas/G-1": gm / gg - 1.0, "meas/WSG-1": gm / gw - 1.0,
                            "WSG/G-1": gw / gg - 1.0, "poisson_se": 1.0 / math.sqrt(cnt) if cnt > 0 else None}
        rep_mom = [m.mdlg_moments(moments[k], dxl) for k in range(R)]
        a2_rep = [x[2] for x in rep_mom]
        r_rep = [x[1] / (3.0 * x[0] ** 2) for x in rep_mom]
        h = dxl / 8.0
        p_md = m.mdlg_pdf_measured(hist)
        p_g, p_w = m.mdlg_pdf_bins(mu2, lam, 0.0, h, n_bin)
        k_g, d_g = m.mdlg_kl_divergence(p_md, p_g)
        k_w, d_w = m.mdlg_kl_divergence(p_md, p_w)
        _, d_wg = m.mdlg_kl_divergence(p_w, p_g)
        samples = int(hist.sum())
        _, lam_vacf = m.mdlg_lambda_vacf(t_t, c_t, dt_cg, 0.01)
        out_rows.append({"row": ri, "dt_cg": dt_cg, "lx": lx, "dx": dxl, "freq": freq, "events": events,
                         "a2": a2, "a2_replica_sd": float(np.std(a2_rep, ddof=1)) if R > 1 else None,
                         "a2_paper": PAPER_A2, "r": r, "r_replica_sd": float(np.std(r_rep, ddof=1)) if R > 1 else None,
                         "lambda2": lam, "lambda1": (1.0 / lam if lam > 0 else None),
                         "lambda_vacf": lam_vacf, "overflow": ovf,
                         "max_abs_meas_minus_G": float(np.max(np.abs(g - gG))),
                         "max_abs_meas_minus_WSG": float(np.max(np.abs(g - gW))), "shells": shells,
                         "kl": {"MD||G": d_g, "MD||WSG": d_w, "WSG||G": d_wg, "samples": samples,
                                "finite_sample_bias": (n_bin + 1) / (2.0 * samples)}})
        pdfs.append({"row": ri, "dt_cg": dt_cg, "h": h, "n_bin": n_bin, "P_MD": p_md.tolist(), "P_G": p_g.tolist(),
                     "P_WSG": p_w.tolist(), "K_MD_G": k_g.tolist(), "K_MD_WSG": k_w.tolist()})
    return out_rows, pdfs


def _displacement_moments(p0, p1, i0, i1, L):
    """mu2, mu4 (pooled over the axes) of the box-frame displacements and their
    standard errors from the spread over particles (host arithmetic of the
    comparison, not of the method)."""
    d = (p1 - p0) + L * (i1 - i0).astype(np.float64)
    d2 = (d * d).ravel()
    d4 = d2 * d2
    n = d2.size
    return (float(d2.mean()), float(d2.std(ddof=1) / math.sqrt(n)), float(d4.mean()), float(d4.std(ddof=1) / math.sqrt(n)))


def paper_oracle_crosscheck(m, torch, pos, vel, L, row=0):
    """One coarse step of Table 1's row `row` from an equilibrated state of one
    system, advanced by the GPU and by the oracle on the host: mu2, mu4 and
    r = mu4 / (3 mu2^2) of the displacements over the step, each with its
    standard error over the particles.  The two trajectories start equal and
    differ by the rounding of the force sums."""
    from oracle import md as omd
    dt_cg, _, lx, freq = TABLE1[row]
    n = pos.shape[0]
    sysm = m.LJSystem(torch.from_numpy(pos).cuda(), torch.from_numpy(vel).cuda(), box_l=L)
    t0 = time.perf_counter()
    sysm.step(freq)
    gp, _, gi = (x.cpu().numpy() for x in sysm.state())
    sysm.check()
    sysm.close()
    t_gpu = time.perf_counter() - t0
    t0 = time.perf_counter()
    op, _, oi, _ = omd.md_run(pos.copy(), vel.copy(), np.zeros((n, 2), np.int64), L, freq)  # md_run works in place
    t_orc = time.perf_counter() - t0
    z = np.zeros((n, 2), np.int64)
    g = _displacement_moments(pos, gp, z, gi, L)
    o = _displacement_moments(pos, op, z, oi, L)
    rg, ro = g[2] / (3 * g[0] ** 2), o[2] / (3 * o[0] ** 2)

    def r_se(mm):  # first-order propagation of the two standard errors
        mu2, s2, mu4, s4 = mm
        return math.sqrt((s4 / (3 * mu2 ** 2)) ** 2 + (2 * mu4 * s2 / (3 * mu2 ** 3)) ** 2)
    out = {"row": row, "md_steps": freq, "particles": n, "gpu": {"mu2": g[0], "mu2_se": g[1], "mu4": g[2],
                                                                   "mu4_se": g[3], "r": rg, "r_se": r_se(g)},
           "oracle": {"mu2": o[0], "mu2_se": o[1], "mu4": o[2], "mu4_se": o[3], "r": ro, "r_se": r_se(o)},
           "oracle_seconds": t_orc, "gpu_seconds": t_gpu,
           "max_abs_position_difference": float(np.max(np.abs((gp + L * gi) - (op + L * oi))))}
    out["within_3se"] = bool(abs(g[0] - o[0]) <= 3 * math.hypot(g[1], o[1]) and abs(g[2] - o[2]) <= 3 * math.hypot(g[3], o[3])
                             and abs(rg - ro) <= 3 * math.hypot(r_se(g), r_se(o)))
    return out


def bench_paper(args):
    """The paper's sweep: R independent systems of N = 99,856 LJ particles in
    L = 1000 at kT = 20 (Table 1's system), equilibrated for `--equil` MD steps
    and then run as one trajectory that serves every Table 1 row: row k takes
    the snapshots at multiples of its MD output frequency and coarse-grains
    each consecutive pair on its own lattice (Eq.(n_i), the standalone
    entry point, per replica), for E coarse steps per row; the displacement
    histograms of the same pairs give P^MD(X_i) of Fig. 2.  A row's E windows
    are the first E freq steps of the trajectory, so all rows cost the MD of
    the longest.  The run can stop at an MD step (--stop-at) and write a
    checkpoint (state, accumulators, the last snapshot of unfinished rows) to
    resume from (--resume).  Also: the velocity autocorrelation (lambda from
    the VACF) and one coarse step of row 0 advanced by the GPU and by the
    oracle from the same equilibrated state (mu2, mu4, r within their standard
    errors)."""
    import torch

    import mdlg_inputs as mi
    import paper_2101_01160_amd as m

    log = lambda s_: print("# " + s_, file=sys.stderr, flush=True)
    R, E, N, L, kT = args.paper_replicas, args.events, PAPER_N, PAPER_L, PAPER_KT
    rows = [int(r) for r in args.rows.split(",")] if args.rows else list(range(len(TABLE1)))
    phi = N * math.pi / (4.0 * L * L)
    ntot = N * R
    n_bin = 97                 # bins of dx / 8 over +-6 dx
    B = 20                     # snapshots per row processed per batch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    offsets = np.arange(R + 1, dtype=np.int64) * N
    t_wall0 = time.perf_counter()
    gpu_ms = {"equil": 0.0, "vacf_md": 0.0, "sweep_md": 0.0}
    if args.resume:
        ck = np.load(args.resume + ".npz", allow_pickle=False)
        meta = json.loads(str(ck["meta"]))
        sysm = m.LJSystem.load(args.resume + ".state")
        t_sweep = int(meta["t_sweep"])
        rows = meta["rows"]
        E = int(meta["E"])
        t_t, c_t, tau_vacf = np.asarray(meta["vacf_t"]), np.asarray(meta["vacf_c"]), meta["tau_vacf"]
        crosscheck, equil_info = meta["crosscheck"], meta["equil_info"]
        gpu_ms = meta["gpu_ms"]
        rows_state = {}
        for ri in rows:
            rows_state[ri] = {"events": int(ck[f"ev_{ri}"]), "counts": ck[f"counts_{ri}"], "moments": ck[f"moments_{ri}"],
                              "hist": ck[f"hist_{ri}"]}
        log(f"resumed at sweep step {t_sweep}: events {[rows_state[ri]['events'] for ri in rows]}")
    else:
        pos, vel = [], []
        for r in range(R):
            rng = np.random.Generator(np.random.PCG64(args.seed + r))
            pos.append(mi.jittered_grid(N, L, rng))
            vel.append(mi.maxwell_velocities(N, kT, rng))
        params = [m.lj_params(N, L, rc=args.paper_rc, force_bits=args.force_bits) for _ in range(R)]
        sysm = m.LJSystem(torch.from_numpy(np.concatenate(pos)).to(dev),
                          torch.from_numpy(np.concatenate(vel)).to(dev), params=params)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        left = args.equil
        while left > 0:   # in pieces, so that a long equilibration reports progress
            k = min(left, 500000)
            sysm.step(k)
            left -= k
            torch.cuda.synchronize()
            log(f"equilibration: {args.equil - left} / {args.equil} MD steps")
        e1.record()
        torch.cuda.synchronize()
        sysm.check()
        gpu_ms["equil"] = e0.elapsed_time(e1)
        equil_info = {"md_steps": args.equil, "rebuild_every": sysm.info()["rebuild_every"]}
        # one coarse step of row 0 by the GPU and by the oracle, from replica 0's equilibrated state
        crosscheck = None
        if args.crosscheck:
            p_all, v_all, _ = (x.cpu().numpy() for x in sysm.state())
            log("oracle cross-check of row 0 (one coarse step on the host) ...")
            crosscheck = paper_oracle_crosscheck(m, torch, np.ascontiguousarray(p_all[:N]),
                                                 np.ascontiguousarray(v_all[:N]), L, 0)
            log(f"cross-check: {json.dumps(crosscheck)}")
        # velocity autocorrelation over 6 tau (a snapshot every 100 MD steps), for lambda from the VACF
        vstride, vsnap = 100, 601
        vs = torch.empty((vsnap, ntot, 2), dtype=torch.float64, device=dev)
        m.lj_md_get_state(sysm.handle, None, vs[0], None)
        e0.record()
        for p_ in range(1, vsnap):
            sysm.step(vstride)
            m.lj_md_get_state(sysm.handle, None, vs[p_], None)
        e1.record()
        torch.cuda.synchronize()
        gpu_ms["vacf_md"] = e0.elapsed_time(e1)
        vlags = sorted({0} | {int(round(x)) for x in np.geomspace(1, vsnap - 1, 64)})
        csum = torch.zeros((R, len(vlags)), dtype=torch.float64, device=dev)
        m.mdlg_vacf(offsets, vs, vlags, csum)
        del vs
        c_t = csum.cpu().numpy().sum(axis=0) / np.array([ntot * (vsnap - l) for l in vlags], dtype=np.float64)
        t_t = np.array(vlags, dtype=np.float64) * vstride * 1e-4
        tau_vacf, _ = m.mdlg_lambda_vacf(t_t, c_t, 1.0, 0.01)
        log(f"VACF: C(0) = {c_t[0]:.3f}, tau = {tau_vacf:.4f}")
        t_sweep = 0
        rows_state = {ri: {"events": 0, "counts": np.zeros((R, 50), np.int64), "moments": np.zeros((R, 5)),
                           "hist": np.zeros((R, 1, 2, n_bin + 2), np.int64)} for ri in rows}
    # device buffers of the rows still running: snapshot stacks and accumulators
    active = [ri for ri in rows if rows_state[ri]["events"] < E]
    dstate = {}
    for ri in active:
        st = rows_state[ri]
        dstate[ri] = {"pos": torch.empty((B + 1, ntot, 2), dtype=torch.float64, device=dev),
                      "img": torch.empty((B + 1, ntot, 2), dtype=torch.int32, device=dev), "j": 0,
                      "counts": torch.from_numpy(st["counts"].copy()).to(dev),
                      "moments": torch.from_numpy(st["moments"].copy()).to(dev),
                      "hist": torch.from_numpy(st["hist"].copy()).to(dev)}
        if args.resume:
            dstate[ri]["pos"][0].copy_(torch.from_numpy(ck[f"last_pos_{ri}"]))
            dstate[ri]["img"][0].copy_(torch.from_numpy(ck[f"last_img_{ri}"]))
        elif st["events"] == 0:
            m.lj_md_get_state(sysm.handle, dstate[ri]["pos"][0], None, dstate[ri]["img"][0])

    def flush(ri):
        """Coarse-grain and histogram the snapshot pairs gathered for row ri."""
        d = dstate[ri]
        j = d["j"]
        if j == 0:
            return
        dt_cg, _, lx, freq = TABLE1[ri]
        for p_ in range(j):
            for r in range(R):
                sl = slice(r * N, (r + 1) * N)
                m.mdlg_coarse_grain(lx, L, d["pos"][p_, sl], d["pos"][p_ + 1, sl], d["counts"][r], d["moments"][r],
                                    d["img"][p_, sl], d["img"][p_ + 1, sl])
        m.mdlg_displacement_hist(offsets, [L] * R, d["pos"][:j + 1], d["img"][:j + 1], [1], [(L / lx) / 8.0], n_bin,
                                 d["hist"])
        d["pos"][0].copy_(d["pos"][j])
        d["img"][0].copy_(d["img"][j])
        d["j"] = 0

    stop_at = args.stop_at if args.stop_at > 0 else None
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    md_steps = 0
    last_log = time.perf_counter()
    while active:
        nxt = {ri: (rows_state[ri]["events"] + 1) * TABLE1[ri][3] for ri in active}
        t_next = min(nxt.values())
        if stop_at is not None and t_next > stop_at:
            break
        e0.record()
        sysm.step(t_next - t_sweep)
        e1.record()
        e1.synchronize()
        gpu_ms["sweep_md"] += e0.elapsed_time(e1)
        md_steps += t_next - t_sweep
        t_sweep = t_next
        due = [ri for ri in active if nxt[ri] == t_next]
        src = None
        for ri in due:
            d = dstate[ri]
            d["j"] += 1
            if src is None:
                m.lj_md_get_state(sysm.handle, d["pos"][d["j"]], None, d["img"][d["j"]])
                src = (d["pos"][d["j"]], d["img"][d["j"]])
            else:
                d["pos"][d["j"]].copy_(src[0])
                d["img"][d["j"]].copy_(src[1])
            rows_state[ri]["events"] += 1
            if d["j"] == B or rows_state[ri]["events"] == E:
                flush(ri)
        active = [ri for ri in active if rows_state[ri]["events"] < E]
        if time.perf_counter() - last_log > 30.0:
            last_log = time.perf_counter()
            log(f"sweep step {t_sweep}: events {[rows_state[ri]['events'] for ri in rows]}")
    for ri in list(dstate):
        flush(ri)
        rows_state[ri]["counts"] = dstate[ri]["counts"].cpu().numpy()
        rows_state[ri]["moments"] = dstate[ri]["moments"].cpu().numpy()
        rows_state[ri]["hist"] = dstate[ri]["hist"].cpu().numpy()
    torch.cuda.synchronize()
    sysm.check()
    if active and args.checkpoint:
        # unfinished rows: state, accumulators and their last snapshot
        sysm.save(args.checkpoint + ".state")
        arrays = {}
        for ri in rows:
            st = rows_state[ri]
            arrays[f"ev_{ri}"] = np.int64(st["events"])
            arrays[f"counts_{ri}"] = st["counts"]
            arrays[f"moments_{ri}"] = st["moments"]
            arrays[f"hist_{ri}"] = st["hist"]
            if ri in active:
                arrays[f"last_pos_{ri}"] = dstate[ri]["pos"][0].cpu().numpy()
                arrays[f"last_img_{ri}"] = dstate[ri]["img"][0].cpu().numpy()
        meta = {"t_sweep": t_sweep, "rows": rows, "E": E, "vacf_t": t_t.tolist(), "vacf_c": c_t.tolist(),
                "tau_vacf": tau_vacf, "crosscheck": crosscheck, "equil_info": equil_info, "gpu_ms": gpu_ms}
        np.savez(args.checkpoint + ".npz", meta=json.dumps(meta), **arrays)
        log(f"checkpoint written at sweep step {t_sweep}")
    sysm.close()
    wall = time.perf_counter() - t_wall0
    out_rows, pdfs = _row_results(m, R, L, E, rows_state, t_t, c_t, n_bin)
    if args.pdf_out:
        with open(args.pdf_out, "w") as f:
            json.dump(pdfs, f)
    value = ntot * md_steps / (gpu_ms["sweep_md"] * 1e-3) if gpu_ms["sweep_md"] > 0 else None
    line = {
        "metric": "MD particle-steps/s, paper regime (Table 1 sweep, one trajectory for all rows)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": md_steps, "warmup": equil_info["md_steps"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.force_bits == 64 else "f64 state, f32 pair forces",
        "data": "synthetic (jittered-grid positions, Maxwellian velocities, seeds %d..%d)" % (args.seed,
                                                                                         args.seed + R - 1),
        "config": {"workload": f"{R} x 2D LJ gas N={N}, L={L}, phi={phi:.6f}, kT={kT}, rc={args.paper_rc:g}, dt=1e-4; "
                               f"{equil_info['md_steps']} equilibration steps; Table 1 rows {rows}, {E} coarse "
                               f"steps each from one trajectory", "replicas": R, "events_per_row": E,
                   "equil_steps": equil_info["md_steps"]},
        "status": "complete" if not active else f"checkpoint at sweep step {t_sweep}",
        "sweep_steps_done": t_sweep, "wall_s_this_call": wall, "gpu_ms": gpu_ms,
        "vacf": {"tau": tau_vacf, "C0": float(c_t[0]), "two_kT": 2 * kT,
                 "t": list(np.asarray(t_t)[::8]), "C_over_C0": list((np.asarray(c_t) / c_t[0])[::8])},
        "oracle_crosscheck_row0": crosscheck,
        "rows": out_rows,
    }
    print(json.dumps(line), flush=True)


def _decay_rate(t, a, floor):
    """Least-squares rate of exp(-g t) through the points with a > floor: (g, points used)."""
    t = np.asarray(t, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    keep = a > floor
    if keep.sum() < 3:
        return float("nan"), int(keep.sum())
    slope = np.polyfit(t[keep], np.log(a[keep]), 1)[0]
    return float(-slope), int(keep.sum())


def bench_neq(args):
    """Non-equilibrium MDLG of an ensemble: R replicas of a small LJ gas (N = 998,
    L = 100, phi = 0.0784, kT = 20) started as the same transverse wave
    v_x = 4 sin(2 pi y / L) over independent thermal noise, a snapshot per
    coarse step (Table 1 row 0: dt_cg = 0.3911, dx = 4, lx = 25), then the
    ensemble sums of n_i(x, t) and of the collision operator Xi_i(x, t) on the
    GPU.  Reports the throughput, the MDLG kernels against their rooflines,
    the decay rate of the flow's momentum mode seen by the MDLB f_i against the
    rate seen in the MD velocities, and the per-cell mass identity of Xi."""
    import torch

    import mdlg_inputs as mi
    import paper_2101_01160_amd as m

    log = lambda s_: print("# " + s_, file=sys.stderr, flush=True)
    R, E = args.neq_replicas, args.neq_events
    n, L, kT, amp, lx, s_cg = 998, 100.0, 20.0, 4.0, 25, 3911
    dt_cg = s_cg * 1e-4
    states = [mi.shear_wave_state(n, L, kT, amp, seed=args.seed + r) for r in range(R)]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sysm = m.LJSystem(torch.from_numpy(np.concatenate([s[0] for s in states])).to(dev),
                      torch.from_numpy(np.concatenate([s[1] for s in states])).to(dev),
                      params=[m.lj_params(n, L, force_bits=args.force_bits) for _ in range(R)])
    ntot = n * R
    info = sysm.info()
    K = info["rebuild_every"]
    sp = torch.empty((E + 1, ntot, 2), dtype=torch.float64, device=dev)
    si = torch.empty((E + 1, ntot, 2), dtype=torch.int32, device=dev)
    sv = torch.empty((E + 1, ntot, 2), dtype=torch.float64, device=dev)
    # kernel times of the step on this ensemble (graph replays with events), then back to the start
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    m.lj_md_get_state(sysm.handle, sp[0], sv[0], si[0])
    e0.record()
    for e in range(E):
        sysm.step(s_cg)
        m.lj_md_get_state(sysm.handle, sp[e + 1], sv[e + 1], si[e + 1])
    e1.record()
    torch.cuda.synchronize()
    sysm.check()
    ms_md = e0.elapsed_time(e1)
    kms, kcnt = sysm.step_timed(3)
    sysm.close()
    log(f"{R} x {n} particles, {E} coarse steps of {s_cg} MD steps in {ms_md:.1f} ms")
    f = torch.empty((E, 49, lx, lx), dtype=torch.int32, device=dev)
    ovf = torch.empty(E, dtype=torch.int64, device=dev)
    xi = torch.empty((E - 1, 49, lx, lx), dtype=torch.int32, device=dev)
    for _ in range(2):
        m.mdlg_neq_mdlg(L, lx, sp, si, f, ovf, xi)
    reps = 20
    t = []
    for with_xi in (False, True):
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(reps):
            m.mdlg_neq_mdlg(L, lx, sp, si, f, ovf, xi if with_xi else None)
        a1.record()
        torch.cuda.synchronize()
        t.append(a0.elapsed_time(a1) / reps)
    ms_scatter, ms_xi = t[0], max(t[1] - t[0], 1e-6)
    F = f.cpu().numpy().astype(np.int64)
    O = ovf.cpu().numpy()
    X = xi.cpu().numpy().astype(np.int64)
    # per-cell identity: sum_i Xi_i(x, t) = (moves out of x that stay in D2Q49) - (moves in); globally
    # sum_x,i Xi(t_p) = ovf(t_p) - ovf(t_{p+1})
    glob = X.sum(axis=(1, 2, 3))
    mass_ok = bool(np.array_equal(glob, O[:-1] - O[1:]))
    # momentum mode of the flow: MDLB lattice momentum per row against the MD velocities
    vt = m.mdlg_velocity_table().astype(np.int64)
    jx = np.einsum("eiyx,i->ey", F, vt[:, 0]) / float(R * lx)          # cells per coarse step per cell
    yc = (np.arange(lx) + 0.5) * (L / lx)
    a_lb = 2.0 / lx * (jx * np.sin(2 * math.pi * yc / L)[None, :]).sum(axis=1)
    P_ = sp.cpu().numpy()
    V_ = sv.cpu().numpy()
    a_md = 2.0 / ntot * (V_[:, :, 0] * np.sin(2 * math.pi * P_[:, :, 1] / L)).sum(axis=1)
    t_lb = (np.arange(1, E + 1) - 0.5) * dt_cg       # each event measures the window ending at t_p
    t_md = np.arange(E + 1) * dt_cg
    # fit while the mode is above a tenth of its start (the thermal noise of the ensemble mean is far below)
    g_md, used_md = _decay_rate(t_md, a_md, 0.1 * a_md[0])
    g_lb, used_lb = _decay_rate(t_lb, a_lb, 0.1 * a_lb[0])
    k2 = (2 * math.pi / L) ** 2
    # roofline of the MDLG kernels: scatter reads one snapshot (24 B) and adds one 4 B counter per
    # particle-event; the collision stencil reads two fields and writes one (12 B per element)
    scatter_bytes = 28.0 * ntot * E
    xi_bytes = 12.0 * (E - 1) * 49 * lx * lx
    t_step = float(kms[0])
    spl = int(info.get("steps_per_launch", 1)) or 1
    launch_ms = spl * t_step
    achieved = spl * STEP_BYTES * ntot / (launch_ms * 1e-3) / 1e9
    value = ntot * E * s_cg / (ms_md * 1e-3)
    line = {
        "metric": "MD particle-steps/s, non-equilibrium MDLG ensemble (shear wave)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": E * s_cg, "warmup": 0,
        "ms_per_step": ms_md / (E * s_cg), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 state; int32 occupation sums",
        "data": "synthetic (jittered grid, Maxwellian + transverse wave, seeds %d..%d)" % (args.seed, args.seed + R - 1),
        "config": {"workload": f"ensemble of {R} x 2D LJ gas N={n}, L={L}, kT={kT}, v_x += {amp} sin(2 pi y/L); "
                               f"lattice {lx}x{lx}, coarse step {s_cg} MD steps, {E} coarse steps recorded",
                   "replicas": R, "events": E},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "MD step kernel",
                     "kernel_ms": launch_ms, "steps_per_launch": spl},
        "mdlg_kernels": {
            "scatter_and_fill_ms": ms_scatter, "scatter_gbs": scatter_bytes / (ms_scatter * 1e-3) / 1e9,
            "xi_ms": ms_xi, "xi_gbs": xi_bytes / (ms_xi * 1e-3) / 1e9,
            "scatter_bytes": scatter_bytes, "xi_bytes": xi_bytes},
        "neq": {"mass_identity_exact": mass_ok, "overflow_per_event": float(O.mean()),
                "omega_l1_over_f_l1": float(np.abs(X).sum() / max(F[:-1].sum(), 1)),
                "momentum_mode_initial": {"md": float(a_md[0]), "mdlb": float(a_lb[0])},
                "decay_rate_md": g_md, "decay_rate_mdlb": g_lb, "points_md": used_md, "points_mdlb": used_lb,
                "nu_md": g_md / k2, "nu_mdlb": g_lb / k2},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
