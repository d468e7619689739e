#!/usr/bin/env python3
"""Throughput of the wildfire cellular automaton on one MI355X.

One benchmark step = one full forward run of the 4096 x 4096 workload
(1000 time steps from a 20 x 20 ignition patch, lakes, per-cell wind, 30 m
cells): reset to the ignition state, then every CA step (candidate
detection, per-edge Eq. 1-5, Eq. 9, Philox draws, transition) on the GPU.
Inputs are resident in HBM before the timed region.

Side legs, reported in the same JSON line:
  plain_step   the same grid advanced one step per launch with no tile
               skipping (the straightforward stencil);
  calibration  64 scenarios of 1024 x 1024, 200 steps, checkpoints every 20:
               forward + Eq. 10 BCE loss + adjoint + AdamW, in grad-steps/s;
  batched      256 scenarios with log-uniform sides 256-2048, 300 steps, one
               launch sequence over all of them;
  paper_sweep  the paper's timing workload shape (square plain map, fixed
               wind, 300 steps) at sides 50 .. 14000, beside its stated times;
  cpu_baseline the FP64 oracle on the host, on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--legs main,plain,calib,batched,cpu]
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cell-updates/s (G cells·steps/s) + % HBM roofline; calibration grad-steps/s"
HBM_PEAK_GBS = 8000.0
# Bytes per cell-step of the dense formulation (every cell reads its 2-bit
# state, F = (1+p_veg)(1+p_den), elevation, wind speed and direction, and
# writes 2 bits): 0.5 + 4 + 4 + 8.
DENSE_BYTES_PER_CELL_STEP = 16.5
# Algorithmic bytes of the work a step kernel actually does: every trial (a
# cell-step whose next state needs a Bernoulli draw) needs that cell-step's
# dense bytes; every tile a launch processes reads and writes its 2-bit state
# once (0.5 B per cell).
TRIAL_BYTES = DENSE_BYTES_PER_CELL_STEP
TILE_STATE_BYTES_PER_CELL = 0.5
DEFAULT_EXEC = dict(tile_rows=32, tile_words=2, depth=32, skip=1)
PLAIN_EXEC = dict(tile_rows=16, tile_words=8, depth=1, skip=False)


def km_bucket(depth):
    """Halo depth of the step kernel that runs `depth` steps per launch."""
    return next(k for k in (1, 4, 8, 16, 32) if k >= depth)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the library sources with comments and blank space removed, so
    that committed counter runs stay matched to the code they measured."""
    import re
    tok = re.compile(r'"(?:\\.|[^"\\])*"|//[^\n]*|/\*.*?\*/', re.S)
    h = hashlib.sha256()
    for f in ("kernels.hip", "api.hip", "internal.h"):
        src = open(os.path.join(ROOT, "paper_2502_18738_amd", "csrc", f)).read()
        code = tok.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", src)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(name):
    """Per-launch HBM bytes from committed rocprofv3 counter runs, if they were
    taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d


def summarize_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes,
                       kernel_regex, out_json):
    """Per-launch HBM bytes of the kernels matching `kernel_regex` from two
    rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each
    scaled by what the same counter reads for a plain device copy of
    `copy_bytes` bytes."""
    import csv
    import re

    def per_dispatch(path, counter, regex):
        vals = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter and re.search(regex, r["Kernel_Name"]):
                vals[r["Dispatch_Id"]] = vals.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
        return list(vals.values())

    def largest(path, counter):
        return max(per_dispatch(path, counter, "copyBuffer|elementwise|copy"))

    f_fetch = copy_bytes / (largest(copy_fetch_csv, "FETCH_SIZE") * 1024.0)
    f_write = copy_bytes / (largest(copy_write_csv, "WRITE_SIZE") * 1024.0)
    fk = per_dispatch(fetch_csv, "FETCH_SIZE", kernel_regex)
    wk = per_dispatch(write_csv, "WRITE_SIZE", kernel_regex)
    fetch_b = sum(fk) / len(fk) * 1024.0 * f_fetch
    write_b = sum(wk) / len(wk) * 1024.0 * f_write
    out = {"kernel_regex": kernel_regex, "kernel_source_sha": kernel_source_hash(),
           "exec": dict(DEFAULT_EXEC),
           "dispatches": [len(fk), len(wk)],
           "fetch_KiB_per_dispatch": sum(fk) / len(fk), "write_KiB_per_dispatch": sum(wk) / len(wk),
           "copy_scale": {"fetch": f_fetch, "write": f_write, "copy_bytes": copy_bytes},
           "bytes_per_launch": fetch_b + write_b, "fetch_bytes": fetch_b, "write_bytes": write_b}
    json.dump(out, open(out_json, "w"), indent=1)
    print(json.dumps(out))


def timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, ev0.elapsed_time(ev1) / 1e3


def step_kernel_name(ex):
    """The forward step instantiation of an execution shape (the last template
    argument, the work-item mode: 0 every tile (skip modes 0 and 2), 1 the
    worklist (skip mode 1), 2 every tile tested against the worklist (skip
    mode 3))."""
    return "k_step<{},{},{},false,{},{}>".format(
        ex["tile_rows"], ex["tile_words"], km_bucket(ex["depth"]),
        ex.get("threads") or (512 if ex["tile_rows"] >= 32 else 256),
        {1: 1, 3: 2}.get(int(ex["skip"]), 0))


def work_counts(Sim, scs, ex, T, torch):
    """Tiles processed, trials and launches of one run (a counting run of the
    same shape; the counters are off in the timed runs)."""
    st = Sim(scs, exec=ex, stats=True)
    st.run(T)
    torch.cuda.synchronize()
    cnt = st.stats()
    del st
    return cnt


def algorithmic_bytes(cnt, ex):
    """Per launch: TRIAL_BYTES per trial plus the 2-bit state in and out of
    every processed tile."""
    tile_cells = ex["tile_rows"] * ex["tile_words"] * 32
    per_run = (cnt["trials"] * TRIAL_BYTES
               + cnt["tiles"] * tile_cells * TILE_STATE_BYTES_PER_CELL)
    return per_run / cnt["launches"]


def timed_steps(sim, T, reps, torch):
    """Seconds of the step launches of one run from a reset, the table built
    beforehand (sim.prepare), on the handle's stream; median over reps."""
    out = []
    for rep in range(reps + 1):   # the first run captures the launch graph: not timed
        sim.reset()
        sim.prepare(T)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(sim.stream):
            e0.record()
            sim.run(T)
            e1.record()
        e1.synchronize()
        if rep:
            out.append(e0.elapsed_time(e1) / 1e3)
    return float(np.median(out))


def leg_main(args, torch, Sim, synth):
    s = synth.config2()
    T = s.T
    sim = Sim([s], exec=DEFAULT_EXEC)
    if args.autotune:
        # tune on a mid-run state (the fire front at 400 steps), then restart
        sim.run(400)
        DEFAULT_EXEC.update(sim.autotune(32))
        log("autotuned shape:", DEFAULT_EXEC)

    # whole job: reset with the run's own seed, 1000 steps; every run is a
    # different realisation of the fire, and the propagation table (which the
    # seeds do not enter) is built by the first run and kept by the others
    seed = [s.seed]

    def run():
        seed[0] += 1
        sim.reset([seed[0]])
        sim.run(T)

    wall, gpu = timed(run, args.steps, args.warmup, torch)
    cells = s.H * s.W
    rate = cells * T * args.steps / wall / 1e9
    # the same with the table rebuilt by every run (parameters set again)
    par = [(s.p_h, s.a, s.c1, s.c2, s.p_continue)]

    def run_rebuild():
        sim.set_params(par)
        run()

    wall_rb, _ = timed(run_rebuild, args.steps, 1, torch)
    # dominant kernel: the step kernel; its launches alone (table built
    # before the events), all of the run's launches in one captured graph
    cnt = work_counts(Sim, [s], DEFAULT_EXEC, T, torch)
    steps_s = timed_steps(sim, T, max(3, args.steps), torch)
    launch_s = steps_s / cnt["launches"]
    alg = algorithmic_bytes(cnt, DEFAULT_EXEC)
    achieved = alg / launch_s / 1e9
    roof = {
        "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
        "kernel": step_kernel_name(DEFAULT_EXEC),
        "launch_us": round(launch_s * 1e6, 2),
        "algorithmic_bytes_per_launch": round(alg),
        "basis": f"per launch: trials x {TRIAL_BYTES} B (the dense bytes of each cell-step "
                 f"that needs a draw) + processed tiles x cells x "
                 f"{TILE_STATE_BYTES_PER_CELL} B (2-bit state in and out); launch time = "
                 "HIP events around the run's step launches (table built before) / launches",
        "limiter": "latency of each step's dependency chain in the busiest tiles "
                   "(a few hundred work-groups per launch), not bandwidth",
        "dense_equivalent_speedup": round(DENSE_BYTES_PER_CELL_STEP * cells * T / steps_s
                                          / 1e9 / HBM_PEAK_GBS, 2),
    }
    tr = load_traffic("k_step_config2")
    if tr and tr.get("exec") != DEFAULT_EXEC:
        tr = None
    if tr:
        roof["traffic"] = round(tr["bytes_per_launch"])
        roof["traffic_GBps"] = round(tr["bytes_per_launch"] / launch_s / 1e9, 1)
        roof["traffic_frac"] = round(tr["bytes_per_launch"] / launch_s / 1e9 / HBM_PEAK_GBS, 4)
    out = {
        "value": round(rate, 3),
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "gpu_ms_per_step": round(gpu / args.steps * 1e3, 3),
        "step_is": "one benchmark step = one whole 1000-step run of the 4096x4096 grid "
                   "(reset with a new seed, 1000 CA steps; the propagation table is built "
                   "by the first run and kept, since seeds do not enter it): ms_per_step "
                   "is ms per run",
        "ms_per_run_table_rebuilt": round(wall_rb / args.steps * 1e3, 3),
        "steps_only_ms_per_run": round(steps_s * 1e3, 3),
        "roofline": roof,
        "work": {"tiles_processed_per_run": cnt["tiles"], "trials_per_run": cnt["trials"],
                 "near_ties_per_run": cnt["ties"], "launches_per_run": cnt["launches"],
                 "tiles_per_launch_if_dense": sim_tiles(s, DEFAULT_EXEC)},
        "config": {"workload": "4096x4096 grid, 1000 steps, 10% lakes, per-cell wind, "
                               "elevation 0-1500 m, 20x20 ignition patch, 30 m cells",
                   "H": s.H, "W": s.W, "T": T, "scenarios": 1, "exec": DEFAULT_EXEC},
    }
    return out, s


def sim_tiles(s, ex):
    pitch = -(-s.W // 32)
    return (-(-s.H // ex["tile_rows"])) * (-(-pitch // ex["tile_words"]))


def leg_plain(args, torch, Sim, s):
    """One step per launch, every tile processed (no skipping, no blocking)."""
    T = 200
    sim = Sim([s], exec=PLAIN_EXEC)

    def run():
        sim.reset()
        sim.run(T)

    wall, gpu = timed(run, 1, 1, torch)
    cells = s.H * s.W
    steps_s = timed_steps(sim, T, 3, torch)
    cnt = work_counts(Sim, [s], PLAIN_EXEC, T, torch)
    launch_s = steps_s / cnt["launches"]
    alg = algorithmic_bytes(cnt, PLAIN_EXEC)
    return {
        "exec": PLAIN_EXEC, "steps": T, "kernel": step_kernel_name(PLAIN_EXEC),
        "G_cell_steps_per_s": round(cells * T / wall / 1e9, 3),
        "launch_us": round(launch_s * 1e6, 2),
        "algorithmic_bytes_per_launch": round(alg),
        "achieved_GBps": round(alg / launch_s / 1e9, 1),
        "frac_of_hbm_peak": round(alg / launch_s / 1e9 / HBM_PEAK_GBS, 4),
        "dense_equivalent_speedup": round(DENSE_BYTES_PER_CELL_STEP * cells / launch_s / 1e9
                                          / HBM_PEAK_GBS, 2),
        "note": "every tile every step: the state planes (about 10 MB) stay in the caches; "
                "dense_equivalent_speedup = the dense formulation's 16.5 B per cell-step "
                "at this rate over the 8 TB/s peak",
    }


def leg_calib(args, torch, Sim, synth):
    n, T, ck = 64, 200, 20
    log("calibration: generating", n, "scenarios")
    cases = [synth.config4_scenario(b) for b in range(n)]
    true_s = [c[0] for c in cases]
    gen = Sim(true_s)
    gen.run(T)
    target = torch.cat([(gen.get_state(b).sum(0) != 0).to(torch.uint8).view(-1)
                        for b in range(n)])
    del gen
    start = [c[1] for c in cases]
    # the autotuner needs a handle without calibration state: tune a forward
    # handle over the same scenarios at mid-run, then use its choice
    tune = Sim(true_s)
    tune.run(100)
    cex = tune.autotune(ck)   # one checkpoint segment: the launch pattern of a calibration run
    del tune
    # The forward probe does not see the checkpoint adjoint's recompute, which
    # launches the tiles of every segment together and pays a dispatch cost
    # per launch: settle the depth on whole gradient steps, for the probe's
    # tile at each halo depth (a segment's steps spread evenly over the fewest
    # launches the halo allows: 7, 10 or 20 steps for halos of 8, 16, 32)
    from paper_2502_18738_amd import SimError
    p0 = [list(start[b]) + [true_s[b].p_continue] for b in range(n)]
    depths = {cex["depth"]}
    for km in (8, 16, 32):
        depths.add(min(-(-ck // -(-ck // km)), cex["tile_rows"]))
    best = None
    for d in sorted(depths):
        ex = dict(cex, depth=d)
        try:
            probe = Sim(true_s, calib=True, T_max=T, ckpt_every=ck, exec=ex)
        except SimError:
            continue            # no halo of that depth compiled for this tile

        def probe_step(i):
            probe.set_params(p0)
            probe.reset([500 + i] * n)
            probe.run(T)
            probe.loss_grad(target, 0)

        probe_step(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(3):
            probe_step(i + 1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        log("calibration depth", d, round(dt / 3 * 1e3, 3), "ms per gradient step")
        del probe
        if best is None or dt < best[0]:
            best = (dt, ex)
    if best:
        cex = best[1]
    sim = Sim(true_s, calib=True, T_max=T, ckpt_every=ck, exec=cex)
    theta = torch.tensor(start, dtype=torch.float32, device="cuda", requires_grad=True)
    opt = torch.optim.AdamW([theta], lr=5e-3)
    lo = torch.tensor([0.2, 0.0, 0.0, 0.0], device="cuda")
    hi = torch.tensor([1.0, 1.0, 1.0, 1.0], device="cuda")
    step = [0]

    def grad_step():
        # theta goes to the library from device memory (no host round trip)
        sim.set_params_device(theta.detach())
        sim.reset([1000 + step[0]] * n)
        sim.run(T)
        loss, g = sim.loss_grad(target, 0)
        theta.grad = g.to(torch.float32)
        opt.step()
        with torch.no_grad():
            theta.copy_(torch.maximum(torch.minimum(theta, hi), lo))
        step[0] += 1
        return loss

    K = max(2, args.steps)
    wall, gpu = timed(grad_step, K, 1, torch)
    sim.set_adjoint("timemap")
    wall_tm, _ = timed(grad_step, K, 1, torch)
    if sim.params_rejected():
        raise RuntimeError("the library rejected parameter rows during the calibration leg")
    cells = 1024 * 1024 * n
    return {
        "metric": "calibration grad-steps/s", "value": round(K / wall, 3),
        "adjoint": "checkpoint every 20 steps, segments recomputed",
        "ms_per_grad_step": round(wall / K * 1e3, 2),
        "G_cell_steps_per_s": round(2 * cells * T * K / wall / 1e9, 3),
        "timemap_adjoint": {"value": round(K / wall_tm, 3),
                            "ms_per_grad_step": round(wall_tm / K * 1e3, 2)},
        "config": {"workload": "64 scenarios 1024x1024, 200 steps, checkpoints every 20, "
                               "BCE loss, AdamW lr 5e-3 with clamps",
                   "exec": cex,
                   "exec_from": "tile from a forward autotune over one checkpoint segment, "
                                "depth from whole gradient steps at each halo depth"},
    }


def leg_batched(args, torch, Sim, synth):
    n, T = 256, 300
    log("batched: generating", n, "scenarios")
    scs = [synth.config3_scenario(b, T=T) for b in range(n)]
    sim = Sim(scs)
    # tune on the workload itself: every candidate shape runs the T steps from
    # the initial state (the autotuner restores the state afterwards)
    ex = sim.autotune(T)

    # every run with new seeds; the propagation tables are built by the first
    # run and kept (seeds do not enter them)
    rep = [0]

    def run():
        rep[0] += 1
        sim.reset([s.seed + 1000 * rep[0] for s in scs])
        sim.run(T)

    K = max(3, args.steps)
    wall, gpu = timed(run, K, 1, torch)
    par = [(s.p_h, s.a, s.c1, s.c2, s.p_continue) for s in scs]

    def run_rebuild():
        sim.set_params(par)
        run()

    wall_rb, _ = timed(run_rebuild, K, 1, torch)
    cells = sum(s.H * s.W for s in scs)
    return {
        "value": round(cells * T * K / wall / 1e9, 3), "unit": "G cell-steps/s",
        "ms_per_run": round(wall / K * 1e3, 2), "cells": cells, "runs": K,
        "ms_per_run_table_rebuilt": round(wall_rb / K * 1e3, 2),
        "config": {"workload": "256 scenarios, sides log-uniform 256-2048, 300 steps, "
                               "+-20% parameter jitter", "exec": ex},
    }


# The paper's stated timings for 300 steps on a square plain map (Sec. 3,
# forward prediction; the figure itself is not available): side -> seconds,
# device.  "<" marks an upper bound stated in the text.
PAPER_300 = {
    800: ("0.52 s (flat for every side <= 800)", "RTX 4090"),
    1200: ("< 1 s", "RTX 4090"),
    1500: ("< 1 s", "A800"),
    8000: ("largest side that fits", "RTX 4090"),
    14000: ("< 60 s", "'a more advanced GPU'"),
}


def leg_paper_sweep(args, torch, Sim, synth):
    """Sides 50 .. 14000 of the paper's 300-step plain-map workload."""
    out = []
    for side in (50, 200, 800, 1200, 1500, 4000, 8000, 14000):
        s = synth.paper_plain(side)
        sim = Sim([s], exec=DEFAULT_EXEC)
        par = [(s.p_h, s.a, s.c1, s.c2, s.p_continue)]

        def run():
            # one prediction from scratch: parameters set, so the run builds
            # its propagation table
            sim.set_params(par)
            sim.reset()
            sim.run(300)

        wall, gpu = timed(run, 2, 1, torch)
        row = {"side": side, "ms_per_300_steps": round(wall / 2 * 1e3, 3),
               "G_cell_steps_per_s": round(side * side * 300 * 2 / wall / 1e9, 3)}
        if side in PAPER_300:
            row["paper"] = {"time": PAPER_300[side][0], "device": PAPER_300[side][1]}
        out.append(row)
        log("paper sweep", row)
        del sim
        torch.cuda.empty_cache()
    return {"workload": "square plain map (flat, neutral fuel), uniform wind 5 m/s toward "
                        "45 deg, centre ignition, 300 steps", "rows": out}


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0))
    omp = int(os.environ.get("OMP_NUM_THREADS", avail) or avail)
    return model, avail, max(1, min(avail, omp))


def leg_cpu(args, s2, synth):
    """The FP64 oracle (plain C loop; its OpenMP build splits the rows of each
    step over the host's cores) on bounded samples of the workloads."""
    import oracle
    model, avail, threads = host_cpu()
    s0, s1 = synth.config0(), synth.config1()
    rows = []

    def one(s, steps, label, n):
        oracle.set_threads(n)
        t0 = time.perf_counter()
        oracle.run(s, steps)
        dt = time.perf_counter() - t0
        r = {"workload": label, "steps": steps, "threads": oracle.threads(),
             "seconds": round(dt, 3), "G_cell_steps_per_s": round(s.H * s.W * steps / dt / 1e9, 5)}
        rows.append(r)
        log("cpu baseline", r)
        return r

    one(s0, s0.T, "128x128, 100 steps (full run)", 1)
    one(s1, s1.T, "1024x1024, 500 steps (full run)", 1)
    one(s2, 40, "4096x4096, steps 1-40 (sample)", 1)
    one(s0, s0.T, "128x128, 100 steps (full run)", threads)
    one(s1, s1.T, "1024x1024, 500 steps (full run)", threads)
    main = one(s2, s2.T, "4096x4096, 1000 steps (full run)", threads)
    oracle.set_threads(1)
    # the larger workloads at the all-core rate of the full 4096 x 4096 run
    # (the oracle's cost per cell-step does not depend on the fire)
    rate = main["G_cell_steps_per_s"] * 1e9
    c3 = sum(h * w for h, w in synth.config3_sizes())
    est = [{"workload": "256 scenarios, sides 256-2048, 300 steps (forward)",
            "cell_steps": c3 * 300, "seconds": round(c3 * 300 / rate, 1)},
           {"workload": "64 scenarios 1024x1024, 200 steps (forward of one gradient step)",
            "cell_steps": 64 * 1024 * 1024 * 200,
            "seconds": round(64 * 1024 * 1024 * 200 / rate, 1)}]
    return {"value": main["G_cell_steps_per_s"], "unit": "G cell-steps/s",
            "cores": main["threads"], "kind": "oracle",
            "sample": "the whole 4096x4096 main workload (1000 steps from the ignition patch), "
                      f"FP64 C loop with rows split over {main['threads']} threads",
            "host": {"cpu_model": model, "cpus_available": avail},
            "runs": rows, "extrapolated": est}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--legs", default="main,plain,calib,batched,paper,cpu")
    ap.add_argument("--exec", default=None, metavar="TR,TC,DEPTH,SKIP[,THREADS]",
                    help="execution shape of the main leg (tile rows, tile words, steps "
                         "per launch, skip 0/1/2/3, work-group size or 0 for the default)")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the main leg's shape on a mid-run state (the batched "
                         "leg always autotunes)")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (reference "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--summarize-counters", nargs=7, default=None,
                    metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV",
                             "COPY_BYTES", "KERNEL_REGEX", "OUT_JSON"),
                    help="write per-launch HBM traffic from rocprofv3 counter CSVs")
    args = ap.parse_args()
    if args.summarize_counters:
        a = args.summarize_counters
        summarize_counters(a[0], a[1], a[2], a[3], int(a[4]), a[5], a[6])
        return
    if args.copy_ref:
        import torch
        a = torch.empty(args.copy_ref // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_ref}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is not built", file=sys.stderr)
        sys.exit(2)
    legs = set(args.legs.split(","))
    if args.exec:
        v = [int(x) for x in args.exec.split(",")]
        DEFAULT_EXEC.update(tile_rows=v[0], tile_words=v[1], depth=v[2], skip=v[3])
        if len(v) > 4:
            DEFAULT_EXEC["threads"] = v[4]

    import torch
    import synth
    from paper_2502_18738_amd.sim import Sim
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    log("main: config 2")
    main_out, s2 = leg_main(args, torch, Sim, synth)
    res = {
        "metric": METRIC, "value": main_out["value"], "unit": "G cell-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_out["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": main_out["config"], "roofline": main_out["roofline"],
        "gpu_ms_per_step": main_out["gpu_ms_per_step"], "work": main_out["work"],
        "step_is": main_out["step_is"], "steps_only_ms_per_run": main_out["steps_only_ms_per_run"],
        "ms_per_run_table_rebuilt": main_out["ms_per_run_table_rebuilt"],
    }
    if "plain" in legs:
        log("plain step")
        res["plain_step"] = leg_plain(args, torch, Sim, s2)
    if "calib" in legs:
        res["calibration"] = leg_calib(args, torch, Sim, synth)
    if "batched" in legs:
        res["batched"] = leg_batched(args, torch, Sim, synth)
    if "paper" in legs:
        res["paper_sweep"] = leg_paper_sweep(args, torch, Sim, synth)
    if "cpu" in legs:
        log("cpu baseline")
        res["cpu_baseline"] = leg_cpu(args, s2, synth)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
