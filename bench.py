"""Benchmark: particle-pushes/s of the full PIC MC step on one MI355X.

Workload: the magnetised sheath slab at 1e5 cells x 200 particles per cell per species
(4.0e7 particles, electrons + argon-mass ions), oblique B (omega_ce/omega_pe = 2 at 80
degrees to x), three null-collision channels with ionisation births, absorbing walls, cell
sort every 20 steps; FP32 cell+offset particles with the FP64 field solve, one fused
particle pass per step replayed from a HIP graph.  A step is the whole hot path: field
solve, gather + Boris push, walls, null-collision MC, births, deposit, and the sort on
every 20th step.  Inputs are synthetic (seeded Philox particle load) and resident in HBM
before the timed region starts.

Prints ONE JSON line.  `--gpus N` with N > 1 exits: the hot path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
B_ALG_PARTICLE = 44.0          # FP32 form: read cell+off+v+id (24 B), write cell+off+v (20 B)
B_ALG_CELL = 8.0               # gather table (E_j, dE_j) per cell, float2
B_ALG_NODE = 16.0              # two species' int64 charge sums per node


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("pic_pass32.hip", "pic_particle.h", "pic_device.h"):
        with open(os.path.join(ROOT, "paper_2606_28534_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload_name, bytes_alg_per_launch):
    """HBM bytes per launch of the fused pass from the committed PMC summary, scaled from
    the counted run's launches to this run's by their algorithmic bytes (the counted run is
    shorter, so it pushes fewer particles per launch); None when the summary is missing or
    was taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", f"pmc_fused_pass_{workload_name}.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    measured, counted_alg = rec.get("bytes_per_launch"), rec.get("bytes_alg_per_launch")
    if measured is None or not counted_alg:
        return None
    return round(measured * bytes_alg_per_launch / counted_alg)


def tuned_shape(pic, work, trial_steps):
    """Launch shape chosen by the library's autotuner on a throw-away run of the workload."""
    if trial_steps <= 0:
        return {}
    t = pic.Sim(work, fused=True)
    shape = t.autotune(trial_steps)
    t.close()
    del t
    return shape


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seed, steps, omp_steps):
    """The FP64 oracle as it stands on the first steps of the same workload (particle load
    excluded from the timing): single-threaded, and the same source built with OpenMP on
    its particle loops, on all the host threads OpenMP is given (OMP_NUM_THREADS)."""
    import oracle
    import synth

    oracle.build(force=False)
    e = synth.c2_sheath(seed=seed)["ensembles"][0]
    legs = {}
    for omp, n in ((False, steps), (True, omp_steps)):
        o = oracle.Oracle(e, omp=omp)
        d0 = o.diag()["pushes"]
        t0 = time.perf_counter()
        o.step(n)
        t1 = time.perf_counter()
        pushes = o.diag()["pushes"] - d0
        legs[omp] = {"value": pushes / (t1 - t0), "threads": oracle.threads(omp), "steps": n,
                     "pushes": pushes, "seconds": round(t1 - t0, 2)}
        del o
    a, one = legs[True], legs[False]
    return {"value": a["value"], "unit": "particle-pushes/s", "cores": a["threads"], "kind": "oracle",
            "sample": f"first {a['steps']} steps of the same 1e5-cell x 200-ppc workload (seed {seed}), "
                      f"{a['pushes']} pushes in {a['seconds']} s, FP64, OpenMP on the particle loops "
                      f"({a['threads']} threads); single-threaded: first {one['steps']} steps, "
                      f"{one['pushes']} pushes in {one['seconds']} s",
            "single_thread": {"value": one["value"], "cores": 1},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def batched_run(pic, shape, steps):
    """The 64-ensemble batched workload (uneven sizes, one launch per stage for all
    ensembles), FP32 fused pass in a HIP graph, at the particle-pass launch shape of the
    main workload."""
    import torch

    import synth

    work = synth.c3_batched()
    sim = pic.Sim(work, fused=True, **shape)
    n_ens = len(work["ensembles"])
    sim.step(20)
    sim.prepare(steps)
    torch.cuda.synchronize()
    p0 = sum(sim.diag(k)["pushes"] for k in range(n_ens))
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p1 = sum(sim.diag(k)["pushes"] for k in range(n_ens))
    particles = sum(2 * e["species"][0]["ppc"] * e["ncells"] for e in work["ensembles"])
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"value": (p1 - p0) / (t1 - t0), "unit": "particle-pushes/s", "steps": steps,
            "ms_per_step": (t1 - t0) / steps * 1e3, "ensembles": n_ens, "particles": particles,
            "cells": sum(e["ncells"] for e in work["ensembles"])}


def walls_variant_run(pic, shape, steps, seed, smooth):
    """The main workload with floating walls (the absorbed charge stays on the walls) and
    `smooth` passes of the density filter before each solve: the same fused graph, with
    the solve's wall boundary condition and smoothed density the only differences."""
    import torch

    import synth

    work = synth.c2_sheath(seed=seed)
    e = work["ensembles"][0]
    e["floating"] = True
    e["smooth"] = smooth
    sim = pic.Sim(work, fused=True, **shape)
    sim.step(20)
    sim.prepare(steps)
    torch.cuda.synchronize()
    p0 = sim.diag()["pushes"]
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p1 = sim.diag()["pushes"]
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"value": (p1 - p0) / (t1 - t0), "unit": "particle-pushes/s", "steps": steps,
            "ms_per_step": (t1 - t0) / steps * 1e3, "boundary": "floating", "smooth": smooth}


def sheath_case_run(pic, shape, case, seed, warmup, steps, refill=0):
    """The paper's two sheath cases at 1e5 cells: "recycling" is the uniform load with its
    three species (4.0e7 charged particles, ions recycled into neutrals at floating walls);
    "source" is the initially empty slab filled by 2e4 electron-ion pairs per step in its
    left half (measured after `warmup` steps of filling).  Same fused graph and launch
    shape as the main workload.  With `refill`, the same run goes on filling until step
    `refill` and is timed again there (entry "filled")."""
    import torch

    import synth

    work = synth.c6_sheath_recycling(seed=seed) if case == "recycling" else synth.c7_sheath_source(seed=seed)
    sim = pic.Sim(work, fused=True, **shape)

    def timed(after):
        sim.prepare(steps)
        torch.cuda.synchronize()
        d0 = sim.diag()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        d1 = sim.diag()
        return {"value": (d1["pushes"] - d0["pushes"]) / (t1 - t0), "unit": "particle-pushes/s",
                "steps": steps, "after_steps": after, "ms_per_step": (t1 - t0) / steps * 1e3,
                "charged_particles": sum(d1["count"]), "neutrals": d1["neutral_count"],
                "recycled": d1["recycled"], "sourced": d1["sourced"]}

    sim.step(warmup)
    out = timed(warmup)
    if refill > warmup + steps:
        sim.step(refill - warmup - steps)
        out["filled"] = timed(refill)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def large_run(pic, shape, seed, warmup, steps):
    """The large single-GPU share: 1e6 cells x 500 ppc x 2 species (1.0e9 particles, about
    60 GB of HBM), oblique B, three channels with births, sort every 10 steps."""
    import torch

    import synth

    work = synth.c5_large(seed=seed)
    sim = pic.Sim(work, fused=True, **shape)
    sim.step(warmup)
    sim.prepare(steps)
    torch.cuda.synchronize()
    p0 = sim.diag()["pushes"]
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    p1 = sim.diag()["pushes"]
    ws = sim.ws_bytes
    sim.close()
    del sim
    torch.cuda.empty_cache()
    pushes = p1 - p0
    return {"value": pushes / (t1 - t0), "unit": "particle-pushes/s", "steps": steps,
            "after_steps": warmup, "ms_per_step": (t1 - t0) / steps * 1e3,
            "particles": 2 * work["ensembles"][0]["species"][0]["ppc"] * work["ensembles"][0]["ncells"],
            "workspace_gb": round(ws / 1e9, 1),
            "frac_of_hbm_peak_46.8B": round((B_ALG_PARTICLE + 48.0 / 10) * pushes / (t1 - t0) / 1e9 / HBM_PEAK_GBS, 4)}


def correctness_configs_run(pic):
    """Time only, for the two correctness configurations: the plain FP64 form on 256 cells x
    100 ppc x 2 species with collisions (the full 1000-step run, eager), and one adjoint
    window of the 2048-cell, 200-ppc Langmuir workload (200 steps, a checkpoint every 20,
    forward, reverse sweep and gradients)."""
    import torch

    import synth

    out = {}
    w = synth.c1_plain_small(seed=1)
    sim = pic.Sim(w, fused=False)
    sim.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(w["steps"] - 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.close()
    out["plain_small_256cells"] = {"steps": w["steps"] - 1, "ms_per_step": (t1 - t0) / (w["steps"] - 1) * 1e3,
                                   "form": "FP64, one kernel per stage, eager"}
    w = synth.c4_langmuir()
    sim = pic.Sim(w, fused=True)
    sim.adjoint_window(w["steps"], 20)  # warm: scratch, graphs of the recompute
    sim.close()
    sim = pic.Sim(w, fused=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.adjoint_window(w["steps"], 20)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    out["adjoint_window_langmuir"] = {"steps": w["steps"], "checkpoint_every": 20, "ms_per_window": (t1 - t0) * 1e3}
    return out


def stream_copy_gbs(torch, pic, gib=4.0, reps=10):
    """Device-to-device copy bandwidth on the same GPU (read + write bytes per second), for
    context next to the HBM peak: a plain torch copy, and the library's copy with the
    particle pass's access pattern (16-byte non-temporal loads and stores, four words a
    thread)."""
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out = {"bytes": 2 * n * 4}
    for name, fn in (("torch_copy", lambda: b.copy_(a)),
                     ("pass_pattern_copy", lambda: pic.stream_copy(a, b, nontemporal=True))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"gbs": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 4)}
    out["gbs"] = out["torch_copy"]["gbs"]
    del a, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--cpu-omp-steps", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--ncells", type=int, default=100_000)
    ap.add_argument("--ppc", type=int, default=200)
    ap.add_argument("--separate", action="store_true",
                    help="profile the FP32 form with one kernel per stage instead of the fused pass")
    ap.add_argument("--tune-steps", type=int, default=10,
                    help="trial steps per candidate launch shape of the autotuner (0 = defaults)")
    ap.add_argument("--shape", type=str, default="",
                    help="fixed launch shape ppt,window,sort_ppt,nontemporal instead of the autotuner")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=40)
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--no-walls-variant", action="store_true")
    ap.add_argument("--no-sheath-cases", action="store_true")
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the timings of the two correctness configurations")
    ap.add_argument("--case", choices=["sheath", "recycling", "source", "large", "batched"], default="sheath",
                    help="main workload: the sheath slab (default), one of the paper's two "
                         "sheath cases, the 1e9-particle share or the 64 batched ensembles "
                         "(for profiling them)")
    ap.add_argument("--fp64", action="store_true",
                    help="main workload in the plain FP64 form (x, v in FP64; with --separate, "
                         "one kernel per stage: the plain form, for profiling it)")
    ap.add_argument("--floating", action="store_true",
                    help="main workload with floating walls (for profiling the variant)")
    ap.add_argument("--smooth", type=int, default=0,
                    help="passes of the density filter in the main workload (for profiling)")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run one copy of this many GiB with the pass's access pattern "
                         "(counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the hot path runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    import paper_2606_28534_amd as pic
    import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.case == "recycling":
        work = synth.c6_sheath_recycling(seed=args.seed, ncells=args.ncells, ppc=args.ppc)
    elif args.case == "source":
        work = synth.c7_sheath_source(seed=args.seed, ncells=args.ncells)
    elif args.case == "large":
        work = synth.c5_large(seed=args.seed)
    elif args.case == "batched":
        work = synth.c3_batched()
    else:
        work = synth.c2_sheath(seed=args.seed, ncells=args.ncells, ppc=args.ppc)
    e = work["ensembles"][0]
    # the variants switch features on; the sheath cases keep their own walls and filter
    if args.floating:
        e["floating"] = True
    if args.smooth:
        e["smooth"] = int(args.smooth)
    if args.shape:
        ppt, window, sort_ppt, nt = (int(v) for v in args.shape.split(","))
        shape = {"ppt": ppt, "window": window, "sort_ppt": sort_ppt, "nontemporal": nt}
    else:
        shape = tuned_shape(pic, work, args.tune_steps)
    sim = pic.Sim(work, fused=not args.separate, precision="fp64" if args.fp64 else None, **shape)
    n_ens = len(work["ensembles"])

    def total(d_list, key):
        return sum(sum(d[key]) if isinstance(d[key], list) else d[key] for d in d_list)

    # warm-up, then instantiate the graphs the timed steps replay (a whole sort cycle from
    # the phase the warm-up ends in, and a shorter tail), so no capture is timed
    sim.step(args.warmup)
    sim.prepare(args.steps)
    torch.cuda.synchronize()
    d0 = [sim.diag(k) for k in range(n_ens)]
    g0 = sim.graph_launches()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    graph_launches = sim.graph_launches() - g0
    d1 = [sim.diag(k) for k in range(n_ens)]
    pushes = total(d1, "pushes") - total(d0, "pushes")
    wall = t1 - t0
    value = pushes / wall

    # dominant kernel: the fused particle pass, timed with HIP events on the library's
    # launch stream over a run of the same steps without the graph (the hook skips the one
    # pass in K that also sorts, a kernel of its own); every pass pushes every live
    # particle, so a launch's pushes are the run's pushes per step
    sim.timing(True)
    dt0 = total([sim.diag(k) for k in range(n_ens)], "pushes")
    nt = min(args.steps, 200)
    sim.step(nt)
    ms_tot, launches = sim.timing_read()
    sim.timing(False)
    dt1 = total([sim.diag(k) for k in range(n_ens)], "pushes")
    pass_pushes = (dt1 - dt0) / nt
    avg_ms = ms_tot / max(launches, 1)
    cells = sum(en["ncells"] for en in work["ensembles"])
    b_part = 68.0 if args.fp64 else B_ALG_PARTICLE
    bytes_per_launch = (b_part * pass_pushes + B_ALG_CELL * cells + B_ALG_NODE * (cells + n_ens))
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    plain_sheath = args.case == "sheath" and not args.floating and not args.smooth and not args.fp64
    traffic = traffic_from_profiles("sheath_1e5", bytes_per_launch) if plain_sheath else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": ("k_particles<" if args.fp64 else "k_pass32<")
                          + ("push>" if args.separate else "push|collide|deposit>"),
                "avg_launch_ms": round(avg_ms, 5), "bytes_alg_per_launch": bytes_per_launch,
                "launches_timed": launches}
    # algorithmic bytes of a whole step: 44 B per push, the sort's 48 B per particle every K
    # steps, 40 B per node for the grid (Q written and read, E written and read) and 24 B per
    # created particle
    created = total(d1, "created") - total(d0, "created")
    step_bytes = ((b_part + (72.0 if args.fp64 else 48.0) / e["sort_every"]) * (pushes / args.steps)
                  + 40.0 * (cells + n_ens) + 24.0 * created / args.steps)
    whole_step = {"bytes_alg_per_step": step_bytes,
                  "frac_of_hbm_peak": round(step_bytes / (wall / args.steps) / 1e9 / HBM_PEAK_GBS, 4)}
    del sim
    torch.cuda.empty_cache()

    plain = None
    if not args.no_plain:
        psim = pic.Sim(work, fused=False, precision="fp64")
        psim.step(2)
        torch.cuda.synchronize()
        p0 = psim.diag()["pushes"]
        pn = max(10, args.steps // 20)
        tp0 = time.perf_counter()
        psim.step(pn)
        torch.cuda.synchronize()
        tp1 = time.perf_counter()
        pp = psim.diag()["pushes"] - p0
        plain = {"value": pp / (tp1 - tp0), "ms_per_step": (tp1 - tp0) / pn * 1e3, "steps": pn,
                 "form": "FP64 x/v particles, one kernel per stage, FP64 atomics deposit, no graph",
                 "frac_of_hbm_peak_68B": round(68.0 * pp / (tp1 - tp0) / 1e9 / HBM_PEAK_GBS, 4)}
        del psim
        torch.cuda.empty_cache()

    batched = None
    if not args.no_batched:
        batched = batched_run(pic, shape, args.batched_steps)

    walls = None
    if not args.no_walls_variant:
        walls = walls_variant_run(pic, shape, args.batched_steps, args.seed, 2)
    cases = None
    if not args.no_sheath_cases:
        cases = {"recycling": sheath_case_run(pic, shape, "recycling", args.seed, 20, args.batched_steps),
                 "source": sheath_case_run(pic, shape, "source", args.seed, 200, args.batched_steps,
                                           refill=800)}

    large = None
    if not args.no_large:
        large = large_run(pic, shape, args.seed, 10, 20)

    small = None
    if not args.no_small:
        small = correctness_configs_run(pic)

    stream = None
    if not args.no_stream:
        stream = stream_copy_gbs(torch, pic)

    cpu = None if args.no_cpu else cpu_baseline(args.seed, args.cpu_steps, args.cpu_omp_steps)
    if args.calib_copy_gib > 0:
        # counter calibration: one copy of known size with the pass's own access pattern
        # (k_stream_copy<true>: 16-byte non-temporal loads and stores)
        n = int(args.calib_copy_gib * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        pic.stream_copy(a, b, nontemporal=True)
        torch.cuda.synchronize()
        del a, b

    out = {
        "metric": "particle-pushes/s per full step at 1 MI355X",
        "value": value, "unit": "particle-pushes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"sheath slab {e['ncells']} cells x {e['species'][0]['ppc']} ppc x 2 species, "
                                f"oblique B, 3 collision channels, sort every {e['sort_every']}"
                                + (", floating walls" if args.floating else "")
                                + (f", {args.smooth} smoothing passes" if args.smooth else ""))
                               if args.case == "sheath" else work["name"],
                   "particles": 2 * e["species"][0]["ppc"] * e["ncells"], "seed": args.seed,
                   "form": ("FP32 cell+offset, fused pass, "
                            + (f"{graph_launches} HIP graph replays" if graph_launches else "eager launches")
                            if not args.separate else "FP32 cell+offset, one kernel per stage"),
                   "parallelism": "single GPU", "launch_shape": shape},
        "roofline": roofline,
        "whole_step": whole_step,
        "plain": plain,
        "batched": batched,
        "floating_walls_smoothed": walls,
        "sheath_cases": cases,
        "large": large,
        "correctness_configs": small,
        "stream_copy": stream,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
