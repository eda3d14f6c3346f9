#!/usr/bin/env python
"""Throughput of the MPCD + rigid-body step on one MI355X.

Headline workload: 512 independent periodic replicas advanced together, cubic
boxes with edges drawn uniformly from 12..24 cells (a = 1), 5 solvent per cell
(17,376,750 solvent in all), one rigid sphere of radius 2 with 100 Fibonacci
surface sites in each; SRD 130 degrees, dt = 0.1, kT = 1 with the cell
thermostat; a random stream per replica; synthetic seeded inputs
(Maxwell-Boltzmann velocities).  The headline value is the batched FP32 form
in the binned solvent layout (FP32 solvent records and sites, exact int64
fixed-point cell sums, FP64 bodies); the dense FP32 form and the plain FP64
form run on the same workload beside it, with the FP32-binned / FP64 ratio.

One step = site thermalization and listing, the brick collision (collide,
stream and bin the solvent for the next step in one pass), momentum transfer
and the rigid-body update; the dense forms bin with a counting sort instead.
Inputs are resident in HBM; the timed region replays a HIP graph of the steps.

The other workloads run after the headline, each form with the roofline of
its dominant kernel: the 60^3 hard-sphere suspension (1.08M solvent, 191
spheres), the 200^3 suspension at volume fraction 0.3 (80M solvent, 21,221
spheres) and the 128^3 complex-shape suspension (21M solvent, 2,000 cubes,
rods and dumbbells with site-site WCA).

The dominant kernel is timed on its own with HIP events on its stream: for the
binned layout, back-to-back launches of mpcd_binned_collide on one step's
input; for the dense forms, of mpcd_collide_drawn repeating the last step's
collide + stream pass.

Prints one JSON line (N = 1).
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SRCS = [os.path.join(ROOT, "paper_2604_14307_amd", "csrc", f) for f in ("mpcd.hip", "detrand.hpp")]
# committed rocprofv3 counter summaries: profiles/<kernel>_<workload>_traffic.txt
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def collide_bytes(N, S, prec_bytes):
    """Algorithmic bytes of one fused collide + stream launch: read and write
    each solvent particle's position and velocity once (12 components), read
    and write each site's velocity once and read its mass."""
    return N * 4 * 3 * prec_bytes + S * (2 * 3 * prec_bytes + 8)


def kernel_source_hash():
    """First 16 hex digits of the SHA-256 of the kernel sources (the HIP file
    and the header of device primitives it includes), concatenated."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, wtag):
    """HBM bytes per launch of `kernel` on workload `wtag` from the committed
    rocprofv3 counter summary, or None when there is none, it covers another
    kernel or the kernel source has changed since the counters were taken."""
    path = os.path.join(PROFILES, "%s_%s_traffic.txt" % (kernel, wtag))
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash() or vals.get("kernel") != kernel:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# Launch shapes: read from the committed cache of tuned shapes (one entry per
# GPU architecture, precision and workload size); a workload missing from it
# is tuned on the spot (untimed) and, with --tune-out, recorded in that file.
# --retune tunes every workload again and writes the cache file it names.
TUNE = {"on": True, "cache": os.path.join(ROOT, "paper_2604_14307_amd", "tuning_gfx950.json"), "write": None,
        "out": None}


def run_gpu(systems, par, prec, steps, warmup, repeats, kernel_reps, rnemd=None, tuning=None, layout="dense"):
    """Time graph replays of the step.  tuning: None = autotune the launch
    shapes on this system first (untimed; unless disabled), else a fixed
    (items, fill, draw_cells).  layout "binned": the binned solvent layout
    (no tunable shapes)."""
    import torch
    from paper_2604_14307_amd import tune
    from paper_2604_14307_amd.sim import GPUSystem

    g = GPUSystem(systems, par, prec=prec, device="cuda:0", layout=layout)
    g.body_forces()
    if rnemd is not None:
        g.set_rnemd(*rnemd)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    # out-of-place graphs hold an even number of steps: split the K timed
    # steps into the most replays (at most `repeats`) of equal even length
    if steps < 2 or steps % 2:
        raise SystemExit("out-of-place graphs step in pairs: the number of timed steps must be even")
    repeats = max(r for r in range(1, repeats + 1) if steps % r == 0 and (steps // r) % 2 == 0)
    per = steps // repeats
    with torch.cuda.stream(side):
        for i in range(warmup):  # eager warmup (also pages in the code objects)
            g.step(1)
    tuned = None
    if layout == "binned":
        pass
    elif tuning is not None:
        g.set_tuning(*tuning)
    elif TUNE["on"]:
        if TUNE["write"]:
            tuned = tune.autotune(g, steps=min(20, per), repeats=3, cache_path=TUNE["write"], retune=True)
        else:
            tuned = tune.autotune(g, steps=min(20, per), repeats=3, cache_path=TUNE["cache"], write=False)
        if tuned["cached"]:
            log("  launch shape %s (tile %s) from the cache" % (tuned["tune"], tuned["tile"]))
        else:
            log("  launch shape %s (tile %s) tuned now: %.4f ms/step, default %.4f"
                % (tuned["tune"], tuned["tile"], tuned["ms_per_step"], tuned["default_ms_per_step"]))
            if TUNE["out"]:  # keep the new entry (merged into that file)
                cache = tune.load_cache(TUNE["out"])
                cache[tune.workload_key(g)] = {k: v for k, v in tuned.items() if k != "cached"}
                with open(TUNE["out"], "w") as f:
                    json.dump(cache, f, indent=1, sort_keys=True)
    with torch.cuda.stream(side):
        g.graph(per)
        g.graph_launch()  # one untimed replay
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(repeats + 1)]
        ev[0].record(side)
        for r in range(repeats):
            g.graph_launch()
            ev[r + 1].record(side)
        torch.cuda.synchronize()
        seg = [ev[r].elapsed_time(ev[r + 1]) for r in range(repeats)]
        kms = None
        fpms = None
        if kernel_reps > 0 and layout == "binned":
            # the current step's sites listed once, then back-to-back launches
            # of the brick collision of that step (its inputs are left
            # unchanged; each launch first clears the next step's region fills)
            g.graph_launch()
            g.binned_sites()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(side)
            for _ in range(kernel_reps):
                g.binned_collide()
            b.record(side)
            torch.cuda.synchronize()
            kms = a.elapsed_time(b) / kernel_reps
        elif kernel_reps > 0:
            # keep the GPU busy with one more replay while the host enqueues the
            # back-to-back launches, so launch latency is not counted; each
            # launch repeats the last step's collide + stream pass (same inputs,
            # same cell lists and draws, same output arrays)
            g.graph_launch()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(side)
            for _ in range(kernel_reps):
                g.recollide_last(restore_sites=False)
            b.record(side)
            torch.cuda.synchronize()
            kms = a.elapsed_time(b) / kernel_reps
            if g.tuning.overlap == 2 and g.B > 0 and g.S > 0:
                # the fused force + next-binning kernel runs in the timed
                # schedule: time it the same way (repeated launches on the
                # state after a replay; the system is not stepped afterwards)
                nxt = g.d_step + 1
                g.graph_launch()
                a.record(side)
                for _ in range(kernel_reps):
                    g.forces_prep(nxt)
                b.record(side)
                torch.cuda.synchronize()
                fpms = a.elapsed_time(b) / kernel_reps
        g.release_graph()
        flags = g.status()
    if flags != 0:
        raise SystemExit("device status flags %d in the %s run" % (flags, prec))
    total_steps = per * repeats
    ms = sum(seg)
    return dict(ms=ms, steps=total_steps, ms_step=ms / total_steps,
                ms_step_median=statistics.median(seg) / per, collide_ms=kms, forces_prep_ms=fpms,
                rate=g.N * total_steps / (ms * 1e-3), N=g.N, S=g.S, B=g.B, C=g.C, nsys=g.nsys,
                tuning=tuning_record(g, tuned), layout=layout)


def tuning_record(g, tuned):
    if g.binned is not None:
        b = g.binned
        return {"layout": "binned", "bricks": int(b.nbricks), "capacity": int(b.capacity),
                "members_per_thread": int(b.items)}
    t = g.tuning
    rec = {"tune_items_fill_drawcells_inline_overlap": [t.tile_items, t.tile_fill, t.draw_cells, t.draws_inline,
                                                         t.overlap],
           "tile_items_cells_cap_tiles": list(g.tile_shape())}
    if tuned:
        rec["source"] = "cache" if tuned["cached"] else "tuned in this run"
        rec["default_ms_per_step_when_tuned"] = tuned["default_ms_per_step"]
    return rec


def collide_kernel_name(items, draws_inline=0, f64=False):
    base = ({1: "k_collide_tiled_f64_i1", 2: "k_collide_tiled_f64", 4: "k_collide_tiled_f64_i4"} if f64 else
            {2: "k_collide_tiled_f32_i2", 4: "k_collide_tiled_f32", 8: "k_collide_tiled_f32_i8"})[items]
    return base + ("_d" if draws_inline else "")


def forces_prep_bytes(N, S, prec_bytes):
    """Algorithmic bytes of one fused forces + next-binning launch: each solvent
    particle's position read and its cell and slot written; each site's
    body-frame offset and mass read and its offset, position, velocity,
    pre-collision velocity, cell and slot written (bodies: negligible)."""
    return N * (3 * prec_bytes + 8) + S * (24 + 8 + 24 + 6 * prec_bytes + 24 + 8)


def step_bytes(N, S, prec_bytes):
    """Algorithmic HBM bytes of one whole step: each solvent particle's x and v
    read and written once, each site's position and velocity written by the
    thermalization and its velocity read and written by the collision, its
    offset, mass and pre-collision velocity read (bodies: negligible)."""
    return N * 4 * 3 * prec_bytes + S * (4 * 3 * prec_bytes + 3 * 8 + 8 + 3 * 8)


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size, for scaling the FETCH_SIZE/WRITE_SIZE
    counters (run under rocprofv3 --pmc)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)  # device-to-device copy (blit kernel)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)  # the same traffic through an elementwise kernel
    torch.cuda.synchronize()
    log("copy calibration: 3 copies and 3 scale-by-one passes of %d bytes" % nbytes)


def run_harmonic(wl, par, dt_md, nsub, periods, repeats):
    """Time per collision period of the harmonic-bond comparator (FP64)."""
    import torch
    from paper_2604_14307_amd import workloads as W
    from paper_2604_14307_amd.sim import HarmonicGPU

    g = HarmonicGPU(W.harmonic_from_rigid(wl), dict(par, thermalize=0), device="cuda:0")
    g.forces()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g.step(dt_md, nsub, 2)
        g.graph(dt_md, nsub, periods)
        g.graph_launch()
        torch.cuda.synchronize()
        ms = []
        for _ in range(repeats):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(side)
            g.graph_launch()
            b.record(side)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b) / periods)
        g.release_graph()
        flags = g.status()
    if flags != 0:
        raise SystemExit("device status flags %d in the harmonic run" % flags)
    return statistics.median(ms)


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return "%s, %d logical CPUs visible" % (model, os.cpu_count() or 0)


def cpu_baseline(systems, par, steps):
    """The oracle as it stands, one thread: `steps` steps of every system."""
    import oracle
    os_ = [oracle.OracleSystem(wl, par, replica=r) for r, wl in enumerate(systems)]
    for o in os_:
        o.body_forces()
    t0 = time.perf_counter()
    for o in os_:
        o.run(0, steps)
    dt = time.perf_counter() - t0
    return sum(o.N for o in os_) * steps / dt, dt


def summary(r):
    return {"value": r["rate"], "ms_per_step": r["ms_step"], "ms_per_step_median_replay": r["ms_step_median"],
            "steps": r["steps"], "solvent": r["N"], "sites": r["S"], "bodies": r["B"], "cells": r["C"],
            "systems": r["nsys"], "tuning": r["tuning"]}


WORKLOADS = {1: "suspension60", 2: "suspension200", 3: "batched512", 4: "shapes128"}


def brick_bytes(N, S):
    """Algorithmic bytes of one brick collision (FP32): each solvent
    particle's position and velocity read and written once; each site's
    position and velocity read, its mass read and its velocity written."""
    return N * 4 * 3 * 4 + S * (3 * 4 + 3 * 4 + 8 + 3 * 4)


def roofline(r, prec_bytes, wtag):
    """Roofline object of the run's dominant kernel: the collide + stream pass
    (or the fused force + next-binning kernel when that launch is longer),
    timed live; algorithmic bytes per launch over its average duration."""
    N, S = r["N"], r["S"]
    if r.get("layout") == "binned":
        kern, ms, nbytes = "k_brick_collide_f32", r["collide_ms"], brick_bytes(N, S)
        ach = nbytes / (ms * 1e-3) / 1e9
        traffic = measured_traffic(kern, wtag)
        return {"bound": "hbm", "kernel": kern + " (binned layout: collide + stream + bin for the next step)",
                "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": ach / PEAK_HBM_GBS,
                "traffic": traffic, "avg_launch_us": ms * 1e3, "algorithmic_bytes_per_launch": nbytes,
                # measured HBM bytes (committed counters) over the live launch time
                "traffic_frac": None if traffic is None else traffic / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    kname = collide_kernel_name(r["tuning"]["tile_items_cells_cap_tiles"][0],
                                r["tuning"]["tune_items_fill_drawcells_inline_overlap"][3], prec_bytes == 8)
    kern, ms, nbytes = kname, r["collide_ms"], collide_bytes(N, S, prec_bytes)
    label = kname + (" (collide + stream + per-cell draws)" if kname.endswith("_d") else " (collide + stream)")
    fp_ms = r.get("forces_prep_ms")
    if fp_ms and fp_ms > ms:
        kern, ms, nbytes = "k_forces_prep", fp_ms, forces_prep_bytes(N, S, prec_bytes)
        label = kern + " (body forces + kick, then the next step's site thermalization and binning)"
    ach = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": label, "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": ach / PEAK_HBM_GBS, "traffic": measured_traffic(kern, wtag), "avg_launch_us": ms * 1e3,
            "algorithmic_bytes_per_launch": nbytes}


def form_summary(r, prec_bytes, wtag):
    out = summary(r)
    out["roofline"] = roofline(r, prec_bytes, wtag)
    out["step_hbm_frac"] = step_bytes(r["N"], r["S"], prec_bytes) / (r["ms_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed steps of the headline (batched FP32) form")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5, help="graph replays the K timed steps are split into")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--other-steps", type=int, default=40, help="timed steps of every other workload")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle steps over all replicas of the headline workload for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-binned", action="store_true", help="skip the binned solvent layout (headline: dense)")
    ap.add_argument("--only-headline", action="store_true", help="skip every other workload")
    ap.add_argument("--no-large", action="store_true", help="skip the 200^3-cell, 80M-solvent suspension")
    ap.add_argument("--no-shapes", action="store_true", help="skip the 128^3 complex-shape suspension")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-harmonic", action="store_true",
                    help="skip the rigid-vs-harmonic time per tau on the paper's benchmark geometry")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes (no cached or tuned shapes)")
    ap.add_argument("--retune", metavar="PATH", default=None,
                    help="tune every workload again (untimed) and write the shapes to this JSON cache")
    ap.add_argument("--no-rnemd", action="store_true",
                    help="skip the step time with the reverse nonequilibrium exchange appended")
    ap.add_argument("--tune-out", metavar="PATH", default=None,
                    help="record the shapes of workloads tuned on the spot (missing from the cache) in this JSON file")
    ap.add_argument("--only-workload", type=int, choices=sorted(WORKLOADS), default=None,
                    help="time this one workload only, in the forms selected (for profiler runs; the JSON line "
                         "then holds that workload's block)")
    ap.add_argument("--forms", default=None,
                    help="comma-separated forms to run among f32_binned, f32, f64 (default: all)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this implementation drives a single MI355X "
              "(how the step would shard over several GPUs is a design note, not a built path).",
              file=sys.stderr)
        sys.exit(2)
    if args.steps < args.repeats:
        raise SystemExit("--steps must be at least --repeats")
    TUNE["on"] = not args.no_tune
    TUNE["write"] = args.retune
    TUNE["out"] = args.tune_out
    # forms: (name, precision, solvent layout); the headline is the first
    forms = [("f32_binned", "f32", "binned"), ("f32", "f32", "dense")] + ([] if args.no_fp64 else
                                                                        [("f64", "f64", "dense")])
    if args.no_binned:
        forms = forms[1:]
    if args.forms:
        keep = args.forms.split(",")
        forms = [f for f in forms if f[0] in keep]
        if not forms:
            raise SystemExit("--forms selects none of f32_binned, f32, f64")
    from paper_2604_14307_amd import workloads as W
    if args.only_workload is not None:
        ci = args.only_workload
        wl, par, meta = W.config(ci, kT_cell=1.0)
        block = {"workload": meta["name"]}
        steps = args.steps if ci == 3 else args.other_steps
        for name, prec, layout in forms:
            log("%s %s: %d timed steps" % (WORKLOADS[ci], name, steps))
            rr = run_gpu(wl, par, prec, steps, 4, 2, args.kernel_reps, layout=layout)
            log("%s %s: %.4f ms/step, dominant kernel %.2f us" % (WORKLOADS[ci], name, rr["ms_step"],
                                                                 rr["collide_ms"] * 1e3))
            block[name] = form_summary(rr, 4 if prec == "f32" else 8, WORKLOADS[ci])
        if args.copy_calibration:
            copy_calibration()
        print(json.dumps({WORKLOADS[ci]: block}), flush=True)
        return

    bsys, bpar, bmeta = W.config(3, kT_cell=1.0)
    res = {}
    for name, prec, layout in forms:
        log("batched replicas %s: warmup %d, %d timed steps in at most %d replays" % (name, args.warmup, args.steps,
                                                                                     args.repeats))
        res[name] = run_gpu(bsys, bpar, prec, args.steps, args.warmup, args.repeats, args.kernel_reps,
                            layout=layout)
        r = res[name]
        log("batched %s: %.4f ms/step (median replay %.4f), dominant kernel %.2f us"
            % (name, r["ms_step"], r["ms_step_median"], r["collide_ms"] * 1e3))
    head = forms[0][0]
    r32 = res[head]
    N, S = r32["N"], r32["S"]
    out = {
        "metric": "solvent particle-steps/s",
        "value": r32["rate"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": r32["steps"],
        "warmup": args.warmup,
        "ms_per_step": r32["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched replicas: 512 periodic boxes, edges uniform in 12..24 cells, 5 solvent "
                               "per cell (17,376,750 solvent), one rigid sphere r=2 x 100 sites each, SRD 130 deg, "
                               "dt=0.1, kT=1, cell thermostat, a random stream per replica",
                   "systems": r32["nsys"], "solvent": N, "sites": S, "bodies": r32["B"], "cells": r32["C"],
                   "form": "FP32 solvent/sites + int64 fixed-point cell sums + FP64 bodies; %s solvent layout; "
                           "HIP graph replays of the step" % r32["layout"]},
        "ms_per_step_median_replay": r32["ms_step_median"],
        "roofline": roofline(r32, 4, WORKLOADS[3]),
        "tuning": r32["tuning"],
        # the whole step against the HBM peak: algorithmic bytes of a step / step time
        "step_hbm_frac": step_bytes(N, S, 4) / (r32["ms_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS,
    }
    for name, prec, layout in forms[1:]:
        out[name] = form_summary(res[name], 4 if prec == "f32" else 8, WORKLOADS[3])
    if "f64" in res:
        out["speedup_batched_fp32_vs_plain_fp64"] = r32["rate"] / res["f64"]["rate"]
    others = [] if args.only_headline else [1] + ([] if args.no_large else [2]) + ([] if args.no_shapes else [4])
    for ci in others:
        wl, par, meta = W.config(ci, kT_cell=1.0)
        block = {"workload": meta["name"]}
        for name, prec, layout in forms:
            log("%s %s: %d timed steps" % (WORKLOADS[ci], name, args.other_steps))
            rr = run_gpu(wl, par, prec, args.other_steps, 4, 2, args.kernel_reps, layout=layout)
            log("%s %s: %.4f ms/step, dominant kernel %.2f us" % (WORKLOADS[ci], name, rr["ms_step"],
                                                                 rr["collide_ms"] * 1e3))
            block[name] = form_summary(rr, 4 if prec == "f32" else 8, WORKLOADS[ci])
        if "f64" in block:
            block["speedup_fp32_vs_fp64"] = block[forms[0][0]]["value"] / block["f64"]["value"]
        out[WORKLOADS[ci]] = block
        del wl
    if not args.no_harmonic and not args.only_headline:
        hw, hpar, hmeta = W.paper_benchmark(0.1)
        res_h = {"workload": hmeta["name"],
                 "protocol": "rigid: one step per collision, dt = 0.1; harmonic: collision every 0.1 tau, "
                             "50 velocity-Verlet steps of 0.002 between collisions (Sec. II.B.1)"}
        for name, prec, layout in (("f64", "f64", "dense"), ("f32", "f32", "dense"), ("f32_binned", "f32", "binned")):
            log("paper geometry, rigid %s: 20 timed steps" % name)
            rr = run_gpu(hw, hpar, prec, 20, 6, 2, 0, layout=layout)
            res_h["rigid_%s_ms_per_tau" % name] = rr["ms_step"] * 10.0
        log("paper geometry, harmonic FP64: 10 timed collision periods")
        hper = run_harmonic(hw, hpar, 0.002, 50, 10, 3)
        res_h["harmonic_f64_ms_per_tau"] = hper * 10.0
        res_h["speedup_rigid_f64_vs_harmonic_f64"] = res_h["harmonic_f64_ms_per_tau"] / res_h["rigid_f64_ms_per_tau"]
        res_h["speedup_rigid_f32_vs_harmonic_f64"] = res_h["harmonic_f64_ms_per_tau"] / res_h["rigid_f32_ms_per_tau"]
        res_h["speedup_rigid_f32_binned_vs_harmonic_f64"] = (res_h["harmonic_f64_ms_per_tau"]
                                                            / res_h["rigid_f32_binned_ms_per_tau"])
        res_h["paper"] = "rigid (dt 0.1) vs harmonic (dt 0.002): nearly an order of magnitude, 1x A100, HOOMD-blue"
        out["rigid_vs_harmonic"] = res_h
        del hw
    if not args.no_rnemd and not args.only_headline:
        vw, vpar, vmeta, vrn = W.paper_viscosity(0.1)
        pv = {"workload": vmeta["name"]}
        for label, rn_v in (("plain", None), ("exchange", vrn)):
            log("paper viscosity geometry FP32, %s: 40 timed steps" % label)
            rv = run_gpu(vw, vpar, "f32", 40, 4, 2, 0, rnemd=rn_v)
            pv["f32_%s_ms_per_step" % label] = rv["ms_step"]
        pv["f32_overhead"] = pv["f32_exchange_ms_per_step"] / pv["f32_plain_ms_per_step"] - 1.0
        out["rnemd"] = {"paper_geometry": pv}
        del vw
    if args.copy_calibration:
        copy_calibration()
    if not args.no_cpu_baseline:
        log("oracle on the host: %d steps of all %d replicas" % (args.cpu_steps, len(bsys)))
        rate, secs = cpu_baseline(bsys, bpar, args.cpu_steps)
        out["cpu_baseline"] = {"value": rate, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
                               "sample": "%d steps of all 512 replicas of the headline workload (FP64 C oracle, "
                                         "one thread, %.1f s)" % (args.cpu_steps, secs),
                               "host": host_cpu()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
