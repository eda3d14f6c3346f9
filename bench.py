#!/usr/bin/env python
"""Throughput of the MPCD + rigid-body step on one MI355X.

Headline workload: hard-sphere suspension, 60^3 cells (a = 1, periodic), 5
solvent per cell (1,080,000 solvent), 191 rigid spheres of radius 3 with 200
Fibonacci surface sites each (volume fraction 0.1), WCA between body centres
(sigma 6, eps = kT), SRD 130 degrees, dt = 0.1, kT = 1 with the cell
thermostat; synthetic seeded inputs (random sequential addition,
Maxwell-Boltzmann velocities).

One step = site thermalization, grid shift + counting sort, SRD collision
(fused with solvent streaming), momentum transfer, rigid-body update.  Inputs
are resident in HBM; the timed region replays a HIP graph of the steps.  The
headline value is the FP32 form (FP32 solvent/sites, exact int64 fixed-point
cell sums, FP64 bodies); the plain FP64 form is measured alongside, and both
forms are also run on 512 independent replicas of uneven box size advanced
together (the batched form).

The solvent is double-buffered: every step writes it out of place in cell
order.  The dominant kernel (the fused collide + stream pass) is timed on its
own with HIP events on its stream: back-to-back launches of mpcd_collide_drawn
repeating the last step's pass (its inputs, cell lists and draws).

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
# committed rocprofv3 counter summaries of the 60^3 FP32 kernels, by kernel family
TRAFFIC_FILES = {"collide": os.path.join(ROOT, "profiles", "collide_f32_suspension60_traffic.txt"),
                 "forces_prep": os.path.join(ROOT, "profiles", "forces_prep_f32_suspension60_traffic.txt")}


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


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when it covers another kernel or the kernel source has
    changed since the counters were taken."""
    path = TRAFFIC_FILES["forces_prep" if "forces_prep" in kernel else "collide"]
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
# is tuned on the spot (untimed).  --retune tunes every workload again and
# writes the cache given by --tune-cache.
TUNE = {"on": True, "cache": os.path.join(ROOT, "paper_2604_14307_amd", "tuning_gfx950.json"), "write": None}


def run_gpu(systems, par, prec, steps, warmup, repeats, kernel_reps, rnemd=None, tuning=None):
    """Time graph replays of the step.  tuning: None = autotune the launch
    shapes on this system first (untimed; unless disabled), else a fixed
    (items, fill, draw_cells)."""
    import torch
    from paper_2604_14307_amd import tune
    from paper_2604_14307_amd.sim import GPUSystem

    g = GPUSystem(systems, par, prec=prec, device="cuda:0")
    g.body_forces()
    if rnemd is not None:
        g.set_rnemd(*rnemd)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    per = max(2, 2 * (steps // (2 * repeats)))  # out-of-place graphs hold an even number of steps
    with torch.cuda.stream(side):
        for i in range(warmup):  # eager warmup (also pages in the code objects)
            g.step(1)
    tuned = None
    if tuning is not None:
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
        if kernel_reps > 0:
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
                tuning=tuning_record(g, tuned))


def tuning_record(g, tuned):
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


def cpu_baseline(wl, par, steps):
    import oracle
    o = oracle.OracleSystem(wl, par)
    o.body_forces()
    t0 = time.perf_counter()
    o.run(0, steps)
    dt = time.perf_counter() - t0
    return o.N * steps / dt, dt


def summary(r):
    return {"value": r["rate"], "ms_per_step": r["ms_step"], "ms_per_step_median_replay": r["ms_step_median"],
            "steps": r["steps"], "solvent": r["N"], "sites": r["S"], "bodies": r["B"], "cells": r["C"],
            "systems": r["nsys"], "tuning": r["tuning"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=25)
    ap.add_argument("--repeats", type=int, default=5, help="graph replays the K timed steps are split into")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--batched-steps", type=int, default=150)
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--large", action="store_true", help="also run the 200^3-cell, 80M-solvent suspension (FP32)")
    ap.add_argument("--shapes", action="store_true",
                    help="also run the 128^3 complex-shape suspension (site-site WCA), FP32 and FP64")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-harmonic", action="store_true",
                    help="skip the rigid-vs-harmonic time per tau on the paper's benchmark geometry")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch shapes (no cached or tuned shapes)")
    ap.add_argument("--retune", metavar="PATH", default=None,
                    help="tune every workload again (untimed) and write the shapes to this JSON cache")
    ap.add_argument("--no-rnemd", action="store_true",
                    help="skip the step time with the reverse nonequilibrium exchange appended")
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

    from paper_2604_14307_amd import workloads as W
    wl, par, meta = W.config(1, kT_cell=1.0)
    res = {}
    for prec in (("f32",) if args.no_fp64 else ("f32", "f64")):
        log("suspension 60^3 %s: warmup %d, %d timed steps in %d replays" % (prec, args.warmup, args.steps,
                                                                            args.repeats))
        res[prec] = run_gpu(wl, par, prec, args.steps, args.warmup, args.repeats, args.kernel_reps)
        r = res[prec]
        log("%s: %.4f ms/step (median replay %.4f), collide %.2f us" % (prec, r["ms_step"], r["ms_step_median"],
                                                                        r["collide_ms"] * 1e3))
    r32 = res["f32"]
    N, S = r32["N"], r32["S"]
    ach = collide_bytes(N, S, 4) / (r32["collide_ms"] * 1e-3) / 1e9
    # the roofline follows the longer launch of the two big kernels of the step
    fp_ms = r32.get("forces_prep_ms")
    if fp_ms and fp_ms > r32["collide_ms"]:
        rl_kernel, rl_ms, rl_bytes = "k_forces_prep<float>", fp_ms, forces_prep_bytes(N, S, 4)
        rl_label = rl_kernel + " (body forces + kick, then the next step's site thermalization and binning)"
    else:
        rl_kernel, rl_ms, rl_bytes = None, r32["collide_ms"], collide_bytes(N, S, 4)
        rl_label = None
    rl_ach = rl_bytes / (rl_ms * 1e-3) / 1e9
    kname = collide_kernel_name(r32["tuning"]["tile_items_cells_cap_tiles"][0],
                                r32["tuning"]["tune_items_fill_drawcells_inline_overlap"][3])
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
        "config": {"workload": "hard-sphere suspension: 60^3 cells, 1,080,000 solvent, 191 rigid spheres "
                               "r=3 x 200 sites, WCA sigma=6, SRD 130 deg, dt=0.1, kT=1, cell thermostat",
                   "solvent": N, "sites": S, "bodies": r32["B"], "cells": r32["C"],
                   "form": "FP32 solvent/sites + int64 fixed-point cell sums + FP64 bodies; "
                           "HIP graph replays of the step"},
        "ms_per_step_median_replay": r32["ms_step_median"],
        "roofline": {"bound": "hbm",
                     "kernel": rl_label or (kname + (" (collide + stream + per-cell draws)" if kname.endswith("_d")
                                                     else " (collide + stream)")),
                     "achieved": rl_ach, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": rl_ach / PEAK_HBM_GBS,
                     "traffic": measured_traffic(rl_kernel or kname), "avg_launch_us": rl_ms * 1e3,
                     "algorithmic_bytes_per_launch": rl_bytes},
        "collide": {"kernel": kname, "avg_launch_us": r32["collide_ms"] * 1e3, "achieved_GBs": ach,
                    "frac": ach / PEAK_HBM_GBS, "traffic": measured_traffic(kname),
                    "algorithmic_bytes_per_launch": collide_bytes(N, S, 4)},
        "tuning": r32["tuning"],
        # the whole step against the HBM peak: algorithmic bytes of a step / step time
        "step_hbm_frac": step_bytes(N, S, 4) / (r32["ms_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS,
    }
    if "f64" in res:
        r64 = res["f64"]
        a64 = collide_bytes(N, S, 8) / (r64["collide_ms"] * 1e-3) / 1e9
        out["fp64"] = dict(summary(r64), speedup_fp32_vs_fp64=r32["rate"] / r64["rate"],
                           collide_us=r64["collide_ms"] * 1e3, collide_GBs=a64)
    if not args.no_batched:
        bsys, bpar, bmeta = W.config(3, kT_cell=1.0)
        out["batched"] = {"workload": bmeta["name"]}
        for prec in (("f32",) if args.no_fp64 else ("f32", "f64")):
            log("batched replicas %s: %d timed steps" % (prec, args.batched_steps))
            rb = run_gpu(bsys, bpar, prec, args.batched_steps, 10, 3, 0)
            log("batched %s: %.4f ms/step" % (prec, rb["ms_step"]))
            out["batched"][prec] = summary(rb)
        if "f64" in out["batched"]:
            out["batched"]["speedup_fp32_vs_fp64"] = out["batched"]["f32"]["value"] / out["batched"]["f64"]["value"]
    if args.large:
        lw, lpar, lmeta = W.config(2, kT_cell=1.0)
        log("large suspension FP32: 50 timed steps")
        rl = run_gpu(lw, lpar, "f32", 50, 5, 5, 5)
        out["large"] = dict(summary(rl), workload=lmeta["name"], collide_us=rl["collide_ms"] * 1e3,
                            collide_GBs=collide_bytes(rl["N"], rl["S"], 4) / (rl["collide_ms"] * 1e-3) / 1e9)
        del lw
    if args.shapes:
        sw, spar, smeta = W.config(4, kT_cell=1.0)
        out["shapes"] = {"workload": smeta["name"]}
        for prec in ("f32", "f64"):
            log("complex shapes %s: 50 timed steps" % prec)
            rs = run_gpu(sw, spar, prec, 50, 6, 5, 0)
            out["shapes"][prec] = summary(rs)
        del sw
    if not args.no_harmonic:
        hw, hpar, hmeta = W.paper_benchmark(0.1)
        res_h = {"workload": hmeta["name"],
                 "protocol": "rigid: one step per collision, dt = 0.1; harmonic: collision every 0.1 tau, "
                             "50 velocity-Verlet steps of 0.002 between collisions (Sec. II.B.1)"}
        for prec in ("f64", "f32"):
            log("paper geometry, rigid %s: 20 timed steps" % prec)
            rr = run_gpu(hw, hpar, prec, 20, 6, 2, 0)
            res_h["rigid_%s_ms_per_tau" % prec] = rr["ms_step"] * 10.0
        log("paper geometry, harmonic FP64: 10 timed collision periods")
        hper = run_harmonic(hw, hpar, 0.002, 50, 10, 3)
        res_h["harmonic_f64_ms_per_tau"] = hper * 10.0
        res_h["speedup_rigid_f64_vs_harmonic_f64"] = res_h["harmonic_f64_ms_per_tau"] / res_h["rigid_f64_ms_per_tau"]
        res_h["speedup_rigid_f32_vs_harmonic_f64"] = res_h["harmonic_f64_ms_per_tau"] / res_h["rigid_f32_ms_per_tau"]
        res_h["paper"] = "rigid (dt 0.1) vs harmonic (dt 0.002): nearly an order of magnitude, 1x A100, HOOMD-blue"
        out["rigid_vs_harmonic"] = res_h
        del hw
    if not args.no_rnemd:
        # slabs of width 1 at y = 0 and y = 30, up to 100 pairs per step (Sec. III.B)
        rn = (0.0, 30.0, 1.0, 0.5, 100)
        res_rn = {"workload": "the headline suspension with the exchange after every step: slabs y in [0, 1) "
                              "and [30, 31), target |v_x| = 0.5, 100 pairs"}
        for prec in (("f32",) if args.no_fp64 else ("f32", "f64")):
            log("suspension 60^3 %s with the exchange: 100 timed steps" % prec)
            rr = run_gpu(wl, par, prec, 100, 6, 2, 0, rnemd=rn)
            res_rn["%s_ms_per_step" % prec] = rr["ms_step"]
            res_rn["%s_overhead" % prec] = rr["ms_step"] / res[prec]["ms_step"] - 1.0
        vw, vpar, vmeta, vrn = W.paper_viscosity(0.1)
        pv = {"workload": vmeta["name"]}
        for label, rn_v in (("plain", None), ("exchange", vrn)):
            log("paper viscosity geometry FP32, %s: 40 timed steps" % label)
            rv = run_gpu(vw, vpar, "f32", 40, 4, 2, 0, rnemd=rn_v)
            pv["f32_%s_ms_per_step" % label] = rv["ms_step"]
        pv["f32_overhead"] = pv["f32_exchange_ms_per_step"] / pv["f32_plain_ms_per_step"] - 1.0
        res_rn["paper_geometry"] = pv
        del vw
        out["rnemd"] = res_rn
    if args.copy_calibration:
        copy_calibration()
    if not args.no_cpu_baseline:
        log("oracle on the host: %d steps" % args.cpu_steps)
        rate, secs = cpu_baseline(wl, par, args.cpu_steps)
        out["cpu_baseline"] = {"value": rate, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
                               "sample": "%d steps of the same 60^3 suspension (FP64 C oracle, one thread, %.1f s)"
                                         % (args.cpu_steps, secs),
                               "host": host_cpu()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
