"""Launch-shape autotuner for the fused step.

The step's launch shapes (``mpcd_tune``: items per thread of a collision
tile, the fill that sets the cells per tile, cells per lane of the per-cell
draws, draws inside the collision or in a pass of their own, and the schedule
of each next step's first kernel in graphs: on a second stream beside the body
update, inside the force kernel, or with the solvent binned by the collision)
change how work is split over blocks and streams, never the results.
The tuner times HIP-graph replays of a few steps of the caller's own system
for each distinct collision shape, then each schedule on top of the two
fastest shapes (which bounds the tuning time), restores the state after every
trial, keeps the fastest shape on the system and records it in a JSON cache
keyed by the GPU architecture, the precision and the system sizes, so a later
run on the same workload reuses it without timing.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import lib as L

FILLS = (40, 55, 70, 85)
ITEMS = {"f32": (2, 4, 8), "f64": (1, 2, 4)}
DRAW_CELLS = (1, 2)
DRAWS_INLINE = (0, 1)
OVERLAP = (0, 1, 2, 3)
SCHEDULE_SHAPES = 2


def arch(device) -> str:
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def prec_name(g) -> str:
    return "f64" if g.prec == L.MPCD_F64 else "f32"


def workload_key(g) -> str:
    return "%s|%s|N%d|S%d|B%d|C%d|nsys%d" % (arch(g.device), prec_name(g), g.N, g.S, g.B, g.C, g.nsys)


def candidates(g):
    """Distinct collision shapes (items, fill, draw_cells, draws_inline, 0):
    tunings with the same tile shape and the same draws are the same launch
    (cells per lane do not matter when the collision draws).  The default
    comes first."""
    seen, out = set(), []
    for items in ITEMS[prec_name(g)]:
        for fill in FILLS:
            for inl in DRAWS_INLINE:
                for dc in (DRAW_CELLS if not inl else (1,)):
                    shape = g.tile_shape((items, fill, dc, inl))
                    key = (shape[0], shape[1], dc, inl)
                    if key not in seen:
                        seen.add(key)
                        out.append((items, fill, dc, inl, 0))
    d = g.tile_shape((0, 0, 0, 0, 0))
    default = next(c for c in out if g.tile_shape(c)[:2] == d[:2] and c[2] == 1 and c[3] == 0)
    out.remove(default)
    return [default] + out


def time_shape(g, tune, steps, repeats):
    """Median ms per step of graph replays of `steps` steps with shape `tune`."""
    g.set_tuning(*tune)
    side = torch.cuda.Stream(device=g.device)
    torch.cuda.synchronize(g.device)
    with torch.cuda.stream(side):
        g.graph(steps)
        g.graph_launch()  # untimed
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(repeats + 1)]
        ev[0].record(side)
        for r in range(repeats):
            g.graph_launch()
            ev[r + 1].record(side)
        torch.cuda.synchronize(g.device)
        g.release_graph()
    return statistics.median(ev[r].elapsed_time(ev[r + 1]) for r in range(repeats)) / steps


def load_cache(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def autotune(g, steps: int = 20, repeats: int = 3, cache_path: str | None = None, retune: bool = False,
             write: bool = True) -> dict:
    """Pick the fastest launch shape for system g and set it.  Returns
    {"tune": (items, fill, draw_cells, draws_inline, overlap), "ms_per_step", "default_ms_per_step",
    "shapes_tried", "tile", "cached"}.  The simulation state is unchanged.  A
    shape cached for this workload is used as it is unless retune; a new
    result is written to cache_path when write."""
    if steps % 2 and g.out_of_place:
        raise ValueError("out-of-place graphs hold an even number of steps")
    key = workload_key(g)
    cache = load_cache(cache_path)
    if key in cache and not retune:
        e = dict(cache[key])
        g.set_tuning(*e["tune"])
        e["cached"] = True
        return e
    if g.status() != 0:  # (synchronizes) a flag from earlier work is not the tuner's
        raise RuntimeError("device status flags %d before tuning" % g.status())
    snap = g.snapshot()
    results = []
    for cand in candidates(g):
        g.restore(snap)
        results.append((time_shape(g, cand, steps, repeats), cand))
    if g.B > 0 and g.S > 0 and g.out_of_place and steps >= 2:  # the schedules need sites and out-of-place graphs
        # each schedule on the SCHEDULE_SHAPES fastest shapes: a schedule moves
        # work into or out of the collision, which can reorder close shapes
        for _, best in sorted(results)[:SCHEDULE_SHAPES]:
            for ov in OVERLAP[1:]:
                g.restore(snap)
                cand = best[:4] + (ov,)
                results.append((time_shape(g, cand, steps, repeats), cand))
    g.restore(snap)
    torch.cuda.synchronize(g.device)
    if g.status() != 0:
        raise RuntimeError("device status flags %d while tuning" % g.status())
    best_ms, best = min(results)
    g.set_tuning(*best)
    e = {"tune": list(best), "ms_per_step": best_ms, "default_ms_per_step": results[0][0],
         "shapes_tried": len(results), "tile": list(g.tile_shape(best)), "cached": False}
    if cache_path and write:
        cache[key] = {k: v for k, v in e.items() if k != "cached"}
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return e
