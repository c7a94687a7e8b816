"""Autotuner for the compositing kernels' launch shape.

For a given batch (device, views, pixel count, Gaussian count, SH degree) it
times, for the forward and the backward tile kernel separately, every
combination of pixels per lane (1, 2 or 4: four, two or one wavefront per
16x16 tile), LDS staging batch (1 or 2 splats per thread) and tile schedule
(one workgroup per tile launched heaviest first or in tile id order, or
persistent workgroups, as many as the GPU holds or half that, drawing tiles
heaviest first from counters) on the real step (eager launches, HIP events,
optimiser state restored afterwards), keeps the fastest and caches the
choice in a JSON file keyed by device name, library version and workload
shape (settings within 2% of the fastest count as tied and the one closest
to the kernel's defaults wins, so that noise does not flip the choice).
Every setting computes the same result (up to the float32 order of
gradient atomics), so tuning changes speed only.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional, Tuple

import torch

from . import gs

CHOICES = (1, 2, 4)
STAGES = (1, 2)
SCHEDULES = {"heaviest_first": gs.GS_SCHEDULE_HEAVIEST_FIRST, "tile_id": gs.GS_SCHEDULE_TILE_ID,
             "persistent": gs.GS_SCHEDULE_PERSISTENT,
             "persistent_half": gs.GS_SCHEDULE_PERSISTENT_HALF}
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gsmi", "tune.json")


def _key(step) -> str:
    name = torch.cuda.get_device_name(step.g.means.device)
    sizes = ",".join(f"{w}x{h}" for w, h in step.views.sizes)
    return f"{name}|{gs.version()}|n={step.n}|deg={step.g.sh_degree}|views={sizes}"


def _load(path: str) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(path: str, data: Dict):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply(fwd_ppl: int, bwd_ppl: int, fwd_schedule: int = 0, bwd_schedule: int = 0,
          fwd_stage: int = 0, bwd_stage: int = 0):
    """Sets the process-wide tuning (0 = the library default)."""
    gs.gs_set_tuning(gs.GS_TUNE_FWD_PIXELS_PER_LANE, fwd_ppl)
    gs.gs_set_tuning(gs.GS_TUNE_BWD_PIXELS_PER_LANE, bwd_ppl)
    gs.gs_set_tuning(gs.GS_TUNE_FWD_SCHEDULE, fwd_schedule)
    gs.gs_set_tuning(gs.GS_TUNE_BWD_SCHEDULE, bwd_schedule)
    gs.gs_set_tuning(gs.GS_TUNE_FWD_STAGE, fwd_stage)
    gs.gs_set_tuning(gs.GS_TUNE_BWD_STAGE, bwd_stage)


def time_config(step, fwd_ppl: int, bwd_ppl: int, reps: int = 3, fwd_schedule: int = 0,
                bwd_schedule: int = 0, fwd_stage: int = 0,
                bwd_stage: int = 0) -> Tuple[float, float]:
    """Mean (forward, backward) tile-kernel milliseconds for one setting."""
    apply(fwd_ppl, bwd_ppl, fwd_schedule, bwd_schedule, fwd_stage, bwd_stage)
    ev = {}
    for k in (gs.GS_KERNEL_RENDER_FWD, gs.GS_KERNEL_RENDER_BWD):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        b.record()
        ev[k] = (a, b)
    torch.cuda.synchronize()
    for k, (a, b) in ev.items():
        gs.gs_set_kernel_events(k, a, b)
    snap = step.adam.snapshot()
    fw, bw = [], []
    try:
        step._body()                                   # warm-up of this variant
        for _ in range(reps):
            step._body()
            torch.cuda.synchronize()
            fw.append(ev[gs.GS_KERNEL_RENDER_FWD][0].elapsed_time(ev[gs.GS_KERNEL_RENDER_FWD][1]))
            bw.append(ev[gs.GS_KERNEL_RENDER_BWD][0].elapsed_time(ev[gs.GS_KERNEL_RENDER_BWD][1]))
    finally:
        for k in ev:
            gs.gs_set_kernel_events(k, None, None)
        step.adam.restore(snap)
        torch.cuda.synchronize()
    return sum(fw) / len(fw), sum(bw) / len(bw)


def _apply_best(best: Dict):
    apply(best["fwd_ppl"], best["bwd_ppl"], best.get("fwd_schedule", 0), best.get("bwd_schedule", 0),
          best.get("fwd_stage", 0), best.get("bwd_stage", 0))


def _label(kernel: str, ppl: int, stage: int, schedule: str) -> str:
    return f"{kernel}{ppl}s{stage}_{schedule}"


# Each kernel's own staging batch per pixels-per-lane setting (the library
# default for GS_TUNE_*_STAGE = 0).
DEFAULT_STAGE = {"fwd": {1: 1, 2: 2, 4: 1}, "bwd": {1: 1, 2: 2, 4: 2}}
TIE = 0.02   # settings within 2% of the fastest count as tied (run-to-run noise)


def _pick(settings, table, kernel: str):
    """The fastest setting; among those within TIE of it, the one that
    departs least from the kernel's defaults (its staging batch, heaviest
    first), so that run-to-run noise does not flip the choice."""
    best = min(table[_label(kernel, *c)] for c in settings)
    tied = [c for c in settings if table[_label(kernel, *c)] <= best * (1.0 + TIE)]
    return min(tied, key=lambda c: ((c[1] != DEFAULT_STAGE[kernel][c[0]]) +
                                    (c[2] != "heaviest_first"), table[_label(kernel, *c)]))


def tune(step, cache: Optional[str] = None, force: bool = False, reps: int = 3) -> Dict:
    """Pick and apply the fastest setting for ``step`` (a replay.BatchedStep).
    Returns {"fwd_ppl", "bwd_ppl", "fwd_stage", "bwd_stage", "fwd_schedule",
    "bwd_schedule" (GS_SCHEDULE_* values) and their names, "fwd_ms", "bwd_ms",
    "cached", "table"}; table keys are "<fwd|bwd><ppl>s<stage>_<schedule>"."""
    cache = cache or os.environ.get("GSMI_TUNE_CACHE", DEFAULT_CACHE)
    key = _key(step)
    data = _load(cache)
    if not force and key in data and "fwd_stage" in data[key]:
        best = data[key]
        _apply_best(best)
        return dict(best, cached=True)
    settings = [(p, st, name) for name in SCHEDULES for p in CHOICES for st in STAGES]
    table = {}
    for p, st, name in settings:
        table[_label("fwd", p, st, name)], _ = time_config(
            step, p, 1, reps, fwd_schedule=SCHEDULES[name], fwd_stage=st)
        _, table[_label("bwd", p, st, name)] = time_config(
            step, 1, p, reps, bwd_schedule=SCHEDULES[name], bwd_stage=st)
    bf = _pick(settings, table, "fwd")
    bb = _pick(settings, table, "bwd")
    best = {"fwd_ppl": bf[0], "bwd_ppl": bb[0], "fwd_stage": bf[1], "bwd_stage": bb[1],
            "fwd_schedule": SCHEDULES[bf[2]], "bwd_schedule": SCHEDULES[bb[2]],
            "fwd_schedule_name": bf[2], "bwd_schedule_name": bb[2],
            "fwd_ms": table[_label("fwd", *bf)], "bwd_ms": table[_label("bwd", *bb)],
            "table": table}
    data[key] = best
    try:
        _save(cache, data)
    except OSError:
        pass
    _apply_best(best)
    return dict(best, cached=False)
