"""Autotuner for the compositing kernels' launch shape.

For a given batch (device, views, pixel count, Gaussian count, SH degree) it
times every pixels-per-lane setting of the forward and backward tile kernels
on the real step (eager launches, HIP events, optimiser state restored
afterwards), keeps the fastest and caches the choice in a JSON file keyed by
device name, library version and workload shape.  Every setting computes the
same result (up to the float32 order of gradient atomics), so tuning changes
speed only.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional, Tuple

import torch

from . import gs

CHOICES = (1, 2, 4)
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


def apply(fwd_ppl: int, bwd_ppl: int):
    gs.gs_set_tuning(gs.GS_TUNE_FWD_PIXELS_PER_LANE, fwd_ppl)
    gs.gs_set_tuning(gs.GS_TUNE_BWD_PIXELS_PER_LANE, bwd_ppl)


def time_config(step, fwd_ppl: int, bwd_ppl: int, reps: int = 3) -> Tuple[float, float]:
    """Mean (forward, backward) tile-kernel milliseconds for one setting."""
    apply(fwd_ppl, bwd_ppl)
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


def tune(step, cache: Optional[str] = None, force: bool = False, reps: int = 3) -> Dict:
    """Pick and apply the fastest setting for ``step`` (a replay.BatchedStep).
    Returns {"fwd_ppl", "bwd_ppl", "fwd_ms", "bwd_ms", "cached", "table"}."""
    cache = cache or os.environ.get("GSMI_TUNE_CACHE", DEFAULT_CACHE)
    key = _key(step)
    data = _load(cache)
    if not force and key in data:
        best = data[key]
        apply(best["fwd_ppl"], best["bwd_ppl"])
        return dict(best, cached=True)
    table = {}
    for f in CHOICES:
        table[f"fwd{f}"], _ = time_config(step, f, 1, reps)
    for b in CHOICES:
        _, table[f"bwd{b}"] = time_config(step, 1, b, reps)
    bf = min(CHOICES, key=lambda f: table[f"fwd{f}"])
    bb = min(CHOICES, key=lambda b: table[f"bwd{b}"])
    best = {"fwd_ppl": bf, "bwd_ppl": bb, "fwd_ms": table[f"fwd{bf}"], "bwd_ms": table[f"bwd{bb}"],
            "table": table}
    data[key] = best
    try:
        _save(cache, data)
    except OSError:
        pass
    apply(bf, bb)
    return dict(best, cached=False)
