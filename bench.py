"""Benchmark: fwd+bwd mapping throughput of the batched rasterizer (Mpix/s).

One step = one mapping iteration over a batch of keyframe views: projection
of every Gaussian into every view, tile binning and sort, compositing, L1
photometric gradient, reverse tile walk, projection backward with pose
tangents, and an Adam update of every parameter group.  The batched step is
one HIP-graph launch; the plain reference runs the same kernels one view at a
time with a key-count readback per view.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload room32]

Prints one JSON line (rank 0).  Inputs are seeded synthetic procedural rooms
resident in device memory before timing starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (builder kwargs, description)
    "room32": dict(kind="metric", n=200000, views=32),
    "room12": dict(kind="metric", n=200000, views=12),
    "room_uneven32": dict(kind="c4", n=500000, views=32),
    "room1": dict(kind="metric", n=200000, views=1),
}

HBM_PEAK_GBS = 8000.0
# VALU issue rate: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (non-packed FP32
# lane-operations per second).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="room32", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-steps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--retune", action="store_true", help="ignore the tuning cache")
    return ap.parse_args()


def _build(spec, seed):
    from paper_2409_09295_amd import scenes
    if spec["kind"] == "c4":
        return scenes.config_c4(seed, n=spec["n"], n_views=spec["views"])
    return scenes.config_metric(seed, n=spec["n"], n_views=spec["views"])


def _cpu_baseline(wl, sample_tiles=400, seed=0):
    """The FP64 oracle on a bounded sample: projection (all Gaussians) and
    compositing forward + backward of ``sample_tiles`` random 16x16 tiles of
    view 0.  Returns (Mpix/s, pixels, seconds, threads)."""
    import numpy as np
    import torch
    from oracle import gs_oracle as O
    cam = wl.cams[0].as_float32()
    TX, TY = O.tile_grid(cam, 16)
    rng = np.random.default_rng(seed)
    flat = rng.choice(TX * TY, size=min(sample_tiles, TX * TY), replace=False)
    picks = [(int(t // TX), int(t % TX)) for t in flat]
    px = sum(min(16, cam.height - 16 * ty) * min(16, cam.width - 16 * tx) for ty, tx in picks)
    dl = np.zeros((3, cam.height, cam.width))
    for ty, tx in picks:
        dl[:, 16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = rng.normal(size=(3, 16, 16))[
            :, :min(16, cam.height - 16 * ty), :min(16, cam.width - 16 * tx)]
    t0 = time.perf_counter()
    O.render(wl.gmap, [cam], dL_dimage=[dl], with_mask=False, tiles=[picks])
    dt = time.perf_counter() - t0
    return px / dt / 1e6, px, dt, torch.get_num_threads()


def main():
    args = _args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2409_09295_amd import gs
    from paper_2409_09295_amd import autotune
    from paper_2409_09295_amd.replay import BatchedStep, PlainStep

    dev = "cuda"
    spec = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    wl = _build(spec, args.seed)
    print(f"[bench] workload {wl.name}: {wl.gmap.n} Gaussians, {len(wl.cams)} views "
          f"(built in {time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)
    g = gs.Gaussians.from_map(wl.gmap, dev)
    views = gs.Views(wl.cams, dev)
    targets = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).to(dev)
    P = views.n_pixels

    # ---------------- batched (headline) ----------------
    step = BatchedStep(g, views, targets)
    tuned = autotune.tune(step, force=args.retune)
    print(f"[bench] tuned: {tuned}", file=sys.stderr, flush=True)
    step.capture()
    for _ in range(args.warmup):
        step.step()
    torch.cuda.synchronize()
    if step.overflowed():
        raise RuntimeError("key capacity overflow during warm-up")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step.step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_batched = e0.elapsed_time(e1) / args.steps
    if step.overflowed():
        raise RuntimeError("key capacity overflow during timing")
    n_keys = step.key_count()
    print(f"[bench] batched: {ms_batched:.3f} ms/step ({wall / args.steps * 1e3:.3f} ms wall), "
          f"{n_keys} keys", file=sys.stderr, flush=True)

    # ---------------- per-kernel durations (HIP events on the launch stream) ---------
    names = {gs.GS_KERNEL_PREPROCESS: "preprocess", gs.GS_KERNEL_BIN_SORT: "bin_sort",
             gs.GS_KERNEL_RENDER_FWD: "render_fwd", gs.GS_KERNEL_RENDER_BWD: "render_bwd",
             gs.GS_KERNEL_PROJECT_BWD: "project_bwd"}
    ev = {k: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for k in names}
    for k, (a, b) in ev.items():
        a.record()          # torch creates the HIP event on first record
        b.record()
    torch.cuda.synchronize()
    for k, (a, b) in ev.items():
        gs.gs_set_kernel_events(k, a, b)
    kt = {k: [] for k in names}
    snap = step.adam.snapshot()
    for _ in range(args.kernel_steps):
        step._body()
        torch.cuda.synchronize()
        for k, (a, b) in ev.items():
            kt[k].append(a.elapsed_time(b))
    step.adam.restore(snap)
    for k in names:
        gs.gs_set_kernel_events(k, None, None)
    kms = {names[k]: float(np.mean(v)) for k, v in kt.items()}
    print(f"[bench] kernel ms: {kms}", file=sys.stderr, flush=True)

    # algorithmic work of the reverse tile walk: list positions each pixel walks
    pairs_bwd = int(step.n_contrib.to(torch.int64).sum().item())

    # ---------------- plain per-view reference ----------------
    ms_plain = None
    if not args.no_plain:
        tv = views.split_images(targets)
        plain = PlainStep(g, wl.cams, tv)
        snap = plain.adam.snapshot()
        plain.step()
        torch.cuda.synchronize()
        p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0.record()
        for _ in range(args.plain_steps):
            plain.step()
        p1.record()
        torch.cuda.synchronize()
        ms_plain = p0.elapsed_time(p1) / args.plain_steps
        plain.adam.restore(snap)
        print(f"[bench] plain: {ms_plain:.3f} ms/step", file=sys.stderr, flush=True)

    mpix = P / (ms_batched * 1e-3) / 1e6
    mpix_plain = P / (ms_plain * 1e-3) / 1e6 if ms_plain else None

    # ---------------- roofline of the dominant kernel ----------------
    dom = max(kms, key=kms.get)
    ops_per_pair_bwd = float(os.environ.get("GSMI_BWD_VALU_PER_PAIR", "48"))
    if dom == "render_bwd":
        achieved = pairs_bwd * ops_per_pair_bwd * 64 / 64 / (kms[dom] * 1e-3) / 1e12
        roof = {"kernel": "render_bwd", "bound": "alu", "achieved": achieved,
                "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
                "traffic": None, "units": pairs_bwd, "per_unit": ops_per_pair_bwd,
                "kernel_ms": kms[dom]}
    elif dom == "render_fwd":
        achieved = pairs_bwd * 20.0 / (kms[dom] * 1e-3) / 1e12
        roof = {"kernel": "render_fwd", "bound": "alu", "achieved": achieved,
                "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
                "traffic": None, "units": pairs_bwd, "per_unit": 20.0, "kernel_ms": kms[dom]}
    else:
        K = (wl.gmap.sh_degree + 1) ** 2
        per_gauss = 4 * (3 + 3 + 4 + 1 + 3 * K)
        nbytes = g.n * (2 * per_gauss) + g.n * len(wl.cams) * (9 * 4 + 4 * 4)
        achieved = nbytes / (kms[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel_ms": kms[dom]}

    # ---------------- CPU oracle baseline ----------------
    cpu = None
    if not args.no_cpu_baseline:
        mp, px, dt, thr = _cpu_baseline(wl)
        cpu = {"value": mp, "unit": "Mpix/s", "cores": thr, "kind": "oracle",
               "sample": f"fwd+bwd of {px} px (400 random 16x16 tiles of view 0) incl. projection "
                         f"and its backward for all {wl.gmap.n} Gaussians; {dt:.1f} s"}
        print(f"[bench] cpu oracle: {mp:.5f} Mpix/s over {dt:.1f}s", file=sys.stderr, flush=True)

    out = {
        "metric": "fwd+bwd Mpix/s at 640x480, 200k Gaussians; batched vs plain, same accuracy",
        "value": mpix, "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_batched, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "gaussians": wl.gmap.n, "views": len(wl.cams),
                   "image_sizes": sorted(set(views.sizes)), "pixels_per_step": P,
                   "sh_degree": wl.gmap.sh_degree, "step": "fwd+bwd+adam, one HIP graph",
                   "keys": n_keys, "parallelism": "single GPU"},
        "plain": {"value": mpix_plain, "ms_per_step": ms_plain,
                  "speedup_batched_over_plain": (mpix / mpix_plain) if mpix_plain else None},
        "kernel_ms": kms,
        "tuning": {"fwd_pixels_per_lane": tuned["fwd_ppl"], "bwd_pixels_per_lane": tuned["bwd_ppl"],
                   "table_ms": tuned.get("table")},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
