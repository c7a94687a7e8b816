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
import gc
import json
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
# VALU peak: the published FP32 vector rate, 157.3 TFLOP/s, counts an FMA as
# two operations: 256 CUs x 128 lanes x 2.4 GHz = 78.6 T lane-operations per
# second, i.e. two wave64 instructions per CU per cycle.  Measured on the
# MI355X, independent chains of v_mul/v_add/v_sub/v_fmac with VGPR (or inline
# constant) operands issue at 1.8-1.9 per CU-cycle; compares, min/max/med3,
# DPP, shifts, conversions and any instruction with an SGPR source issue at
# half that, v_exp/v_rcp at a quarter.
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12

# VALU instructions per (pixel, splat) pair in the per-pixel body of the
# compositing loops, counted in the gfx950 assembly of this library: every
# walked pair pays the evaluation (offsets, quadratic form -- its x terms
# shared by a lane's two pixels in one column --, clamp, exp2, opacity
# product, alpha clamp and the tests; the forward adds the transmittance
# product, its test and the termination mark); a pair that is blended pays
# the rest.
# Wave-level overheads (LDS staging, the 9-value reduction and its atomics,
# loop control) are not counted: they are what separates the achieved rate
# from the peak.
BWD_VALU_EVAL, BWD_VALU_BLEND = 12, 26
FWD_VALU_EVAL, FWD_VALU_BLEND = 15, 4
# Fraction of walked pairs that are blended, measured by the oracle on the
# 200k-Gaussian room at 640x480 (used when the oracle leg is skipped).
DEFAULT_BLEND_FRACTION = 0.44

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_bwd_room32_traffic.txt")
TRAFFIC_SOURCES = ("paper_2409_09295_amd/csrc/render_bwd.hip", "paper_2409_09295_amd/csrc/gs_internal.h")


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
    ap.add_argument("--no-v12", action="store_true", help="skip the 12-view (8 window + 4 past) line")
    ap.add_argument("--no-initialiser", action="store_true",
                    help="skip the initialisers' timing (cost volume, belief propagation, U-Net)")
    ap.add_argument("--no-mapping", action="store_true",
                    help="skip the mapping-loop overhead-memory measurement")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a float32 copy of this size first (scales HBM counters)")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the step eagerly instead of replaying a HIP graph (profiling)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate length of the CPU oracle sample")
    return ap.parse_args()


def _build(spec, seed):
    from paper_2409_09295_amd import scenes
    if spec["kind"] == "c4":
        return scenes.config_c4(seed, n=spec["n"], n_views=spec["views"])
    return scenes.config_metric(seed, n=spec["n"], n_views=spec["views"])


def _cpu_baseline(wl, budget_s=15.0, max_views=32, seed=0):
    """The FP64 oracle, as it stands, on a bounded sample of the same step:
    projection of all Gaussians, compositing of every pixel and the full
    backward (pixels -> 2D -> 3D parameters and pose) of whole views, taken
    in trajectory order until about ``budget_s`` seconds have passed.
    Returns (Mpix/s, views, pixels, seconds, threads, blended fraction)."""
    import numpy as np
    import torch
    from oracle import gs_oracle as O
    rng = np.random.default_rng(seed)
    px, dt, walked, blended, nv = 0, 0.0, 0, 0, 0
    while nv < min(max_views, len(wl.cams)) and dt < budget_s:
        cam = wl.cams[nv].as_float32()
        dl = rng.normal(size=(3, cam.height, cam.width))
        t0 = time.perf_counter()
        r = O.render(wl.gmap, [cam], dL_dimage=[dl], with_mask=False)
        dt += time.perf_counter() - t0
        v = r["views"][0]
        walked += int(v["n_contrib"].sum())
        blended += int(v["n_blended"].sum())
        px += cam.width * cam.height
        nv += 1
    return px / dt / 1e6, nv, px, dt, torch.get_num_threads(), blended / max(walked, 1)


def _cpu_one_thread(wl, seed=0):
    """The same oracle work on one thread: fwd+bwd of the first view."""
    import numpy as np
    import torch
    from oracle import gs_oracle as O
    rng = np.random.default_rng(seed)
    cam = wl.cams[0].as_float32()
    dl = rng.normal(size=(3, cam.height, cam.width))
    prev = torch.get_num_threads()
    torch.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        O.render(wl.gmap, [cam], dL_dimage=[dl], with_mask=False)
        dt = time.perf_counter() - t0
    finally:
        torch.set_num_threads(prev)
    return cam.width * cam.height / dt / 1e6, dt


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _traffic(variant: str):
    """HBM bytes per launch of the reverse tile walk from the committed
    counter summary, or None when the kernel's sources changed since or the
    summary was taken on another tuned variant of it."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != h.hexdigest() or vals.get("kernel_variant") != variant:
        return None
    try:
        return float(vals["fetch_bytes"]) + float(vals["write_bytes"])
    except (KeyError, ValueError):
        return None


def _bwd_variant(tuned) -> str:
    """The tuned backward tile kernel, as the traffic summary names it."""
    return (f"ppl={tuned['bwd_ppl']} stage={tuned.get('bwd_stage')} "
            f"schedule={tuned.get('bwd_schedule_name')}")


def _time_batched(step, steps, warmup):
    import torch
    if step.use_graph:
        step.capture()
    for _ in range(warmup):
        step.step()
    torch.cuda.synchronize()
    if step.overflowed():
        raise RuntimeError("key capacity overflow during warm-up")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        step.step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    if step.overflowed():
        raise RuntimeError("key capacity overflow during timing")
    return e0.elapsed_time(e1) / steps, wall / steps * 1e3


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

    if args.copy_probe_mib:
        # a plain elementwise copy of known size: reads and writes n bytes
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.rand(n, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b

    # ---------------- batched (headline) ----------------
    step = BatchedStep(g, views, targets, use_graph=not args.no_graph)
    tuned = autotune.tune(step, force=args.retune)
    print(f"[bench] tuned: {tuned}", file=sys.stderr, flush=True)
    ms_batched, wall_ms = _time_batched(step, args.steps, args.warmup)
    n_keys = step.key_count()
    print(f"[bench] batched: {ms_batched:.3f} ms/step ({wall_ms:.3f} ms wall), "
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

    # ---------------- selective optimisation: E_k(g), the active set ---------------
    selective = None
    try:
        err = torch.empty(len(wl.cams), g.n, device=dev)
        gs.gs_render_error(step.proj, g.n, step.bins, views, step.image, targets, step.n_contrib, err)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.kernel_steps):
            gs.gs_render_error(step.proj, g.n, step.bins, views, step.image, targets, step.n_contrib,
                               err)
        e1.record()
        torch.cuda.synchronize()
        emax = err.max(dim=0).values
        eps = float(torch.quantile(emax[emax > 0].float(), 0.85)) if bool((emax > 0).any()) else 0.0
        mask = torch.zeros(g.n, dtype=torch.uint8, device=dev)
        n_act = torch.zeros(1, dtype=torch.int32, device=dev)
        gs.gs_active_set(err, g.n, len(wl.cams), eps, mask, n_active=n_act)
        selective = {"render_error_ms": e0.elapsed_time(e1) / args.kernel_steps,
                     "eps_rule": "0.85 quantile of the non-zero max_k E_k(g)", "eps": eps,
                     "active_fraction": int(n_act.item()) / g.n}
        del err, mask
    except Exception as exc:   # reported, never fatal to the headline line
        selective = {"error": repr(exc)}

    # ---------------- initialisers (Sec. III-A): the last of 8 rendered views ------------
    init_ms = None
    if not args.no_initialiser:
        try:
            from paper_2409_09295_amd import initnet
            imgs = views.split_images(step.image)[:8]
            kf = torch.stack([im.view(3, *im.shape[-2:]) for im in imgs]).clamp(0.0, 1.0).contiguous()
            cams8 = wl.cams[:8]

            def timed_ms(fn, reps=5):
                fn()
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    fn()
                b.record()
                torch.cuda.synchronize()
                return a.elapsed_time(b) / reps

            net = initnet.UNet(seed=args.seed)
            one = kf[-1:].contiguous()
            init_ms = {"keyframes": 8, "resolution": list(kf.shape[-1:-3:-1]),
                       "cost_volume_wta": timed_ms(lambda: initnet.plain_depth(kf, cams8)),
                       "cost_volume_bp": timed_ms(lambda: initnet.plain_depth(kf, cams8, method="bp")),
                       "unet_forward": timed_ms(lambda: net.forward(one))}
            del net, kf, one
        except Exception as exc:   # reported, never fatal to the headline line
            init_ms = {"error": repr(exc)}

    # algorithmic work of the reverse tile walk: list positions each pixel walks
    pairs_bwd = int(step.n_contrib.to(torch.int64).sum().item())
    n_visible = int((step.proj.radius > 0).sum().item())
    n_binned = int((step.proj.tiles != 0).sum().item())   # visible splats that touch a tile
    del step
    gc.collect()
    torch.cuda.empty_cache()

    # ---------------- paper-shaped batch: 8 window + 4 past views ----------------
    v12 = None
    if not args.no_v12 and len(wl.cams) > 12:
        views12 = gs.Views(wl.cams[:12], dev)
        t12 = targets[:3 * views12.n_pixels]
        step12 = BatchedStep(g, views12, t12, use_graph=not args.no_graph)
        ms12, _ = _time_batched(step12, args.steps, args.warmup)
        v12 = {"views": 12, "ms_per_step": ms12,
               "value": views12.n_pixels / (ms12 * 1e-3) / 1e6, "unit": "Mpix/s"}
        print(f"[bench] 12 views: {ms12:.3f} ms/step", file=sys.stderr, flush=True)
        del step12
        gc.collect()
        torch.cuda.empty_cache()

    # ---------------- overhead memory of the mapping loop (Sec. IV-B) ----------------
    memory = None
    if not args.no_mapping:
        try:
            from paper_2409_09295_amd.mapping import run_sequence
            t1 = time.perf_counter()
            ms = run_sequence(640, 480, 12, 8, n_gauss=200000, seed=args.seed, n_past=4)
            memory = {"frames": 12, "window": 8, "past_views": 4, "resolution": [640, 480],
                      "overhead_peak_MB": ms["overhead_peak_MB"],
                      "peak_by_category_MB": ms["peak_by_category_MB"],
                      "all_keyframes_MB": ms["all_keyframes_MB"], "map_MB": ms["map_MB"],
                      "psnr_mean_dB": ms["psnr_mean"], "seconds": time.perf_counter() - t1}
            print(f"[bench] mapping loop: overhead {ms['overhead_peak_MB']:.1f} MB",
                  file=sys.stderr, flush=True)
        except Exception as exc:
            memory = {"error": repr(exc)}
        gc.collect()
        torch.cuda.empty_cache()

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

    # ---------------- CPU oracle baseline ----------------
    cpu, blend_frac = None, DEFAULT_BLEND_FRACTION
    if not args.no_cpu_baseline:
        mp, nv, px, dt, thr, blend_frac = _cpu_baseline(wl, args.cpu_seconds)
        mp1, dt1 = _cpu_one_thread(wl)
        cpu = {"value": mp, "unit": "Mpix/s", "cores": thr, "kind": "oracle",
               "sample": f"fwd+bwd of {nv} whole {wl.cams[0].width}x{wl.cams[0].height} views "
                         f"({px} px; projection, compositing and backward of all {wl.gmap.n} "
                         f"Gaussians per view) in {dt:.1f} s",
               "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
               "one_thread": {"value": mp1, "unit": "Mpix/s", "cores": 1,
                              "sample": f"fwd+bwd of the first view in {dt1:.1f} s"}}
        print(f"[bench] cpu oracle: {mp:.5f} Mpix/s over {dt:.1f}s; blended fraction "
              f"{blend_frac:.3f}", file=sys.stderr, flush=True)

    # ---------------- roofline of the dominant kernel ----------------
    dom = max(kms, key=kms.get)
    bwd_per_pair = BWD_VALU_EVAL + BWD_VALU_BLEND * blend_frac
    fwd_per_pair = FWD_VALU_EVAL + FWD_VALU_BLEND * blend_frac
    if dom in ("render_bwd", "render_fwd"):
        per = bwd_per_pair if dom == "render_bwd" else fwd_per_pair
        achieved = pairs_bwd * per / (kms[dom] * 1e-3) / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                "unit": "T VALU lane-ops/s", "frac": achieved / VALU_PEAK_TOPS,
                "traffic": _traffic(_bwd_variant(tuned)) if dom == "render_bwd" else None,
                "units": pairs_bwd, "unit_name": "walked (pixel, splat) pairs",
                "per_unit": per, "blend_fraction": blend_frac, "kernel_ms": kms[dom]}
    else:
        K = (wl.gmap.sh_degree + 1) ** 2
        per_gauss = 4 * (3 + 3 + 4 + 1 + 3 * K)
        nbytes = g.n * per_gauss + g.n * len(wl.cams) * (2 + 4 + 4 + 1) * 4
        achieved = nbytes / (kms[dom] * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel_ms": kms[dom]}

    # HBM-bound stages: algorithmic bytes per launch / event-timed duration
    K = (wl.gmap.sh_degree + 1) ** 2
    # preprocess: the map once, a 48-byte splat (with its tile count) per
    # visible (Gaussian, view), a radius and a zero count per culled one
    pre_bytes = (g.n * 4 * (3 + 3 + 4 + 1 + 3 * K) + n_visible * (8 + 16 + 16 + 4 + 4)
                 + (g.n * len(wl.cams) - n_visible) * 8)
    # binning (the step bins without keys): the tile count of every entry
    # (4 B), the centre, radius and depth of every binned splat (one that
    # touches a tile: 16 B), per key its (depth, entry) pair staged in its
    # tile's segment and read back by the segment sort (16 B) and its value
    # (4 B), per tile its range (8 B) and launch-order slot (4 B)
    sort_bytes = (g.n * len(wl.cams) * 4 + n_binned * 16 + n_keys * (16 + 4)
                  + views.n_tiles * 12)
    # gradient projection: the map once (read) and its gradients once
    # (written), every entry's radius, and per visible entry its 36-byte
    # screen-space gradient record read and cleared
    proj_bytes = (g.n * 4 * (3 + 3 + 4 + 1 + 3 * K) * 2 + g.n * len(wl.cams) * 4
                  + n_visible * 36 * 2)
    hbm = {name: {"bytes": b, "ms": kms[name], "GB/s": b / (kms[name] * 1e-3) / 1e9,
                  "frac": b / (kms[name] * 1e-3) / 1e9 / HBM_PEAK_GBS}
           for name, b in (("preprocess", pre_bytes), ("bin_sort", sort_bytes),
                           ("project_bwd", proj_bytes))}

    out = {
        "metric": "fwd+bwd Mpix/s at 640x480, 200k Gaussians; batched vs plain, same accuracy",
        "value": mpix, "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_batched, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "gaussians": wl.gmap.n, "views": len(wl.cams),
                   "image_sizes": sorted(set(views.sizes)), "pixels_per_step": P,
                   "sh_degree": wl.gmap.sh_degree,
                   "step": "fwd+bwd+adam, " + ("eager launches" if args.no_graph else "one HIP graph"),
                   "keys": n_keys, "parallelism": "single GPU"},
        "plain": {"value": mpix_plain, "ms_per_step": ms_plain,
                  "speedup_batched_over_plain": (mpix / mpix_plain) if mpix_plain else None},
        "paper_shaped_12_views": v12,
        "kernel_ms": kms,
        "tuning": {"fwd_pixels_per_lane": tuned["fwd_ppl"], "bwd_pixels_per_lane": tuned["bwd_ppl"],
                   "fwd_stage_per_thread": tuned.get("fwd_stage"),
                   "bwd_stage_per_thread": tuned.get("bwd_stage"),
                   "fwd_schedule": tuned.get("fwd_schedule_name"),
                   "bwd_schedule": tuned.get("bwd_schedule_name"),
                   "table_ms": tuned.get("table")},
        "roofline": roof,
        "hbm_kernels": hbm,
        "selective": selective,
        "initialiser_ms": init_ms,
        "mapping_memory": memory,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
