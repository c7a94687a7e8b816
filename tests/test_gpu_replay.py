"""Batched replay (one graph launch over many views) vs the eager and the
per-view paths, and the batched launch at the benchmark's full sizes vs the
FP64 oracle on sampled tiles (needs an MI355X)."""
import time

import numpy as np
import pytest
import torch

from oracle import gs_oracle as O
from paper_2409_09295_amd import scenes
from tests.gpu_helpers import (assert_grad_close, assert_same_up_to_order, f32, np_, term_mass,
                               random_dl)

pytestmark = pytest.mark.gpu
DEV = "cuda"
GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _log(msg):
    print(msg, flush=True)


def _snap(step):
    return (step.image.clone(), {k: getattr(step.grads, k).clone() for k in GROUPS + ("xi",)})


def _small_uneven(seed=0):
    """A 30k-Gaussian room seen by 5 keyframes of four different sizes."""
    return scenes.config_c4(seed, n=30000, n_views=5)


def test_graph_replay_matches_eager_and_plain(gs):
    from paper_2409_09295_amd.replay import BatchedStep, PlainStep
    wl = _small_uneven()
    g = gs.Gaussians.from_map(wl.gmap)
    views = gs.Views(wl.cams)
    targets = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).to(DEV)
    step = BatchedStep(g, views, targets, optimize=False)
    step._body()
    torch.cuda.synchronize()
    img0, gr0 = _snap(step)
    step.capture()
    for rep in range(3):
        step.step()
        torch.cuda.synchronize()
        img, gr = _snap(step)
        _log(f"replay {rep}: checking against the eager step")
        torch.testing.assert_close(img, img0, rtol=0, atol=0)       # same kernels, same order
        for k in GROUPS + ("xi",):
            assert_same_up_to_order(k, np_(gr[k]), np_(gr0[k]))
        # eager work of the program between replays
        _ = (targets * 2).sum().item()
    # per-view reference path: same images bit for bit, same summed gradients
    plain = PlainStep(g, wl.cams, views.split_images(targets), optimize=False)
    plain.step()
    torch.cuda.synchronize()
    for v, im in enumerate(views.split_images(img0)):
        torch.testing.assert_close(plain.rasts[v].image.view_as(im), im, rtol=0, atol=0)
    for k in GROUPS:
        assert_same_up_to_order(k, np_(getattr(plain.grads, k)), np_(gr0[k]))
    assert_same_up_to_order("xi", np_(plain.xi), np_(gr0["xi"]))


def test_graph_replay_with_adam_tracks_eager(gs):
    """Three optimisation steps replayed from the graph land where three
    eager steps do (Adam's step counter lives on the device).  Gradients
    differ in the float32 order of their atomics, and Adam's first steps move
    every parameter with a nonzero gradient by about lr whatever its size, so
    a parameter whose gradient is pure cancellation noise may move either
    way: such parameters are rare, and no parameter differs by more than the
    three steps could move it."""
    from paper_2409_09295_amd.replay import DEFAULT_LR, BatchedStep
    wl = _small_uneven(1)
    targets = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).to(DEV)
    runs, counters = {}, {}
    for mode in ("eager", "graph"):
        g = gs.Gaussians.from_map(wl.gmap)
        step = BatchedStep(g, gs.Views(wl.cams), targets, use_graph=(mode == "graph"))
        for _ in range(3):
            step.step()
            torch.cuda.synchronize()
        runs[mode] = {k: getattr(g, k).clone() for k in GROUPS}
        counters[mode] = int(step.adam.step_dev.item())
    assert counters == {"eager": 3, "graph": 3}
    for k in GROUPS:
        a, b = np_(runs["graph"][k]), np_(runs["eager"][k])
        d = np.abs(a - b)
        assert d.max() <= 3 * 2 * DEFAULT_LR[k] * 1.001, (k, d.max())
        off = d > 1e-5 * np.abs(b).max() + 1e-7
        assert off.mean() < 5e-3, (k, off.mean())


@pytest.mark.parametrize("ppl", [1, 4])
def test_persistent_schedule_matches_per_tile_launch(gs, ppl):
    """The benchmark's batch (38,400 tiles): persistent workgroups drawing
    tiles from the bins' counters give the image and n_contrib of one
    workgroup per tile bit for bit, and its gradients up to the order of the
    atomic additions, eagerly and over three graph replays with eager work
    between them (each launch leaves its counter at zero for the next)."""
    from paper_2409_09295_amd import autotune
    from paper_2409_09295_amd.replay import BatchedStep
    wl = scenes.config_metric(0)
    views = gs.Views(wl.cams)
    rng = np.random.default_rng(12)
    targets = torch.from_numpy(rng.random(3 * views.n_pixels).astype(np.float32)).to(DEV)
    step = BatchedStep(gs.Gaussians.from_map(wl.gmap), views, targets, optimize=False)
    try:
        autotune.apply(ppl, ppl, gs.GS_SCHEDULE_HEAVIEST_FIRST, gs.GS_SCHEDULE_HEAVIEST_FIRST)
        step._body()
        torch.cuda.synchronize()
        img0, gr0 = _snap(step)
        nc0 = step.n_contrib.clone()
        autotune.apply(ppl, ppl, gs.GS_SCHEDULE_PERSISTENT, gs.GS_SCHEDULE_PERSISTENT)

        def check(label):
            torch.cuda.synchronize()
            img, gr = _snap(step)
            _log(f"ppl {ppl} persistent, {label}: checking against one workgroup per tile")
            torch.testing.assert_close(img, img0, rtol=0, atol=0)
            torch.testing.assert_close(step.n_contrib, nc0, rtol=0, atol=0)
            for k in GROUPS + ("xi",):
                assert_same_up_to_order(k, np_(gr[k]), np_(gr0[k]))
            assert int(step.bins.queue.abs().sum().item()) == 0

        step._body()
        check("eager")
        step.capture()
        for rep in range(3):
            step.step()
            check(f"replay {rep}")
            _ = (targets * 2).sum().item()
    finally:
        autotune.apply(0, 0)


def _pick_tiles(cams, tiles_per_view, seed):
    rng = np.random.default_rng(seed)
    picks = []
    for c in cams:
        TX, TY = O.tile_grid(c, 16)
        p = {(int(rng.integers(0, TY)), int(rng.integers(0, TX))) for _ in range(tiles_per_view)}
        p |= {(0, 0), (TY - 1, TX - 1), (TY // 2, TX // 2)}
        picks.append(sorted(p))
    return picks


def _timed_step_parity(gs, wl, view_ids, tiles_per_view, seed, max_masked):
    """The benchmark's step itself, one replay of its HIP graph (projection
    of every view, binning with the device key count, compositing fused with
    the L1 gradient, reverse tile walk on a workspace kept clear, projection
    backward with pose tangents, grouped Adam), against the oracle on sampled
    tiles of ``view_ids``.

    The targets equal the step's own render everywhere except on the sampled
    tiles (minus their near-threshold pixels), where they are random: the L1
    gradient is then exactly zero elsewhere, and every gradient of the step
    comes from pixels the oracle composites.  Checked: images and n_contrib
    on the sampled tiles, dL/dC (zero elsewhere; the sign of the oracle's
    residual on the sampled pixels), the loss, every parameter group's and
    every pose's gradient, and the parameters after Adam (the oracle's Adam
    applied to the step's own gradients)."""
    from paper_2409_09295_amd import autotune
    from paper_2409_09295_amd.replay import BETA1, BETA2, DEFAULT_LR, EPS, BatchedStep
    g = gs.Gaussians.from_map(wl.gmap)
    views = gs.Views(wl.cams)
    P = views.n_pixels
    targets = torch.zeros(3 * P, dtype=torch.float32, device=DEV)
    step = BatchedStep(g, views, targets, bg=wl.bg)
    tuned = autotune.tune(step)
    _log(f"{wl.name}: tuned {tuned['fwd_ppl']}/{tuned['bwd_ppl']} "
         f"{tuned.get('fwd_schedule_name')}/{tuned.get('bwd_schedule_name')}")
    try:
        snap = step.adam.snapshot()
        step._body()
        torch.cuda.synchronize()
        step.adam.restore(snap)
        render = np_(step.image).copy()
        sub = [wl.cams[v].as_float32() for v in view_ids]
        picks = _pick_tiles(sub, tiles_per_view, seed)
        _log(f"{wl.name}: oracle forward on {sum(map(len, picks))} sampled tiles of views {view_ids}")
        res0 = O.render(wl.gmap, sub, bg=wl.bg, tiles=picks)
        tgt = render.copy()
        offs = views.pixel_offsets()
        rng = np.random.default_rng(seed + 1)
        keeps = []
        masked = 0
        for j, v in enumerate(view_ids):
            w, h = views.sizes[v]
            keep = np.zeros((h, w), bool)
            for ty, tx in picks[j]:
                keep[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = True
            masked += int((keep & res0["views"][j]["mask"]).sum())
            keep &= ~res0["views"][j]["mask"]
            blk = tgt[3 * offs[v]:3 * (offs[v] + w * h)].reshape(3, h, w)
            blk[:, keep] = rng.random((3, int(keep.sum())))
            keeps.append(keep)
        _log(f"{wl.name}: {masked} near-threshold px on the sampled tiles (bound {max_masked})")
        assert masked <= max_masked, masked
        targets.copy_(torch.from_numpy(tgt))
        params0 = [np_(t).copy() for t in g.tensors()]
        _log(f"{wl.name}: capture and one replay of the step, {len(wl.cams)} views")
        step.capture()
        step.step()
        torch.cuda.synchronize()
        assert not step.overflowed()
        assert int(step.adam.step_dev.item()) == 1
    finally:
        autotune.apply(0, 0)
    img = np_(step.image)
    dl = np_(step.dL)
    imgs = views.split_images(step.image)
    worst = 0.0
    sub_dl = []
    dl_zero = np.ones(3 * P, bool)
    loss_ref = 0.0
    for j, v in enumerate(view_ids):
        w, h = views.sizes[v]
        r = res0["views"][j]
        m = ~r["mask"] & np.isfinite(r["image"][0])
        d = np.abs(np_(imgs[v]) - r["image"])[:, m]
        worst = max(worst, float(d.max()))
        np.testing.assert_array_equal(np_(views.split_maps(step.n_contrib)[v])[m], r["n_contrib"][m])
        blk = dl[3 * offs[v]:3 * (offs[v] + w * h)].reshape(3, h, w)
        t = tgt[3 * offs[v]:3 * (offs[v] + w * h)].reshape(3, h, w)
        resid = r["image"][:, keeps[j]] - t[:, keeps[j]]
        expect = np.sign(resid) / (3.0 * w * h)
        clear = np.abs(resid) > 1e-4          # sign not decided by the 1e-4 image tolerance
        np.testing.assert_array_equal(blk[:, keeps[j]][clear], expect[clear].astype(np.float32))
        loss_ref += float(np.abs(resid).sum()) / (3.0 * w * h)
        sub_dl.append(blk.astype(np.float64))
        zb = dl_zero[3 * offs[v]:3 * (offs[v] + w * h)].reshape(3, h, w)
        zb[:, keeps[j]] = False
    _log(f"{wl.name}: image worst {worst:.3e}")
    assert worst <= 1e-4
    assert (dl[dl_zero] == 0.0).all(), "dL/dC nonzero where the target equals the render"
    n_changed = sum(int(k.sum()) for k in keeps)
    loss_tol = 1e-4 * 3 * n_changed / (3.0 * min(w * h for w, h in views.sizes))
    assert abs(float(step.loss.item()) - loss_ref) <= loss_tol, (float(step.loss.item()), loss_ref)
    _log(f"{wl.name}: oracle backward")
    res = O.render(wl.gmap, sub, bg=wl.bg, dL_dimage=sub_dl, tiles=picks)
    mass = term_mass(wl.gmap, sub, sub_dl, tiles=picks, bg=wl.bg)
    gr = step.grads
    for k in GROUPS:
        assert_grad_close(k, np_(getattr(gr, k)), res["grads"][k], mass_fn=mass)
    xi = np_(gr.xi)
    assert_grad_close("xi", xi[view_ids], res["grads"]["xi"])
    others = np.setdiff1d(np.arange(len(wl.cams)), view_ids)
    assert np.abs(xi[others]).max() == 0.0
    # Adam, as the step applied it: the oracle's update of the initial
    # parameters with the step's own gradients
    for k, p0, p1 in zip(GROUPS, params0, g.tensors()):
        ref_p, _, _ = O.adam_step(p0, np_(getattr(gr, k)), np.zeros_like(p0), np.zeros_like(p0),
                                  f32(DEFAULT_LR[k]), f32(BETA1), f32(BETA2), f32(EPS), 1)
        np.testing.assert_allclose(np_(p1), ref_p, rtol=2e-6, atol=1e-7, err_msg=k)


def test_timed_step_metric_workload(gs):
    """200k Gaussians, 32 views at 640x480: the benchmark's batch."""
    _timed_step_parity(gs, scenes.config_metric(0), [0, 17, 31], 6, seed=40, max_masked=10)


def test_timed_step_uneven_views(gs):
    """500k Gaussians, 32 keyframes of four sizes up to 1200x680."""
    _timed_step_parity(gs, scenes.config_c4(0), [0, 1, 2, 3], 4, seed=50, max_masked=10)


FULL_BIN_CASES = {
    # the benchmark's batch: 38,400 tiles (two 8-bit tile passes)
    "metric_32x640x480": lambda: scenes.config_metric(0),
    # 77,400 tiles: above 2^16, so the tile bits take three passes
    "wide_24x1200x680": lambda: scenes.room_views(200000, [(1200, 680)] * 24, 3, "room_24_1200x680"),
}


@pytest.mark.parametrize("case", list(FULL_BIN_CASES))
def test_bin_sort_full_size_bit_exact(gs, case):
    """Binning of the GPU's own projected splats at full size: keys, values,
    ranges and the tile order bit for bit against the oracle's integer
    binning of the same splats, with keys (synchronous) and without
    (capacity mode, as the step runs it)."""
    wl = FULL_BIN_CASES[case]()
    g = gs.Gaussians.from_map(wl.gmap)
    views = gs.Views(wl.cams)
    V, N = views.n_views, g.n
    proj = gs.Projected.empty(V, N)
    gs.gs_preprocess(g, views, proj)
    torch.cuda.synchronize()
    xy, rd, rad = np_(proj.xy), np_(proj.rgb_depth), np_(proj.radius)
    rad = np.where(rad > 0, rad, 0)
    _log(f"{case}: {views.n_tiles} tiles; oracle binning")
    keys, vals, ranges, _, _ = O.bin_splats([xy[v] for v in range(V)], [rd[v, :, 3] for v in range(V)],
                                            [rad[v] for v in range(V)], wl.cams, 16)
    _log(f"{case}: {len(keys)} keys")
    for with_keys, sync in ((True, True), (False, False)):
        bins = gs.Bins.empty(len(keys) + 1024, views.n_tiles, keys=with_keys)
        ws = gs.workspace(gs.gs_bin_sort_workspace_size(N, views, bins.capacity))
        gs.gs_bin_sort(proj, N, views, bins, ws, sync=sync)
        torch.cuda.synchronize()
        n = int(np_(bins.n_keys).view(np.uint32)[0])
        assert n == len(keys)
        if with_keys:
            np.testing.assert_array_equal(np_(bins.keys)[:n].view(np.uint64), keys)
        np.testing.assert_array_equal(np_(bins.values)[:n].view(np.uint32), vals)
        np.testing.assert_array_equal(np_(bins.ranges).view(np.uint32), ranges)
        ln = ranges[:, 1].astype(np.int64) - ranges[:, 0]
        lg = np.floor(np.log2(np.maximum(ln, 1))).astype(np.int64)
        half = np.where(lg > 0, (ln >> np.maximum(lg - 1, 0)) & 1, 0)
        grp = np.where(ln == 0, 0, np.minimum(31, 1 + 2 * lg + half))
        np.testing.assert_array_equal(np_(bins.order).view(np.uint32), np.argsort(-grp, kind="stable"))
        del bins, ws


def test_batched_at_least_3x_plain(gs):
    """The metric: one graph launch over 32 views vs 32 per-view calls with a
    key-count readback each, same kernels and same results."""
    from paper_2409_09295_amd.replay import BatchedStep, PlainStep
    wl = scenes.config_metric(0)
    g = gs.Gaussians.from_map(wl.gmap)
    views = gs.Views(wl.cams)
    targets = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).to(DEV)
    step = BatchedStep(g, views, targets, optimize=False)
    step.capture()
    plain = PlainStep(g, wl.cams, views.split_images(targets), optimize=False)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    tb = timed(step.step, 10)
    tp = timed(plain.step, 3)
    _log(f"batched {tb * 1e3:.2f} ms, plain {tp * 1e3:.2f} ms, ratio {tp / tb:.2f}")
    assert tp / tb >= 3.0
    for v, im in enumerate(views.split_images(step.image)):
        torch.testing.assert_close(plain.rasts[v].image.view_as(im), im, rtol=0, atol=0)


def test_autotuner_caches_its_choice(gs, tmp_path):
    from paper_2409_09295_amd import autotune
    from paper_2409_09295_amd.replay import BatchedStep
    wl = _small_uneven(2)
    targets = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).to(DEV)
    step = BatchedStep(gs.Gaussians.from_map(wl.gmap), gs.Views(wl.cams), targets)
    cache = str(tmp_path / "tune.json")
    try:
        a = autotune.tune(step, cache=cache, reps=1)
        assert not a["cached"] and a["fwd_ppl"] in autotune.CHOICES and a["bwd_ppl"] in autotune.CHOICES
        assert len(a["table"]) == 2 * len(autotune.CHOICES) * len(autotune.STAGES) * len(autotune.SCHEDULES)
        assert gs.gs_get_tuning(gs.GS_TUNE_BWD_STAGE) == a["bwd_stage"]
        assert gs.gs_get_tuning(gs.GS_TUNE_FWD_PIXELS_PER_LANE) == a["fwd_ppl"]
        assert gs.gs_get_tuning(gs.GS_TUNE_FWD_SCHEDULE) == a["fwd_schedule"]
        assert gs.gs_get_tuning(gs.GS_TUNE_BWD_SCHEDULE) == a["bwd_schedule"]
        autotune.apply(0, 0)
        b = autotune.tune(step, cache=cache)
        assert b["cached"]
        for k in ("fwd_ppl", "bwd_ppl", "fwd_schedule", "bwd_schedule", "fwd_stage", "bwd_stage"):
            assert b[k] == a[k], k
        assert gs.gs_get_tuning(gs.GS_TUNE_BWD_SCHEDULE) == a["bwd_schedule"]
    finally:
        autotune.apply(0, 0)
