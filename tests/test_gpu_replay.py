"""Batched replay (one graph launch over many views) vs the eager and the
per-view paths, and the batched launch at the benchmark's full sizes vs the
FP64 oracle on sampled tiles (needs an MI355X)."""
import time

import numpy as np
import pytest
import torch

from oracle import gs_oracle as O
from paper_2409_09295_amd import scenes
from tests.gpu_helpers import assert_grad_close, np_, random_dl

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
            assert_grad_close(k, np_(gr[k]), np_(gr0[k]), rel=1e-5)
        # eager work of the program between replays
        _ = (targets * 2).sum().item()
    # per-view reference path: same images bit for bit, same summed gradients
    plain = PlainStep(g, wl.cams, views.split_images(targets), optimize=False)
    plain.step()
    torch.cuda.synchronize()
    for v, im in enumerate(views.split_images(img0)):
        torch.testing.assert_close(plain.rasts[v].image.view_as(im), im, rtol=0, atol=0)
    for k in GROUPS:
        assert_grad_close(k, np_(getattr(plain.grads, k)), np_(gr0[k]), rel=1e-5)
    assert_grad_close("xi", np_(plain.xi), np_(gr0["xi"]), rel=1e-5)


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


def _sampled_parity(gs, wl, view_ids, tiles_per_view, seed):
    """Every view rendered in one batched launch; images compared with the
    oracle on sampled tiles of ``view_ids``; gradients with dL/dC nonzero only
    on those tiles."""
    from tests.test_gpu_parity import _run_gpu
    views = gs.Views(wl.cams)
    rng = np.random.default_rng(seed)
    sub = [wl.cams[v].as_float32() for v in view_ids]
    picks = []
    for c in sub:
        TX, TY = O.tile_grid(c, 16)
        p = {(int(rng.integers(0, TY)), int(rng.integers(0, TX))) for _ in range(tiles_per_view)}
        p |= {(0, 0), (TY - 1, TX - 1), (TY // 2, TX // 2)}
        picks.append(sorted(p))
    _log(f"{wl.name}: oracle forward on {sum(map(len, picks))} sampled tiles of views {view_ids}")
    res0 = O.render(wl.gmap, sub, bg=wl.bg, tiles=picks)
    # dL/dC: random on the sampled tiles of the chosen views, zero elsewhere
    dl = np.zeros(3 * views.n_pixels, np.float32)
    offs = views.pixel_offsets()
    sub_dl = []
    for j, v in enumerate(view_ids):
        w, h = views.sizes[v]
        blk = random_dl([(w, h)], seed + j).reshape(3, h, w)
        keep = np.zeros((h, w), bool)
        for ty, tx in picks[j]:
            keep[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = True
        blk[:, ~keep] = 0.0
        blk[:, res0["views"][j]["mask"]] = 0.0
        dl[3 * offs[v]:3 * (offs[v] + w * h)] = blk.reshape(-1)
        sub_dl.append(blk.astype(np.float64))
    _log(f"{wl.name}: GPU, {len(wl.cams)} views in one launch")
    out = _run_gpu(gs, wl, dl)
    imgs = views.split_images(out["image"])
    worst, masked = 0.0, 0
    for j, v in enumerate(view_ids):
        r = res0["views"][j]
        m = ~r["mask"] & np.isfinite(r["image"][0])
        masked += int(r["mask"].sum())
        d = np.abs(np_(imgs[v]) - r["image"])[:, m]
        worst = max(worst, float(d.max()))
        ncg = np_(views.split_maps(out["nc"])[v])
        np.testing.assert_array_equal(ncg[m], r["n_contrib"][m])
    _log(f"{wl.name}: image worst {worst:.3e}, {masked} near-threshold px")
    assert worst <= 1e-4
    _log(f"{wl.name}: oracle backward")
    res = O.render(wl.gmap, sub, bg=wl.bg, dL_dimage=sub_dl, tiles=picks)
    gr = out["grads"]
    for k in GROUPS:
        assert_grad_close(k, np_(getattr(gr, k)), res["grads"][k])
    xi = np_(gr.xi)
    assert_grad_close("xi", xi[view_ids], res["grads"]["xi"])
    others = np.setdiff1d(np.arange(len(wl.cams)), view_ids)
    assert np.abs(xi[others]).max() == 0.0


def test_metric_workload_sampled_parity(gs):
    """200k Gaussians, 32 views at 640x480: the benchmark's batch."""
    from paper_2409_09295_amd import autotune
    from paper_2409_09295_amd.replay import BatchedStep
    wl = scenes.config_metric(0)
    # the launch shape the benchmark times
    g = gs.Gaussians.from_map(wl.gmap)
    targets = torch.from_numpy(np.concatenate([t.reshape(-1) for t in wl.targets])).to(DEV)
    tuned = autotune.tune(BatchedStep(g, gs.Views(wl.cams), targets))
    _log(f"tuned {tuned['fwd_ppl']}/{tuned['bwd_ppl']}")
    try:
        _sampled_parity(gs, wl, [0, 17, 31], 6, seed=40)
    finally:
        autotune.apply(0, 0)


def test_uneven_views_sampled_parity(gs):
    """500k Gaussians, 32 keyframes of four sizes up to 1200x680."""
    wl = scenes.config_c4(0)
    _sampled_parity(gs, wl, [0, 1, 2, 3], 4, seed=50)


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
        assert gs.gs_get_tuning(gs.GS_TUNE_FWD_PIXELS_PER_LANE) == a["fwd_ppl"]
        b = autotune.tune(step, cache=cache)
        assert b["cached"] and (b["fwd_ppl"], b["bwd_ppl"]) == (a["fwd_ppl"], a["bwd_ppl"])
    finally:
        autotune.apply(0, 0)
