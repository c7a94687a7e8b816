"""Selective optimisation of the global stage (Sec. III-B2) on the GPU: the
per-Gaussian rendering error E_k(g), the active set thresholding and the
masked Adam update, against the FP64 oracle (needs an MI355X)."""
import numpy as np
import pytest
import torch

from oracle import gs_oracle as O
from paper_2409_09295_amd import scenes
from tests.gpu_helpers import f32, np_

pytestmark = pytest.mark.gpu
DEV = "cuda"
GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def _log(msg):
    print(msg, flush=True)


def _render(gs, wl):
    from paper_2409_09295_amd.rasterizer import Rasterizer
    g = gs.Gaussians.from_map(wl.gmap)
    views = gs.Views(wl.cams)
    rast = Rasterizer(g.n, views)
    rast.forward(g, wl.bg)
    torch.cuda.synchronize()
    return g, views, rast


def _gpu_error(gs, views, rast, n, target):
    err = torch.empty(views.n_views, n, dtype=torch.float32, device=DEV)
    gs.gs_render_error(rast.proj, n, rast.bins, views, rast.image, target, rast.n_contrib, err)
    torch.cuda.synchronize()
    return err


def _check_error(got, res, max_img_err=1e-4):
    """E_gpu vs E_ref: the GPU's residuals come from its own image, which is
    within max_img_err per channel of the oracle's, so a pixel's L1 residual
    may differ by 3 max_img_err and E by that times the splat's summed weight;
    on top, 1e-4 relative for the float32 weights and sums."""
    ref, wsum = res["err"], res["weight"]
    tol = 1e-4 * np.abs(ref) + 3 * max_img_err * wsum + 1e-7 * max(np.abs(ref).max(), 1e-30)
    d = np.abs(np.asarray(got, np.float64) - ref)
    worst = np.unravel_index(np.argmax(d / tol), d.shape)
    _log(f"  E: {int((ref > 0).sum())} nonzero entries, worst err/tol {d[worst] / tol[worst]:.3f}, "
         f"max rel {np.max(d / np.maximum(ref, 1e-30) * (ref > 1e-6 * ref.max())):.2e}")
    assert (d <= tol).all(), (worst, got[worst], ref[worst], tol[worst])


def _near_threshold_masks(gmap, cams, bg):
    res = O.render(gmap, cams, bg=bg)
    return [v["mask"] for v in res["views"]]


@pytest.fixture(params=[1, 3], ids=["per_tile", "persistent"])
def bwd_schedule(gs, request):
    """The backward tile schedule, which the error walk follows: one
    workgroup per tile (heaviest first), or persistent workgroups."""
    gs.gs_set_tuning(gs.GS_TUNE_BWD_SCHEDULE, request.param)
    yield request.param
    gs.gs_set_tuning(gs.GS_TUNE_BWD_SCHEDULE, 0)


@pytest.mark.parametrize("case", ["c1", "two_views_bg", "c2"])
def test_render_error_matches_oracle(gs, case, bwd_schedule):
    if case == "c1":
        wl = scenes.config_c1(0)
    elif case == "c2":
        wl = scenes.config_c2(0)
    else:
        base = scenes.config_c1(3)
        cam2 = scenes.perturb_pose(scenes.Camera(np.eye(3), np.zeros(3), 120.0, 120.0, 50.0, 40.0, 100,
                                                 72), np.random.default_rng(4))
        wl = scenes.Workload("c1_two_views", base.gmap, [base.cams[0], cam2], [], bg=(0.3, 0.6, 0.1))
    cams = [c.as_float32() for c in wl.cams]
    g, views, rast = _render(gs, wl)
    masks = _near_threshold_masks(wl.gmap, cams, wl.bg)
    rng = np.random.default_rng(8)
    img = views.split_images(rast.image)
    tg = []
    for v, (w, h) in enumerate(views.sizes):
        t = rng.random((3, h, w)).astype(np.float32)
        # near-threshold pixels: the target equals the GPU's own render, so
        # their residual is exactly 0 there; the oracle leaves them out
        t[:, masks[v]] = np_(img[v])[:, masks[v]]
        tg.append(t)
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in tg])).to(DEV)
    _log(f"{case}: {sum(int(m.sum()) for m in masks)} near-threshold px left out")
    err = _gpu_error(gs, views, rast, g.n, target)
    res = O.render_error(wl.gmap, cams, [t.astype(np.float64) for t in tg], bg=wl.bg, pixel_mask=masks)
    _check_error(np_(err), res)
    # repeat: only the float32 order of the atomic additions may differ
    err2 = _gpu_error(gs, views, rast, g.n, target)
    np.testing.assert_allclose(np_(err2), np_(err), rtol=1e-5, atol=1e-7 * float(err.max()))
    assert int(rast.bins.queue.abs().sum().item()) == 0


def test_render_error_metric_workload_sampled(gs):
    """200k-Gaussian room, 32 views at 640x480 (the benchmark's batch): the
    target equals the GPU's render except on sampled tiles of three views,
    so E comes from those tiles only, which the oracle composites; every
    other view's errors are exactly 0."""
    wl = scenes.config_metric(0)
    g, views, rast = _render(gs, wl)
    view_ids = [0, 17, 31]
    sub = [wl.cams[v].as_float32() for v in view_ids]
    rng = np.random.default_rng(70)
    picks = []
    for c in sub:
        TX, TY = O.tile_grid(c, 16)
        p = {(int(rng.integers(0, TY)), int(rng.integers(0, TX))) for _ in range(6)}
        picks.append(sorted(p | {(0, 0), (TY // 2, TX // 2)}))
    res0 = O.render(wl.gmap, sub, bg=wl.bg, tiles=picks)
    tgt = np_(rast.image).copy()
    offs = views.pixel_offsets()
    sub_t, masks = [], []
    for j, v in enumerate(view_ids):
        w, h = views.sizes[v]
        keep = np.zeros((h, w), bool)
        for ty, tx in picks[j]:
            keep[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = True
        m = res0["views"][j]["mask"]
        assert int((keep & m).sum()) <= 10
        keep &= ~m
        blk = tgt[3 * offs[v]:3 * (offs[v] + w * h)].reshape(3, h, w)
        blk[:, keep] = rng.random((3, int(keep.sum())))
        sub_t.append(blk.astype(np.float64))
        masks.append(m)
    target = torch.from_numpy(tgt).to(DEV)
    err = np_(_gpu_error(gs, views, rast, g.n, target))
    others = np.setdiff1d(np.arange(views.n_views), view_ids)
    assert (err[others] == 0.0).all()
    _log("metric: oracle error on the sampled tiles")
    res = O.render_error(wl.gmap, sub, sub_t, bg=wl.bg, pixel_mask=masks, tiles=picks)
    _check_error(err[view_ids], res)


@pytest.mark.parametrize("n,n_views", [(1, 1), (1000, 3), (70001, 5)])
def test_active_set_thresholding_bit_exact(gs, n, n_views):
    """The mask equals the float32 comparison max_k E_k(g) > eps, united with
    the always-on Gaussians; the count and the maxima are exact."""
    rng = np.random.default_rng(n)
    err = rng.exponential(1.0, size=(n_views, n)).astype(np.float32)
    err[:, ::7] = 0.0
    eps = np.float32(np.quantile(err.max(axis=0), 0.8))
    err[0, :3] = eps                         # ties with eps are not above it
    always = (rng.random(n) < 0.05).astype(np.uint8)
    e = torch.from_numpy(err).to(DEV)
    a = torch.from_numpy(always).to(DEV)
    mask = torch.full((n,), 7, dtype=torch.uint8, device=DEV)
    emax = torch.empty(n, dtype=torch.float32, device=DEV)
    cnt = torch.full((1,), 12345, dtype=torch.int32, device=DEV)
    gs.gs_active_set(e, n, n_views, float(eps), mask, a, emax, cnt)
    torch.cuda.synchronize()
    ref = (err.max(axis=0) > eps) | (always != 0)
    np.testing.assert_array_equal(np_(mask), ref.astype(np.uint8))
    np.testing.assert_array_equal(np_(emax), err.max(axis=0))
    assert int(cnt.item()) == int(ref.sum())
    # the oracle's thresholding of the same (exactly representable) values
    np.testing.assert_array_equal(ref, O.active_set(err.astype(np.float64), float(eps), always))


@pytest.mark.parametrize("n_gauss", [1, 1003, 4096])
def test_masked_adam_updates_only_the_active_set(gs, n_gauss):
    """Groups laid out [C][n]: elements of active Gaussians match the
    unmasked update bit for bit (and the FP64 oracle), the others keep their
    parameter and both moments."""
    rng = np.random.default_rng(n_gauss)
    comps = [3, 3, 4, 1, 48]
    lrs = [1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3]
    mask = (rng.random(n_gauss) < 0.3).astype(np.uint8)
    mask[0] = 1

    def make():
        out = []
        for c in comps:
            b = [rng.normal(size=c * n_gauss).astype(np.float32) for _ in range(4)]
            b[3] = np.abs(b[3])
            out.append(b)
        return out

    base = make()
    A = [[torch.from_numpy(x.copy()).to(DEV) for x in grp] for grp in base]
    B = [[torch.from_numpy(x.copy()).to(DEV) for x in grp] for grp in base]
    sa = torch.full((1,), 4, dtype=torch.int32, device=DEV)
    sb = torch.full((1,), 4, dtype=torch.int32, device=DEV)
    ga = gs.adam_groups([(p, g, m, v, lr) for (p, g, m, v), lr in zip(A, lrs)])
    gb = gs.adam_groups([(p, g, m, v, lr) for (p, g, m, v), lr in zip(B, lrs)])
    gs.gs_adam_step_groups_masked_dev(ga, 0.9, 0.999, 1e-15, sa, torch.from_numpy(mask).to(DEV), n_gauss)
    gs.gs_adam_step_groups_dev(gb, 0.9, 0.999, 1e-15, sb)
    torch.cuda.synchronize()
    assert int(sa.item()) == int(sb.item()) == 5
    for c, grp_a, grp_b, b0, lr in zip(comps, A, B, base, lrs):
        on = np.tile(mask != 0, c)
        for x, y, x0 in zip((grp_a[0], grp_a[2], grp_a[3]), (grp_b[0], grp_b[2], grp_b[3]),
                            (b0[0], b0[2], b0[3])):
            xa, ya = np_(x), np_(y)
            np.testing.assert_array_equal(xa[on], ya[on])
            np.testing.assert_array_equal(xa[~on], x0[~on])
        p, m, v = O.adam_step(b0[0], b0[1], b0[2], b0[3], f32(lr), f32(0.9), f32(0.999), f32(1e-15), 5,
                              mask=on)
        # float32 update: a few ulp of the parameter plus 1e-6 of the step
        # (bias corrections, square root and division each round once)
        d = np.abs(np_(grp_a[0]) - p)
        assert (d <= 2e-6 * np.abs(p) + 1e-6 * np.abs(p - b0[0]) + 1e-7).all(), d.max()


def test_selective_step_end_to_end(gs):
    """E on a two-view window, the active set at a threshold, and a masked
    Adam step: the GPU's set equals the oracle's FP64 set except for
    Gaussians whose error lies within tolerance of the threshold, and only
    active Gaussians move."""
    wl = scenes.config_c2(1)
    cams = [c.as_float32() for c in wl.cams]
    cam2 = scenes.perturb_pose(wl.cams[0], np.random.default_rng(9))
    wl = scenes.Workload("c2_two", wl.gmap, [wl.cams[0], cam2], [])
    cams = [c.as_float32() for c in wl.cams]
    g, views, rast = _render(gs, wl)
    masks = _near_threshold_masks(wl.gmap, cams, wl.bg)
    rng = np.random.default_rng(10)
    img = views.split_images(rast.image)
    tg = []
    for v, (w, h) in enumerate(views.sizes):
        t = np.clip(np_(img[v]) + rng.normal(0, 0.1, size=(3, h, w)), 0, 1).astype(np.float32)
        t[:, masks[v]] = np_(img[v])[:, masks[v]]
        tg.append(t)
    target = torch.from_numpy(np.concatenate([t.reshape(-1) for t in tg])).to(DEV)
    err = _gpu_error(gs, views, rast, g.n, target)
    res = O.render_error(wl.gmap, cams, [t.astype(np.float64) for t in tg], pixel_mask=masks)
    emax_ref = res["err"].max(axis=0)
    eps = float(np.quantile(emax_ref[emax_ref > 0], 0.85))
    always = np.zeros(g.n, np.uint8)
    always[-500:] = 1                     # the newly inserted local map
    mask = torch.empty(g.n, dtype=torch.uint8, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
    gs.gs_active_set(err, g.n, views.n_views, eps, mask, torch.from_numpy(always).to(DEV), None, cnt)
    torch.cuda.synchronize()
    got = np_(mask).astype(bool)
    ref = O.active_set(res["err"], eps, always)
    tol = 1e-4 * emax_ref + 3e-4 * res["weight"].max(axis=0) + 1e-7 * emax_ref.max()
    near = np.abs(emax_ref - eps) <= tol
    _log(f"active {int(got.sum())} of {g.n} ({got.mean():.1%}); {int(near.sum())} within tolerance of eps")
    np.testing.assert_array_equal(got[~near], ref[~near])
    assert int(cnt.item()) == int(got.sum())
    # a masked step moves exactly the active Gaussians
    grads = gs.Grads.zeros_like(g, views.n_views)
    dl = torch.from_numpy(np.sign(np.concatenate([(np_(i) - t).reshape(-1) for i, t in zip(img, tg)]))
                          .astype(np.float32) * 1e-5).to(DEV)
    rast.backward(g, dl, grads, gs.GS_BWD_OVERWRITE | gs.GS_BWD_NO_POSE, wl.bg)
    before = [np_(t).copy() for t in g.tensors()]
    mom = [(torch.zeros_like(t), torch.zeros_like(t)) for t in g.tensors()]
    gl = [grads.means, grads.log_scales, grads.quats, grads.opacity_logits, grads.sh]
    arr = gs.adam_groups([(p, gg, m, v, 1e-2) for p, gg, (m, v) in zip(g.tensors(), gl, mom)])
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    gs.gs_adam_step_groups_masked_dev(arr, 0.9, 0.999, 1e-15, step, mask, g.n)
    torch.cuda.synchronize()
    for k, t, b in zip(GROUPS, g.tensors(), before):
        moved = (np_(t) != b).reshape(-1, g.n).any(axis=0)
        assert not (moved & ~got).any(), k
