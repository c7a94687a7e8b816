"""GPU vs FP64 oracle parity, stage by stage and end to end (needs an MI355X)."""
import math

import numpy as np
import pytest
import torch

from oracle import gs_oracle as O
from paper_2409_09295_amd import scenes
from tests.gpu_helpers import (assert_grad_close, assert_same_up_to_order, f32, np_, term_mass,
                               random_dl, u32, u64)

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _log(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# binning: bit-exact keys, values, ranges given the same splats
# ---------------------------------------------------------------------------

BIN_CASES = {
    "one_view_160x120": [scenes.pinhole(160, 120, 150.0)],
    "ragged_multi_view": [scenes.pinhole(100, 70, 80.0), scenes.pinhole(320, 240, 300.0),
                          scenes.pinhole(48, 40, 40.0), scenes.pinhole(1200, 680, 984.0)],
    # 1 + 6 tiles: fewer tiles than the persistent schedule's counters
    "tiny_views": [scenes.pinhole(16, 16, 14.0), scenes.pinhole(40, 20, 30.0)],
}


def _oracle_tile_counts(sp, cams):
    """Per-(view, splat) tile counts from the oracle's rectangles, as the
    projection stores them."""
    return np.stack([O.tile_rects(sp.xy[v, :, 0].astype(np.float64), sp.xy[v, :, 1].astype(np.float64),
                                  sp.radius[v], c.width, c.height, 16)[4]
                     for v, c in enumerate(cams)]).astype(np.int32)


def _gpu_bins(gs, sp, cams, capacity=None, sync=True, stored_counts=False, keys=True):
    views = gs.Views(cams)
    proj = gs.Projected.from_splats(sp)
    if stored_counts:   # the path that takes the projection's tile counts
        proj.tiles = torch.from_numpy(_oracle_tile_counts(sp, cams)).to(DEV)
    V, N = sp.radius.shape
    cap = capacity if capacity is not None else 64 * N * V + 1024
    bins = gs.Bins.empty(cap, views.n_tiles, keys=keys)
    ws = gs.workspace(gs.gs_bin_sort_workspace_size(N, views, cap))
    n = gs.gs_bin_sort(proj, N, views, bins, ws, sync=sync)
    torch.cuda.synchronize()
    return views, proj, bins, n


@pytest.mark.parametrize("case", list(BIN_CASES))
@pytest.mark.parametrize("sync", [True, False])
@pytest.mark.parametrize("stored", [False, True], ids=["counted", "stored_counts"])
@pytest.mark.parametrize("with_keys", [True, False], ids=["keys", "tile_ids"])
def test_bin_sort_bit_exact(gs, case, sync, stored, with_keys):
    cams = BIN_CASES[case]
    n = 2500 if case != "ragged_multi_view" else 6000
    sp = scenes.random_splats(n, cams, seed=21, depth_ties=0.2, cull_frac=0.05)
    _log(f"bin_sort case={case} sync={sync} stored_counts={stored} keys={with_keys} n={n}")
    keys, vals, ranges, _, _ = O.bin_splats([sp.xy[v] for v in range(len(cams))],
                                            [sp.rgb_depth[v, :, 3] for v in range(len(cams))],
                                            [sp.radius[v] for v in range(len(cams))], cams, 16)
    views, proj, bins, nk = _gpu_bins(gs, sp, cams, sync=sync, stored_counts=stored,
                                      keys=with_keys)
    got_n = int(u32(bins.n_keys)[0])
    assert got_n == len(keys)
    if sync:
        assert nk == len(keys)
    if with_keys:
        np.testing.assert_array_equal(u64(bins.keys)[:got_n], keys)
    else:
        assert bins.keys is None
    np.testing.assert_array_equal(u32(bins.values)[:got_n], vals)
    np.testing.assert_array_equal(u32(bins.ranges), ranges)
    # repeat: integer outputs are deterministic
    views2, proj2, bins2, _ = _gpu_bins(gs, sp, cams, sync=sync, stored_counts=stored,
                                        keys=with_keys)
    if with_keys:
        np.testing.assert_array_equal(u64(bins2.keys)[:got_n], u64(bins.keys)[:got_n])
    np.testing.assert_array_equal(u32(bins2.values)[:got_n], u32(bins.values)[:got_n])
    np.testing.assert_array_equal(u32(bins2.order), u32(bins.order))


@pytest.mark.parametrize("n", [700, 1500, 3000, 6000])
def test_bin_sort_crowded_tiles(gs, n):
    """Every splat covers the same few tiles: per-tile lists of up to n keys
    (through every per-tile sort: one wavefront, four wavefronts with 8 or 16
    pairs per lane, and the radix sort past 4,096), a third of them at
    repeated depths so that ties fall back to the Gaussian index."""
    cams = [scenes.pinhole(48, 40, 40.0)]
    sp = scenes.random_splats(n, cams, seed=33, depth_ties=0.35, cull_frac=0.02)
    rng = np.random.default_rng(34)
    sp.xy[0, :, 0] = rng.uniform(14.0, 18.0, n)
    sp.xy[0, :, 1] = rng.uniform(14.0, 18.0, n)
    sp.radius[0] = np.where(sp.radius[0] > 0, rng.integers(1, 6, n), 0).astype(np.int32)
    keys, vals, ranges, _, _ = O.bin_splats([sp.xy[0]], [sp.rgb_depth[0, :, 3]], [sp.radius[0]],
                                            cams, 16)
    longest = int((ranges[:, 1] - ranges[:, 0]).max())
    _log(f"crowded tiles n={n}: {len(keys)} keys, longest list {longest}")
    for sync, with_keys in ((True, True), (False, True), (False, False)):
        views, proj, bins, nk = _gpu_bins(gs, sp, cams, sync=sync, keys=with_keys)
        got_n = int(u32(bins.n_keys)[0])
        assert got_n == len(keys)
        if with_keys:
            np.testing.assert_array_equal(u64(bins.keys)[:got_n], keys)
        np.testing.assert_array_equal(u32(bins.values)[:got_n], vals)
        np.testing.assert_array_equal(u32(bins.ranges), ranges)


def _length_group(x):
    """Group of a tile list of x keys in the tile order: 0 when empty, then
    half octaves (1 + 2 floor(log2 x) + the bit below the leading one)."""
    if x == 0:
        return 0
    lg = int(x).bit_length() - 1
    half = (int(x) >> (lg - 1)) & 1 if lg > 0 else 0
    return min(31, 1 + 2 * lg + half)


def test_tile_order_longest_first(gs):
    """bins.order is the stable sort of the tiles by list-length group (half
    octaves), longest group first, and compositing gives the same image with
    it as in plain tile order."""
    cams = BIN_CASES["ragged_multi_view"]
    sp = scenes.random_splats(4000, cams, seed=33)
    views, proj, bins, nk = _gpu_bins(gs, sp, cams)
    assert views.n_tiles > 4 * 256   # several workgroups of the order kernels
    order = np_(bins.order).astype(np.int64)
    assert sorted(order.tolist()) == list(range(views.n_tiles))
    rg = np_(bins.ranges).astype(np.int64)
    ln = rg[:, 1] - rg[:, 0]

    groups = np.array([_length_group(x) for x in ln])
    np.testing.assert_array_equal(order, np.argsort(-groups, kind="stable"))
    assert ln[order[0]] == ln.max()
    outs = []
    for use_order in (True, False):
        b = bins if use_order else gs.Bins(bins.keys, bins.values, bins.ranges, bins.n_keys,
                                           bins.capacity, None)
        P = views.n_pixels
        img = torch.empty(3 * P, device=DEV)
        Tf = torch.empty(P, device=DEV)
        nc = torch.empty(P, dtype=torch.int32, device=DEV)
        gs.gs_render_fwd(proj, sp.radius.shape[1], b, views, (0.2, 0.1, 0.05), img, Tf, nc, None)
        torch.cuda.synchronize()
        outs.append((img, Tf, nc))
    for a, c in zip(*outs):
        torch.testing.assert_close(a, c, rtol=0, atol=0)


def test_bin_sort_all_culled(gs):
    cams = [scenes.pinhole(64, 48, 60.0)]
    sp = scenes.random_splats(500, cams, seed=2)
    sp.radius[:] = 0
    views, proj, bins, nk = _gpu_bins(gs, sp, cams)
    assert nk == 0
    assert int(u32(bins.n_keys)[0]) == 0
    assert (u32(bins.ranges) == 0).all()
    # returned before any range existed: the order is the identity
    np.testing.assert_array_equal(u32(bins.order), np.arange(views.n_tiles))


@pytest.mark.parametrize("size", [(16, 16), (40, 23)], ids=["one_tile", "six_tiles"])
def test_tile_order_small_grids(gs, size):
    """Grids smaller than one workgroup of the order kernels, with empty
    tiles: the order is still the stable sort by list-length group."""
    cams = [scenes.pinhole(size[0], size[1], 20.0)]
    sp = scenes.random_splats(40, cams, seed=9)
    views, proj, bins, nk = _gpu_bins(gs, sp, cams)
    rg = u32(bins.ranges).astype(np.int64).reshape(-1, 2)
    ln = rg[:, 1] - rg[:, 0]
    grp = np.array([_length_group(x) for x in ln])
    np.testing.assert_array_equal(u32(bins.order), np.argsort(-grp, kind="stable"))


def test_bin_sort_capacity(gs):
    cams = [scenes.pinhole(160, 120, 150.0)]
    sp = scenes.random_splats(800, cams, seed=5)
    keys, *_ = O.bin_splats([sp.xy[0]], [sp.rgb_depth[0, :, 3]], [sp.radius[0]], cams, 16)
    # synchronous: reports the required capacity and enqueues nothing more
    with pytest.raises(gs.GsError) as ei:
        _gpu_bins(gs, sp, cams, capacity=len(keys) - 1, sync=True)
    assert ei.value.status == gs.GS_ERR_CAPACITY
    assert ei.value.required == len(keys)
    # asynchronous: the device count reports the overflow, no key is emitted
    views, proj, bins, _ = _gpu_bins(gs, sp, cams, capacity=len(keys) - 1, sync=False)
    assert int(u32(bins.n_keys)[0]) == len(keys)
    assert (u32(bins.ranges) == 0).all()
    # exact capacity succeeds
    views, proj, bins, nk = _gpu_bins(gs, sp, cams, capacity=len(keys), sync=True)
    assert nk == len(keys)
    np.testing.assert_array_equal(u64(bins.keys)[:nk], keys)


# ---------------------------------------------------------------------------
# compositing from given splats
# ---------------------------------------------------------------------------

def _render_gpu(gs, sp, cams, bg=(0.0, 0.0, 0.0)):
    views, proj, bins, nk = _gpu_bins(gs, sp, cams)
    P = views.n_pixels
    img = torch.empty(3 * P, device=DEV)
    Tf = torch.empty(P, device=DEV)
    nc = torch.empty(P, dtype=torch.int32, device=DEV)
    dep = torch.empty(P, device=DEV)
    gs.gs_render_fwd(proj, sp.radius.shape[1], bins, views, bg, img, Tf, nc, dep)
    torch.cuda.synchronize()
    return views, img, Tf, nc, dep


@pytest.fixture
def ppl_setting(gs, request):
    """Runs a test under a (forward, backward) pixels-per-lane setting of the
    tile kernels and, when given, a tile schedule for both."""
    fwd, bwd, *rest = request.param
    sched = rest[0] if rest else 0
    stage = rest[1] if len(rest) > 1 else 0
    gs.gs_set_tuning(gs.GS_TUNE_FWD_PIXELS_PER_LANE, fwd)
    gs.gs_set_tuning(gs.GS_TUNE_BWD_PIXELS_PER_LANE, bwd)
    for key in (gs.GS_TUNE_FWD_SCHEDULE, gs.GS_TUNE_BWD_SCHEDULE):
        gs.gs_set_tuning(key, sched)
    for key in (gs.GS_TUNE_FWD_STAGE, gs.GS_TUNE_BWD_STAGE):
        gs.gs_set_tuning(key, stage)
    yield request.param
    for key in (gs.GS_TUNE_FWD_PIXELS_PER_LANE, gs.GS_TUNE_BWD_PIXELS_PER_LANE,
                gs.GS_TUNE_FWD_SCHEDULE, gs.GS_TUNE_BWD_SCHEDULE, gs.GS_TUNE_FWD_STAGE,
                gs.GS_TUNE_BWD_STAGE):
        gs.gs_set_tuning(key, 0)


# (forward, backward pixels per lane[, tile schedule[, splats staged per
# thread]]): one workgroup per tile (heaviest first: the default; tile id
# order), persistent workgroups drawing tiles from counters (as many as fit,
# or half), and both LDS batch sizes
_HF, _ID, _PS, _PH = 1, 2, 3, 4
PPL_SETTINGS = [(1, 1), (2, 2), (4, 4), (4, 4, _ID), (1, 1, _PS), (2, 2, _PS), (4, 4, _PS),
                (4, 4, _HF, 2), (4, 4, _HF, 1), (2, 2, _HF, 1), (1, 1, _PH, 2)]


@pytest.mark.parametrize("ppl_setting", PPL_SETTINGS, indirect=True)
@pytest.mark.parametrize("case", list(BIN_CASES))
def test_render_fwd_splats(gs, case, ppl_setting):
    cams = BIN_CASES[case]
    n = 2500 if case != "ragged_multi_view" else 4000
    sp = scenes.random_splats(n, cams, seed=31)
    bg = (0.2, 0.1, 0.05)
    _log(f"render_fwd splats case={case}")
    res, *_ = O.render_splats(sp, 16, bg=bg)
    views, img, Tf, nc, dep = _render_gpu(gs, sp, cams, bg)
    imgs = views.split_images(img)
    Tfs = views.split_maps(Tf)
    ncs = views.split_maps(nc)
    deps = views.split_maps(dep)
    total_masked = 0
    for v, r in enumerate(res):
        m = ~r["mask"]
        total_masked += int(r["mask"].sum())
        d = np.abs(np_(imgs[v]) - r["image"])[:, m]
        assert d.max() <= 1e-4, (v, d.max())
        assert np.abs(np_(Tfs[v]) - r["T_final"])[m].max() <= 1e-4
        np.testing.assert_array_equal(np_(ncs[v])[m], r["n_contrib"][m])
        assert np.abs(np_(deps[v]) - r["depth"])[m].max() <= 1e-3
    assert total_masked <= 0.01 * views.n_pixels, total_masked


# ---------------------------------------------------------------------------
# full pipeline from Gaussian parameters
# ---------------------------------------------------------------------------

def ocams(wl):
    """The cameras exactly as the float32 records hand them to the kernels."""
    return [c.as_float32() for c in wl.cams]


def _run_gpu(gs, wl, dl=None, flags=0):
    from paper_2409_09295_amd.rasterizer import Rasterizer
    g = gs.Gaussians.from_map(wl.gmap)
    views = gs.Views(wl.cams)
    rast = Rasterizer(g.n, views)
    img = rast.forward(g, wl.bg)
    out = dict(views=views, rast=rast, g=g, image=img.clone(), T=rast.final_T.clone(),
               nc=rast.n_contrib.clone())
    if dl is not None:
        grads = gs.Grads.zeros_like(g, views.n_views)
        rast.backward(g, torch.from_numpy(dl).to(DEV), grads, flags, wl.bg)
        out["grads"] = grads
    torch.cuda.synchronize()
    return out


def _check_projection(gs, wl, out, res):
    V = len(wl.cams)
    proj = out["rast"].proj
    for v in range(V):
        P = res["proj"][v]
        vis = P["visible"]
        rad = np_(proj.radius[v])
        xy = np_(proj.xy[v])
        co = np_(proj.conic_opacity[v])
        rd = np_(proj.rgb_depth[v])
        ext = P["ext"]
        amb = np.abs(ext - np.round(ext)) < O.BAND_EXTENT * np.maximum(ext, 1.0)
        z_amb = np.abs(P["z"] - O.Z_NEAR) < 1e-5
        ok = ~(amb | z_amb)
        np.testing.assert_array_equal((rad > 0)[ok], vis[ok])
        np.testing.assert_array_equal(rad[ok & vis], P["radius"][ok & vis])
        sel = vis & (rad > 0)
        np.testing.assert_allclose(xy[sel, 0], P["u"][sel], rtol=2e-6, atol=2e-4)
        np.testing.assert_allclose(xy[sel, 1], P["v"][sel], rtol=2e-6, atol=2e-4)
        np.testing.assert_allclose(rd[sel, 3], P["z"][sel], rtol=1e-6)
        np.testing.assert_allclose(co[sel, 3], P["opacity"][sel], rtol=1e-6)
        np.testing.assert_allclose(rd[sel, :3], P["rgb"][sel], atol=2e-5)
        conic = P["conic"][sel]
        scale = np.abs(conic).max(axis=1, keepdims=True)
        assert (np.abs(co[sel, :3] - conic) <= 2e-5 * scale + 1e-9).all()
        # stored tile counts: the oracle's rectangles of the stored centres and radii
        cam = wl.cams[v]
        *_, cnt = O.tile_rects(xy[:, 0].astype(np.float64), xy[:, 1].astype(np.float64),
                               np.where(rad > 0, rad, 0), int(cam.width), int(cam.height), 16)
        np.testing.assert_array_equal(np_(proj.tiles[v]).astype(np.int64), cnt)


# Near-threshold pixels (a splat within float32 rounding of the 1/255 or 0.99
# alpha bounds, of the 1e-4 transmittance stop, of a tile edge or of another
# splat's depth) are left out of the comparison.  They must stay rare, or the
# comparison would silently cover less: at most this fraction of the pixels
# compared (the oracle flags 3 of 19,200 pixels at 160x120, 96 of 76,800 at
# 320x240 and 1 of 3,072 on the sampled tiles of the 640x480 room).
MAX_MASKED_FRAC = 2e-3


def _compare_images(views, out, res, tol=1e-4, max_masked=None):
    imgs = views.split_images(out["image"])
    masked = 0
    compared = 0
    worst = 0.0
    for v, r in enumerate(res["views"]):
        finite = np.isfinite(r["image"][0])
        m = ~r["mask"] & finite
        masked += int(r["mask"].sum())
        compared += int(finite.sum())
        d = np.abs(np_(imgs[v]) - r["image"])[:, m]
        worst = max(worst, float(d.max()) if d.size else 0.0)
    bound = max_masked if max_masked is not None else int(MAX_MASKED_FRAC * compared)
    _log(f"  images: worst {worst:.3e} over {compared - masked} px, {masked} near-threshold px "
         f"(bound {bound})")
    assert worst <= tol, worst
    assert masked <= bound, (masked, bound)
    return masked, worst


def _masked_dl(views, res, dl):
    """Zero dL/dC at near-threshold pixels (both paths get the same)."""
    dl = dl.copy()
    off = 0
    for (w, h), r in zip(views.sizes, res["views"]):
        blk = dl[3 * off:3 * (off + w * h)].reshape(3, h, w)
        blk[:, r["mask"]] = 0.0
        off += w * h
    return dl


def _split_dl(views, dl):
    out, off = [], 0
    for (w, h) in views.sizes:
        out.append(dl[3 * off:3 * (off + w * h)].reshape(3, h, w).astype(np.float64))
        off += w * h
    return out


def _grad_parity(gs, wl, seed, check_pose=True):
    views = gs.Views(wl.cams)
    _log(f"grad parity {wl.name}: oracle forward")
    res0 = O.render(wl.gmap, ocams(wl), bg=wl.bg)
    dl = _masked_dl(views, res0, random_dl(views.sizes, seed))
    _log(f"grad parity {wl.name}: GPU")
    out = _run_gpu(gs, wl, dl)
    _compare_images(views, out, res0)
    _log(f"grad parity {wl.name}: oracle backward")
    res = O.render(wl.gmap, ocams(wl), bg=wl.bg, dL_dimage=_split_dl(views, dl))
    mass = term_mass(wl.gmap, ocams(wl), _split_dl(views, dl), bg=wl.bg)
    g = out["grads"]
    stats = {}
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        stats[name] = assert_grad_close(name, np_(getattr(g, name)), res["grads"][name], mass_fn=mass)
    if check_pose:
        stats["xi"] = assert_grad_close("xi", np_(g.xi), res["grads"]["xi"])
    _log(f"grad parity {wl.name}: relative L2 {stats}")
    return out, res


def test_c1_projection_and_image(gs):
    wl = scenes.config_c1(0)
    res = O.render(wl.gmap, ocams(wl), bg=wl.bg)
    out = _run_gpu(gs, wl)
    _check_projection(gs, wl, out, res)
    masked, worst = _compare_images(out["views"], out, res)
    _log(f"c1 image: {masked} near-threshold px, worst {worst:.3e} elsewhere")
    # c1 passes with no exclusions: every pixel, flagged or not
    full = np.abs(np_(out["image"]).reshape(3, 120, 160) - res["views"][0]["image"]).max()
    assert full <= 1e-4, full
    nc = np_(out["nc"]).reshape(120, 160)
    np.testing.assert_array_equal(nc, res["views"][0]["n_contrib"])


@pytest.mark.parametrize("ppl_setting", PPL_SETTINGS, indirect=True)
def test_c1_gradients(gs, ppl_setting):
    _grad_parity(gs, scenes.config_c1(0), seed=5)


def test_c2_gradients(gs):
    _grad_parity(gs, scenes.config_c2(0), seed=6)


@pytest.mark.parametrize("ppl_setting", [(2, 4)], indirect=True)
def test_background_and_multi_view_gradients(gs, ppl_setting):
    # two views of one cloud, non-black background: gradients sum over views
    wl = scenes.config_c1(3)
    rng = np.random.default_rng(4)
    cam2 = scenes.perturb_pose(scenes.Camera(np.eye(3), np.zeros(3), 120.0, 120.0, 50.0, 40.0, 100, 72),
                               rng)
    wl = scenes.Workload("c1_two_views", wl.gmap, [wl.cams[0], cam2], [], bg=(0.3, 0.6, 0.1))
    _grad_parity(gs, wl, seed=7)


def test_c3_sampled_tiles(gs):
    """Full-size single-view mapping workload (640x480, 200k Gaussians, SH 3):
    images on sampled tiles, and all gradients with dL/dC restricted to those
    tiles (so the oracle composites only the sampled tiles)."""
    wl = scenes.config_c3(0)
    views = gs.Views(wl.cams)
    rng = np.random.default_rng(0)
    TX, TY = 40, 30
    picks = [(int(ty), int(tx)) for ty, tx in zip(rng.integers(0, TY, 10), rng.integers(0, TX, 10))]
    picks += [(0, 0), (TY - 1, TX - 1), (TY // 2, TX // 2)]
    _log("c3: oracle forward on sampled tiles")
    res0 = O.render(wl.gmap, ocams(wl), tiles=[picks])
    dl = random_dl(views.sizes, 11).reshape(3, 480, 640)
    keep = np.zeros((480, 640), bool)
    for ty, tx in picks:
        keep[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = True
    dl[:, ~keep] = 0.0
    dl = _masked_dl(views, res0, dl.reshape(-1))
    _log("c3: GPU")
    out = _run_gpu(gs, wl, dl)
    masked, worst = _compare_images(views, out, res0, max_masked=10)
    _log(f"c3 sampled image: masked {masked} px, worst {worst:.3e}")
    _log("c3: oracle backward on sampled tiles")
    res = O.render(wl.gmap, ocams(wl), dL_dimage=_split_dl(views, dl), tiles=[picks])
    mass = term_mass(wl.gmap, ocams(wl), _split_dl(views, dl), tiles=[picks])
    g = out["grads"]
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        assert_grad_close(name, np_(getattr(g, name)), res["grads"][name], mass_fn=mass)
    assert_grad_close("xi", np_(g.xi), res["grads"]["xi"])


def test_pose_only_matches_full(gs):
    wl = scenes.config_c1(1)
    views = gs.Views(wl.cams)
    dl = random_dl(views.sizes, 3)
    full = _run_gpu(gs, wl, dl, flags=0)["grads"]
    po = _run_gpu(gs, wl, dl, flags=gs.GS_BWD_POSE_ONLY)["grads"]
    np.testing.assert_allclose(np_(po.xi), np_(full.xi), rtol=1e-5, atol=1e-9)
    assert np.abs(np_(po.means)).max() == 0.0
    nop = _run_gpu(gs, wl, dl, flags=gs.GS_BWD_NO_POSE)["grads"]
    assert np.abs(np_(nop.xi)).max() == 0.0
    assert_same_up_to_order("means", np_(nop.means), np_(full.means), rel=1e-4)


def test_keep_clear_matches_clearing_backward(gs):
    """GS_BWD_KEEP_CLEAR on a zeroed workspace, twice in a row with different
    dL/dC, gives each time the gradients of a backward that clears its
    partials first: the first call leaves the workspace clear."""
    from paper_2409_09295_amd.rasterizer import Rasterizer
    wl = scenes.config_c1(2)
    g = gs.Gaussians.from_map(wl.gmap)
    views = gs.Views(wl.cams)
    rast = Rasterizer(g.n, views)
    rast.forward(g, wl.bg)
    ws = gs.workspace(gs.gs_render_bwd_workspace_size(g.n, views), DEV).zero_()
    for seed in (4, 5):
        dl = torch.from_numpy(random_dl(views.sizes, seed)).to(DEV)
        ref = gs.Grads.zeros_like(g, views.n_views)
        rast.backward(g, dl, ref, gs.GS_BWD_OVERWRITE, wl.bg)
        got = gs.Grads.zeros_like(g, views.n_views)
        gs.gs_render_bwd(g, rast.proj, rast.bins, views, wl.bg, dl, rast.final_T, rast.n_contrib,
                         got, gs.GS_BWD_OVERWRITE | gs.GS_BWD_KEEP_CLEAR, ws)
        torch.cuda.synchronize()
        _log(f"keep-clear call with dL seed {seed}")
        for k in ("means", "log_scales", "quats", "opacity_logits", "sh", "xi"):
            assert_same_up_to_order(k, np_(getattr(got, k)), np_(getattr(ref, k)))


# ---------------------------------------------------------------------------
# elementwise kernels
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,offset,masked", [(1, 0, False), (1003, 0, False), (4096, 1, False),
                                             (5000, 0, True)])
def test_adam_step(gs, n, offset, masked):
    rng = np.random.default_rng(n)
    base = [rng.normal(size=n + offset).astype(np.float32) for _ in range(4)]
    base[3] = np.abs(base[3])
    mask = (rng.random(n) < 0.5).astype(np.uint8) if masked else None
    t = [torch.from_numpy(b).to(DEV)[offset:] for b in base]
    p, g, m, v = t
    for step in (1, 2, 7):
        ref = O.adam_step(np_(p), np_(g), np_(m), np_(v), f32(1e-3), f32(0.9), f32(0.999), f32(1e-8),
                          step, mask)
        gs.gs_adam_step(p, g, m, v, 1e-3, 0.9, 0.999, 1e-8, step,
                        torch.from_numpy(mask).to(DEV) if mask is not None else None)
        torch.cuda.synchronize()
        for got, r in zip((p, m, v), ref):
            np.testing.assert_allclose(np_(got), r, rtol=2e-6, atol=1e-7)


def test_adam_groups_match_per_group_calls(gs):
    """The single-launch grouped update equals one device-step call per
    group bit for bit (ragged and unaligned groups included), and skips
    everything, counter included, when the binning guard reports overflow."""
    rng = np.random.default_rng(9)
    sizes = [(1, 0), (1003, 0), (4096, 1), (37, 3), (250000, 0)]
    lrs = [1e-3, 5e-2, 2.5e-3, 1e-2, 1.6e-4]

    def make():
        out = []
        for (n, off) in sizes:
            b = [rng.normal(size=n + off).astype(np.float32) for _ in range(4)]
            b[3] = np.abs(b[3])
            out.append([torch.from_numpy(x).to(DEV)[off:] for x in b])
        return out

    A = make()
    B = [[t.clone() for t in grp] for grp in A]
    sa = torch.zeros(1, dtype=torch.int32, device=DEV)
    sb = torch.zeros(1, dtype=torch.int32, device=DEV)
    guard = torch.tensor([10], dtype=torch.int32, device=DEV)
    arr = gs.adam_groups([(p, g, m, v, lr) for (p, g, m, v), lr in zip(A, lrs)])
    for step in range(3):
        gs.gs_adam_step_groups_dev(arr, 0.9, 0.999, 1e-15, sa, guard_n_keys=guard, guard_capacity=20)
        for k, ((p, g, m, v), lr) in enumerate(zip(B, lrs)):
            gs.gs_adam_step_dev(p, g, m, v, lr, 0.9, 0.999, 1e-15, sb, k == len(B) - 1,
                                guard_n_keys=guard, guard_capacity=20)
    torch.cuda.synchronize()
    assert int(sa.item()) == int(sb.item()) == 3
    for ga, gb in zip(A, B):
        for x, y in zip(ga, gb):
            torch.testing.assert_close(x, y, rtol=0, atol=0)
    before = [t.clone() for grp in A for t in grp]
    gs.gs_adam_step_groups_dev(arr, 0.9, 0.999, 1e-15, sa, guard_n_keys=guard, guard_capacity=5)
    torch.cuda.synchronize()
    assert int(sa.item()) == 3
    for x, y in zip([t for grp in A for t in grp], before):
        torch.testing.assert_close(x, y, rtol=0, atol=0)


@pytest.mark.parametrize("ppl_setting", PPL_SETTINGS, indirect=True)
def test_render_fwd_l1_matches_separate_calls(gs, ppl_setting):
    """The fused compositing + L1 pass gives the same image, final T,
    n_contrib and dL/dC bit for bit as gs_render_fwd then gs_l1_loss_grad,
    and the same loss up to summation order (ragged views, background)."""
    cams = BIN_CASES["ragged_multi_view"]
    sp = scenes.random_splats(3000, cams, seed=41)
    views, proj, bins, nk = _gpu_bins(gs, sp, cams)
    P = views.n_pixels
    bg = (0.1, 0.3, 0.2)
    rng = np.random.default_rng(42)
    target = torch.from_numpy(rng.random(3 * P).astype(np.float32)).to(DEV)
    a = [torch.empty(3 * P, device=DEV), torch.empty(P, device=DEV),
         torch.empty(P, dtype=torch.int32, device=DEV), torch.empty(3 * P, device=DEV),
         torch.zeros(1, dtype=torch.float64, device=DEV)]
    b = [t.clone() for t in a]
    N = sp.radius.shape[1]
    gs.gs_render_fwd(proj, N, bins, views, bg, a[0], a[1], a[2])
    gs.gs_l1_loss_grad(a[0], target, views, a[3], a[4])
    ws = gs.workspace(gs.gs_render_fwd_l1_workspace_size(views))
    gs.gs_render_fwd_l1(proj, N, bins, views, bg, b[0], b[1], b[2], target, b[3], b[4], ws)
    torch.cuda.synchronize()
    for x, y in zip(a[:4], b[:4]):
        torch.testing.assert_close(x, y, rtol=0, atol=0)
    np.testing.assert_allclose(float(b[4].item()), float(a[4].item()), rtol=1e-6)


def test_l1_loss_grad(gs):
    cams = [scenes.pinhole(50, 30, 40.0), scenes.pinhole(17, 9, 10.0)]
    views = gs.Views(cams)
    rng = np.random.default_rng(0)
    imgs = [rng.random((3, h, w)).astype(np.float32) for (w, h) in views.sizes]
    tgts = [rng.random((3, h, w)).astype(np.float32) for (w, h) in views.sizes]
    tgts[0][0, 0, :5] = imgs[0][0, 0, :5]       # exact ties -> sign 0
    img = torch.from_numpy(np.concatenate([x.reshape(-1) for x in imgs])).to(DEV)
    tgt = torch.from_numpy(np.concatenate([x.reshape(-1) for x in tgts])).to(DEV)
    dl = torch.empty_like(img)
    loss = torch.zeros(1, dtype=torch.float64, device=DEV)
    gs.gs_l1_loss_grad(img, tgt, views, dl, loss)
    torch.cuda.synchronize()
    L_ref, off = 0.0, 0
    for (w, h), a, b in zip(views.sizes, imgs, tgts):
        L, g = O.l1_loss_grad(a, b)
        L_ref += L
        np.testing.assert_allclose(np_(dl)[3 * off:3 * (off + w * h)], g.reshape(-1), rtol=1e-6)
        off += w * h
    np.testing.assert_allclose(float(np_(loss)[0]), L_ref, rtol=1e-6)


# ---------------------------------------------------------------------------
# degenerate batches
# ---------------------------------------------------------------------------

def _degenerate_workload(case, max_views):
    rng = np.random.default_rng(77)
    if case == "thin_views":
        # 1x1, 17x1 and 1x33 images: tiles that are almost all outside the image
        g = scenes.random_cloud(400, 1, 3, box=((-0.5, 0.5), (-0.5, 0.5), (2, 3)), log_scale_mu=-2.0)
        cams = [scenes.pinhole(1, 1, 2.0), scenes.pinhole(17, 1, 15.0), scenes.pinhole(1, 33, 30.0)]
    elif case == "max_views":
        # as many views as one batch takes, each a small perturbed pinhole
        g = scenes.random_cloud(600, 1, 4)
        cams = [scenes.perturb_pose(scenes.pinhole(24, 16, 20.0), rng) for _ in range(max_views)]
    elif case == "one_gaussian":
        g = scenes.random_cloud(1, 3, 5, box=((-0.1, 0.1), (-0.1, 0.1), (2.5, 3)), log_scale_mu=-1.5)
        cams = [scenes.pinhole(48, 40, 40.0)]
    else:   # opaque_stack: clamped alphas, every pixel terminating early
        g = scenes.random_cloud(300, 0, 6, box=((-0.3, 0.3), (-0.3, 0.3), (2, 4)), log_scale_mu=-1.0)
        g.opacity_logits[:] = 8.0
        cams = [scenes.pinhole(64, 48, 60.0)]
    targets = [np.zeros((3, c.height, c.width), np.float32) for c in cams]
    return scenes.Workload(f"degenerate_{case}", g, cams, targets, bg=(0.25, 0.5, 0.75))


@pytest.mark.parametrize("case", ["thin_views", "max_views", "one_gaussian", "opaque_stack"])
def test_degenerate_batches(gs, case):
    """Images, n_contrib and every gradient against the oracle on batches at
    the edges of the method: images a pixel wide, the largest view count a
    batch takes, a single Gaussian, and a stack of clamped (alpha = 0.99)
    splats under which every pixel stops early."""
    wl = _degenerate_workload(case, gs.GS_MAX_VIEWS)
    out, res = _grad_parity(gs, wl, seed=11)
    for v, r in enumerate(res["views"]):
        nc = np_(out["views"].split_maps(out["nc"])[v])
        m = ~r["mask"]
        np.testing.assert_array_equal(nc[m], r["n_contrib"][m])
    for v, r in enumerate(res["views"]):
        T = np_(out["views"].split_maps(out["T"])[v])
        m = ~r["mask"]
        np.testing.assert_allclose(T[m], r["T_final"][m], rtol=1e-3, atol=1e-7)
    if case == "opaque_stack":   # most pixels stop just before T would fall below 1e-4
        assert (np_(out["T"]) < 1e-3).mean() > 0.5


def test_empty_map_renders_background(gs):
    """No Gaussians at all: the image is the background, T = 1 and
    n_contrib = 0 everywhere, and the backward adds nothing to the pose
    gradient, or writes zero under GS_BWD_OVERWRITE (closed form; the oracle
    is not needed)."""
    from paper_2409_09295_amd.rasterizer import Rasterizer
    g0 = scenes.random_cloud(1, 0, 1)
    empty = scenes.GaussianMap(g0.means[:, :0].copy(), g0.log_scales[:, :0].copy(),
                               g0.quats[:, :0].copy(), g0.opacity_logits[:0].copy(),
                               g0.sh[:, :, :0].copy(), 0)
    cams = [scenes.pinhole(40, 30, 30.0), scenes.pinhole(17, 5, 12.0)]
    g = gs.Gaussians.from_map(empty)
    views = gs.Views(cams)
    rast = Rasterizer(g.n, views)
    bg = (0.25, 0.5, 0.75)
    img = np_(rast.forward(g, bg))
    P = views.n_pixels
    off = 0
    for (w, h) in views.sizes:
        blk = img[3 * off:3 * (off + w * h)].reshape(3, h, w)
        for ch in range(3):
            assert (blk[ch] == np.float32(bg[ch])).all()
        off += w * h
    assert (np_(rast.final_T) == 1.0).all() and (np_(rast.n_contrib) == 0).all()
    grads = gs.Grads.zeros_like(g, views.n_views)
    dl = torch.ones(3 * P, device=DEV)
    grads.xi.fill_(7.0)
    rast.backward(g, dl, grads, 0, bg)                      # accumulate: unchanged
    torch.cuda.synchronize()
    assert (np_(grads.xi) == 7.0).all()
    rast.backward(g, dl, grads, gs.GS_BWD_OVERWRITE, bg)    # overwrite: zero
    torch.cuda.synchronize()
    assert (np_(grads.xi) == 0.0).all()


def test_persistent_schedule_without_a_queue(gs):
    """The persistent schedule needs the bins' counters; without a queue it
    launches one workgroup per tile instead.  Both give the default
    schedule's image, final T and n_contrib bit for bit."""
    cams = BIN_CASES["ragged_multi_view"]
    sp = scenes.random_splats(3000, cams, seed=43)
    views, proj, bins, nk = _gpu_bins(gs, sp, cams)
    P = views.n_pixels
    N = sp.radius.shape[1]

    def render(b):
        out = [torch.empty(3 * P, device=DEV), torch.empty(P, device=DEV),
               torch.empty(P, dtype=torch.int32, device=DEV)]
        gs.gs_render_fwd(proj, N, b, views, (0.1, 0.2, 0.3), out[0], out[1], out[2])
        torch.cuda.synchronize()
        return out

    ref = render(bins)
    no_queue = gs.Bins(bins.keys, bins.values, bins.ranges, bins.n_keys, bins.capacity, bins.order, None)
    try:
        gs.gs_set_tuning(gs.GS_TUNE_FWD_SCHEDULE, gs.GS_SCHEDULE_PERSISTENT)
        for b in (bins, no_queue):
            for x, y in zip(render(b), ref):
                torch.testing.assert_close(x, y, rtol=0, atol=0)
        assert int(bins.queue.abs().sum().item()) == 0
    finally:
        gs.gs_set_tuning(gs.GS_TUNE_FWD_SCHEDULE, 0)
