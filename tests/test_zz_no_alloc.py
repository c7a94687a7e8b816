"""The allocation-free entry point gs_render_fwd_l1_noalloc against
gs_render_fwd_l1 with a caller workspace, through the C ABI: two calls in a
row, the second on a smaller batch (the static scratch keeps the first
call's shares beyond the second's tiles), results equal bit for bit; a batch
above the scratch's tile limit is refused before any work (needs an
MI355X)."""
import numpy as np
import pytest
import torch

from paper_2409_09295_amd import scenes

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _binned(gs, cams, n, seed):
    sp = scenes.random_splats(n, cams, seed=seed)
    views = gs.Views(cams)
    proj = gs.Projected.from_splats(sp)
    V, N = sp.radius.shape
    cap = 64 * N * V + 1024
    bins = gs.Bins.empty(cap, views.n_tiles)
    ws = gs.workspace(gs.gs_bin_sort_workspace_size(N, views, cap))
    gs.gs_bin_sort(proj, N, views, bins, ws, sync=True)
    return views, proj, bins, N


def _outputs(views):
    P = views.n_pixels
    return [torch.full((3 * P,), np.nan, device=DEV), torch.full((P,), np.nan, device=DEV),
            torch.zeros(P, dtype=torch.int32, device=DEV), torch.full((3 * P,), np.nan, device=DEV),
            torch.zeros(1, dtype=torch.float64, device=DEV)]


@pytest.mark.parametrize("ppl", [1, 4])
def test_noalloc_matches_workspace_call(gs, ppl):
    gs.gs_set_tuning(gs.GS_TUNE_FWD_PIXELS_PER_LANE, ppl)
    try:
        batches = [
            # 4 views up to 1200x680: 3,433 tiles
            [scenes.pinhole(100, 70, 80.0), scenes.pinhole(320, 240, 300.0),
             scenes.pinhole(48, 40, 40.0), scenes.pinhole(1200, 680, 984.0)],
            # then a smaller batch: one 160x120 view, 80 tiles
            [scenes.pinhole(160, 120, 150.0)],
        ]
        for k, cams in enumerate(batches):
            views, proj, bins, N = _binned(gs, cams, 3000, seed=60 + k)
            rng = np.random.default_rng(61 + k)
            target = torch.from_numpy(rng.random(3 * views.n_pixels).astype(np.float32)).to(DEV)
            bg = (0.1, 0.3, 0.2)
            ref = _outputs(views)
            ws = gs.workspace(gs.gs_render_fwd_l1_workspace_size(views))
            gs.gs_render_fwd_l1(proj, N, bins, views, bg, ref[0], ref[1], ref[2], target, ref[3], ref[4], ws)
            got = _outputs(views)
            gs.gs_render_fwd_l1_noalloc(proj, N, bins, views, bg, got[0], got[1], got[2], target, got[3],
                                        got[4])
            torch.cuda.synchronize()
            print(f"call {k}: {views.n_tiles} tiles, loss {float(got[4].item()):.6f}", flush=True)
            for a, b in zip(got, ref):
                torch.testing.assert_close(a, b, rtol=0, atol=0)
    finally:
        gs.gs_set_tuning(gs.GS_TUNE_FWD_PIXELS_PER_LANE, 0)


def test_noalloc_rejects_batches_above_its_scratch(gs):
    """One 16384x16384 view has 1,048,576 tiles: refused with
    GS_ERR_CAPACITY by the host-side check (no buffer is touched)."""
    views = gs.Views([scenes.pinhole(16384, 16384, 10000.0)])
    assert views.n_tiles > gs.GS_NOALLOC_MAX_TILES
    proj = gs.Projected.empty(1, 1)
    bins = gs.Bins.empty(1, 1)
    one = torch.zeros(3, device=DEV)
    with pytest.raises(gs.GsError) as ei:
        gs.gs_render_fwd_l1_noalloc(proj, 1, bins, views, None, one, one, one.view(torch.int32), one,
                                    one, None)
    assert ei.value.status == gs.GS_ERR_CAPACITY
    assert b"tile shares" in gs.lib().gs_last_error()
