"""The mapping loop (local stage, global stage with re-rendered past views,
pruning) over a synthetic keyframe sequence, and its overhead-memory ledger
(Sec. IV-B): the ledger's peak equals the essential buffers' bytes in closed
form (needs an MI355X)."""
import pytest

from paper_2409_09295_amd import gs

pytestmark = pytest.mark.gpu


def test_mapping_loop_overhead_matches_closed_form(gs):
    from paper_2409_09295_amd.mapping import run_sequence
    W, H, N, n_past, frames = 160, 120, 4, 4, 10
    out = run_sequence(W, H, frames, N, n_gauss=60000, seed=1, n_past=n_past,
                       log=lambda m: print(m, flush=True))
    px = W * H
    keyframes = N * 3 * px * 4
    poses = frames * 80
    # the largest temporary set: a global stage's re-rendered past views
    # (3 floats per pixel) and the blend state of window + past views
    # (8 bytes per pixel); it exceeds the initialiser's cost volume and the
    # local stage's blend state
    stage = n_past * 3 * px * 4 + (N + n_past) * px * 8
    init = gs.gs_cost_volume_workspace_size(N, H, W) + 4 * px
    assert stage > max(init, N * px * 8)
    expect = keyframes + poses + stage
    print(out["overhead_peak_MB"], expect / 1e6, out["peak_by_category_MB"], flush=True)
    assert abs(out["overhead_peak_MB"] * 1e6 - expect) < 1.0
    assert out["all_keyframes_MB"] > out["peak_by_category_MB"]["keyframes"]
    # the loop maps: the map renders the last keyframe, and the first (which
    # left the window long ago), at least 10 dB closer than an empty map does
    print(f"PSNR last {out['psnr_last']:.2f} dB (empty map {out['psnr_empty_last']:.2f}), first "
          f"{out['psnr_first']:.2f} dB (empty map {out['psnr_empty_first']:.2f}), "
          f"{out['map_gaussians']} Gaussians", flush=True)
    assert out["psnr_last"] > out["psnr_empty_last"] + 10.0
    assert out["psnr_first"] > out["psnr_empty_first"] + 10.0
    fr = [h["active_fraction"] for h in out["history"] if "active_fraction" in h]
    assert fr and max(fr) < 1.0
