"""A GEVO mapping loop over a keyframe sequence, with the paper's overhead-
memory accounting.

GEVO keeps only the keyframes of its current sliding window; past keyframes
are re-rendered from the map when the global stage needs them (Sec. I,
Sec. III-B2).  Its memory is reported as the map plus the overhead, the
inputs and temporaries that are essential to the algorithm, tracked where
they are created and freed (Sec. IV-B).  ``MappingLoop`` runs that loop on
the library's kernels and registers every essential buffer in the native
ledger (``gs_mem_*``):

    keyframes       the window's full-resolution RGB images (float32 on the
                    device, as the kernels read them)
    poses           the camera record of every keyframe (past poses are kept
                    for the consistency loss)
    init            the initialiser's cost volume (Eq. 1) and depth image,
                    while a new keyframe is initialised
    render_targets  the re-rendered past views of E_pc during a global stage
    blend_state     per-pixel final transmittance and last-splat index
                    between forward and backward, while a stage runs
    map, optimiser  the map and its Adam moments (not overhead)

Per new keyframe (every frame is a keyframe here; the paper's keyframe
selection belongs to tracking): the plain initialiser proposes Gaussians
from the window's cost volume, the local stage optimises them on the window
(E_pho + E_iso, Eq. 2), and the global stage merges them into the map
(selection by rendering error, E_pc on past views, insertion at opacity
0.2, selective optimisation, pruning; Eq. 3).  Poses come from the input
(tracking is not part of this loop) and stay fixed.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional

import numpy as np
import torch

from . import gs, scenes
from .global_stage import ISO_WEIGHT, GlobalStage, prune
from .initnet import learned_depth, plain_depth, propose
from .replay import DEFAULT_LR, BatchedStep

Y00 = 0.28209479177387814   # degree-0 real spherical harmonic

# Step sizes of the mapping stages: a map grown from a few hundred inserted
# Gaussians needs faster opacity and scale changes than refining a dense one.
MAPPING_LR = dict(DEFAULT_LR, opacity_logits=0.1, means=1e-3, log_scales=1e-2)


def _map_bytes(g: gs.Gaussians) -> int:
    return sum(t.numel() * t.element_size() for t in g.tensors())


class MappingLoop:
    def __init__(self, width: int, height: int, fx: float, *, window: int = 8, n_past: int = 4,
                 stride: int = 8, local_iters: int = 60, global_iters: int = 100,
                 active_quantile: float = 0.85, sh_degree: int = 0, seed: int = 0,
                 lrs: Optional[Dict[str, float]] = None, init_net=None, device="cuda"):
        self.W, self.H, self.fx = width, height, fx
        self.N, self.n_past, self.stride = window, n_past, stride
        self.local_iters, self.global_iters = local_iters, global_iters
        self.q = active_quantile
        self.lrs = dict(MAPPING_LR) if lrs is None else lrs
        self.init_net = init_net          # learned initialiser (initnet.UNet) or None
        self.sh_degree = sh_degree
        self.device = device
        self.rng = np.random.default_rng(seed)
        self.window: List[dict] = []          # {"image", "cam", "track"}
        self.poses: List[scenes.Camera] = []
        self.pose_tracks: List[gs.Tracked] = []
        self.map: Optional[gs.Gaussians] = None
        self.map_track: Optional[gs.Tracked] = None
        self.history: List[Dict] = []

    # -- helpers -------------------------------------------------------------
    def _set_map(self, g: gs.Gaussians):
        if self.map_track is not None:
            self.map_track.release()
        self.map = g
        self.map_track = gs.Tracked(gs.GS_MEM_MAP, _map_bytes(g))

    def _window_tensor(self) -> torch.Tensor:
        return torch.stack([k["image"] for k in self.window])

    def _initialise(self) -> gs.Gaussians:
        """New Gaussians for the newest keyframe, one per stride x stride block
        with a depth, coloured from the keyframe, isotropic, opacity 0.5.  The
        depth (and scale) comes from the learned initialiser when one is
        given and its output is finite (Sec. III-A1), else from the window's
        cost volume (Eq. 1, winner-take-all)."""
        kfs = self._window_tensor()
        cams = [k["cam"] for k in self.window]
        k, _, H, W = kfs.shape
        lsmap = None
        if self.init_net is not None:
            depth, lsmap, used = learned_depth(self.init_net, kfs, cams, self.device)
            cv = gs.Tracked(gs.GS_MEM_INIT, self.init_net.buffer_bytes())
            self.init_source = "network" if used else "plain"
        else:
            cv = gs.Tracked(gs.GS_MEM_INIT, gs.gs_cost_volume_workspace_size(k, H, W) + 4 * H * W)
            depth = plain_depth(kfs, cams, self.device)
            self.init_source = "plain"
        means, ls = propose(depth, cams[-1], self.stride, lsmap)
        cv.release()
        m = means.shape[1]
        img = self.window[-1]["image"]
        cam = cams[-1]
        # colour at the proposing pixels (the ray through the mean)
        R = torch.as_tensor(np.asarray(cam.R), dtype=torch.float32, device=self.device)
        t = torch.as_tensor(np.asarray(cam.t), dtype=torch.float32, device=self.device)
        pc = R @ means + t[:, None]
        u = (cam.fx * pc[0] / pc[2] + cam.cx).long().clamp(0, W - 1)
        v = (cam.fy * pc[1] / pc[2] + cam.cy).long().clamp(0, H - 1)
        rgb = img[:, v, u]                                           # (3, m)
        K = (self.sh_degree + 1) ** 2
        sh = torch.zeros(3, K, m, dtype=torch.float32, device=self.device)
        sh[:, 0, :] = (rgb - 0.5) / Y00
        quats = torch.zeros(4, m, dtype=torch.float32, device=self.device)
        quats[0] = 1.0
        return gs.Gaussians(means.contiguous(), ls.contiguous(), quats,
                            torch.zeros(m, dtype=torch.float32, device=self.device), sh,
                            self.sh_degree)

    def _local_stage(self, local: gs.Gaussians) -> gs.Gaussians:
        """E_pho + E_iso on the window, all of the local map optimised (Eq. 2)."""
        views = gs.Views([k["cam"] for k in self.window], self.device)
        targets = self._window_tensor().reshape(-1)
        blend = gs.Tracked(gs.GS_MEM_BLEND_STATE, 8 * views.n_pixels)
        opt = gs.Tracked(gs.GS_MEM_OPTIMISER, 2 * _map_bytes(local))
        step = BatchedStep(local, views, targets, lrs=self.lrs, iso_weight=ISO_WEIGHT, pose=False)
        for _ in range(self.local_iters):
            step.step_checked()
        del step
        blend.release()
        opt.release()
        return local

    def _global_stage(self, local: gs.Gaussians) -> Dict:
        wcams = [k["cam"] for k in self.window]
        # past poses outside the window, sampled uniformly (Sec. III-B2)
        n_old = len(self.poses) - len(self.window)
        past = []
        if n_old > 0 and self.n_past > 0:
            idx = self.rng.integers(0, n_old, self.n_past)
            past = [self.poses[i] for i in idx]
        kfs = self._window_tensor().reshape(-1)
        P_all = sum(c.width * c.height for c in wcams + past)
        targets_t = gs.Tracked(gs.GS_MEM_RENDER_TARGETS, 12 * sum(c.width * c.height for c in past))
        blend = gs.Tracked(gs.GS_MEM_BLEND_STATE, 8 * P_all)
        # the threshold: the active_quantile of the Gaussians' largest errors
        # (the paper does not state its value)
        stage = GlobalStage(self.map, local, wcams, kfs, past, None, eps_quantile=self.q,
                            lrs=self.lrs, pose_lr=None)
        eps = stage.eps
        opt = gs.Tracked(gs.GS_MEM_OPTIMISER, 2 * _map_bytes(stage.map))
        stage.iterate(self.global_iters)
        active = stage.active_fraction()
        new_map, keep = stage.finish()
        n_before = stage.map.n
        del stage
        targets_t.release()
        blend.release()
        opt.release()
        self._set_map(new_map)
        return {"eps": eps, "active_fraction": active, "before_prune": n_before, "after_prune": new_map.n}

    # -- public --------------------------------------------------------------
    def add_keyframe(self, image: torch.Tensor, cam: scenes.Camera) -> Dict:
        """image: (3, H, W) float32 on the device."""
        kf = {"image": image.contiguous(), "cam": cam,
              "track": gs.Tracked(gs.GS_MEM_KEYFRAMES, image)}
        self.window.append(kf)
        self.poses.append(cam)
        self.pose_tracks.append(gs.Tracked(gs.GS_MEM_POSES, 80))
        while len(self.window) > self.N:              # the window W_t holds N keyframes
            self.window.pop(0)["track"].release()
        info: Dict = {"keyframe": len(self.poses) - 1}
        if len(self.window) >= 2:
            local = self._local_stage(self._initialise())
            info["new_gaussians"] = local.n
            info["init"] = self.init_source
            if self.map is None:
                pruned, _ = prune(local)
                self._set_map(pruned)
            else:
                info.update(self._global_stage(local))
        info["map_gaussians"] = 0 if self.map is None else self.map.n
        self.history.append(info)
        return info

    def render(self, cam: scenes.Camera) -> torch.Tensor:
        from .rasterizer import Rasterizer
        r = Rasterizer(self.map.n, gs.Views([cam], self.device))
        return r.forward(self.map).view(3, cam.height, cam.width).clone()


def local_stage_psnr(frames: List[torch.Tensor], cams: List[scenes.Camera], init_net=None,
                     iters: int = 30, stride: int = 8, device="cuda") -> float:
    """The initialisers compared on one window: new Gaussians for the newest
    keyframe from `init_net` (or the plain initialiser when None), then
    `iters` local-stage iterations (E_pho + E_iso on the window, Eq. 2); the
    PSNR of that local map on the newest keyframe."""
    loop = MappingLoop(cams[0].width, cams[0].height, cams[0].fx, window=len(frames), stride=stride,
                       local_iters=iters, init_net=init_net, device=device)
    for f, c in zip(frames, cams):
        loop.window.append({"image": f.contiguous(), "cam": c,
                            "track": gs.Tracked(gs.GS_MEM_KEYFRAMES, f)})
    local = loop._local_stage(loop._initialise())
    loop.map = local
    out = psnr(loop.render(cams[-1]), frames[-1])
    for k in loop.window:
        k["track"].release()
    return out


def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    mse = float(((a.clamp(0, 1) - b) ** 2).mean().item())
    return 10.0 * math.log10(1.0 / max(mse, 1e-12))


def run_sequence(width: int, height: int, n_frames: int, window: int, n_gauss: int = 200000,
                 seed: int = 0, device="cuda", log=None, **kw) -> Dict:
    """The loop over a procedural-room trajectory whose frames are renders of
    a ground-truth room map; returns the ledger's overhead figures and the
    final map's PSNR on the last frame, on the first mapped one (a past
    view) and averaged over every mapped frame."""
    from .initnet import trajectory_cams
    from .rasterizer import Rasterizer
    gt, boxes = scenes.procedural_room(n_gauss, seed, sh_degree=0)
    cams = trajectory_cams(n_frames, seed + 7, boxes, width, height)
    g = gs.Gaussians.from_map(gt, device)
    gs.gs_mem_reset_peaks()
    base = gs.gs_mem_report()
    loop = MappingLoop(width, height, cams[0].fx, window=window, device=device, seed=seed, **kw)
    frames = []
    for i, c in enumerate(cams):
        r = Rasterizer(g.n, gs.Views([c], device))
        img = r.forward(g).view(3, height, width).clone()
        frames.append(img)
        info = loop.add_keyframe(img, c)
        if log:
            log(f"keyframe {i}: {info}")
    rep = gs.gs_mem_report()
    out = {
        "frames": n_frames, "window": window, "resolution": [width, height],
        "overhead_peak_MB": (rep["overhead_peak"] - base["overhead_current"]) / 1e6,
        "peak_by_category_MB": {k: (v - base["current"][k]) / 1e6 for k, v in rep["peak"].items()},
        "map_gaussians": loop.map.n,
        "map_MB": _map_bytes(loop.map) / 1e6,
        "all_keyframes_MB": n_frames * 3 * width * height * 4 / 1e6,
        "psnr_mean": float(np.mean([psnr(loop.render(c), f) for c, f in zip(cams[1:], frames[1:])])),
        "psnr_last": psnr(loop.render(cams[-1]), frames[-1]),
        "psnr_first": psnr(loop.render(cams[1]), frames[1]),
        "psnr_empty_last": psnr(torch.zeros_like(frames[-1]), frames[-1]),
        "psnr_empty_first": psnr(torch.zeros_like(frames[1]), frames[1]),
        "history": loop.history,
    }
    return out
