"""The global mapping stage of GEVO (Sec. III-B2) on the GPU.

Given the previous global map M_{t-1}, the local map M~_t optimised on the
current keyframe window W_t, the window's keyframes and poses, and a few past
camera poses, one stage runs

    selection    E_k(g) of every Gaussian of M_{t-1} in every window view
                 (gs_render_error on renders of M_{t-1}); E_t = {g : max_k
                 E_k(g) > eps} (gs_active_set)
    targets      R(M_{t-1}, T_{k_l}) at the past poses, rendered once and held
                 fixed (the stop-gradient targets of E_pc)
    insertion    M'_t = M_{t-1} united with M~_t, whose opacity is lowered to
                 0.2 (gs_concat); the active set A_t = E_t united with M~_t
    optimisation iterations of E_pho (window) + E_pc (past views) + E_iso over
                 A_t and the window poses (Eq. 3): one captured HIP graph per
                 iteration (batched replay with masked Adam, the isotropic
                 regulariser and the pose step)
    pruning      Gaussians of opacity below 0.7 are removed (gs_prune_mask,
                 gs_compact); the occupancy rule of the paper needs its free-
                 space Gaussian mixture and is not part of this stage

and returns the new global map M_t.  Every arithmetic step runs in the
library's kernels; this module sequences calls and owns buffers.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence

import torch

from . import gs
from .rasterizer import Rasterizer
from .replay import BETA1, BETA2, DEFAULT_LR, EPS, GROUPS, BatchedStep

INSERT_OPACITY = 0.2
PRUNE_OPACITY = 0.7
ISO_WEIGHT = 10.0


def _logit(p: float) -> float:
    return math.log(p / (1.0 - p))


def _components(g: gs.Gaussians):
    K = (g.sh_degree + 1) ** 2
    return (3, 3, 4, 1, 3 * K)


def insert(global_map: gs.Gaussians, local_map: gs.Gaussians,
           opacity: float = INSERT_OPACITY) -> gs.Gaussians:
    """M'_t = M_{t-1} followed by M~_t, the latter at opacity ``opacity``."""
    if global_map.sh_degree != local_map.sh_degree:
        raise ValueError("both maps need the same SH degree")
    na, nb = global_map.n, local_map.n
    dev = global_map.means.device
    out = []
    arrays = []
    for k, (a, b, c) in enumerate(zip(global_map.tensors(), local_map.tensors(),
                                      _components(global_map))):
        shape = a.shape[:-1] + (na + nb,)
        dst = torch.empty(shape, dtype=torch.float32, device=dev)
        out.append(dst)
        if k == 3:   # opacity logits of the inserted Gaussians: a constant
            arrays.append((a.reshape(-1), None, dst.reshape(-1), c, _logit(opacity)))
        else:
            arrays.append((a.reshape(-1), b.reshape(-1), dst.reshape(-1), c, 0.0))
    gs.gs_concat(arrays, na, nb)
    return gs.Gaussians(*out, global_map.sh_degree)


def prune(g: gs.Gaussians, min_opacity: float = PRUNE_OPACITY):
    """Removes Gaussians of opacity below ``min_opacity``; returns the
    compacted map and the keep mask (one host read of the kept count)."""
    dev = g.means.device
    keep = torch.empty(g.n, dtype=torch.uint8, device=dev)
    gs.gs_prune_mask(g.opacity_logits, min_opacity, keep)
    dsts = [torch.empty_like(t) for t in g.tensors()]
    n_kept = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = gs.workspace(gs.gs_compact_workspace_size(g.n), dev)
    gs.gs_compact([(t.reshape(-1), d.reshape(-1), c)
                   for t, d, c in zip(g.tensors(), dsts, _components(g))], g.n, keep, n_kept, ws)
    m = int(n_kept.item())
    out = [d.reshape(-1)[:c * m].reshape(t.shape[:-1] + (m,)).clone()
           for t, d, c in zip(g.tensors(), dsts, _components(g))]
    return gs.Gaussians(*out, g.sh_degree), keep


class GlobalStage:
    """One global stage over a window.

    window_cams, window_images: the keyframes of W_t (images packed
    [V][3][H][W] float32 on the device); past_cams: the past poses T_{k_l}
    of E_pc; eps: threshold of the rendering error, or None to take the
    eps_quantile quantile of the Gaussians' largest nonzero errors (the paper
    does not state its threshold).  lrs: per-group Adam learning rates;
    pose_lr: (translation, rotation) rates of the window poses (None: poses
    fixed)."""

    def __init__(self, global_map: gs.Gaussians, local_map: gs.Gaussians, window_cams,
                 window_images: torch.Tensor, past_cams, eps: Optional[float], *,
                 eps_quantile: float = 0.85,
                 lrs: Optional[Dict[str, float]] = None, iso_weight: float = ISO_WEIGHT,
                 pose_lr=(1e-4, 1e-4), bg: Sequence[float] = (0.0, 0.0, 0.0),
                 insert_opacity: float = INSERT_OPACITY, prune_opacity: float = PRUNE_OPACITY,
                 use_graph: bool = True):
        self.prev = global_map
        self.local = local_map
        self.window_cams = list(window_cams)
        self.past_cams = list(past_cams)
        self.bg = tuple(bg)
        self.prune_opacity = prune_opacity
        dev = global_map.means.device
        nw, npast = len(self.window_cams), len(self.past_cams)
        # selection: E_k(g) of M_{t-1} on the window
        wviews = gs.Views(self.window_cams, dev)
        r = Rasterizer(global_map.n, wviews)
        r.forward(global_map, self.bg)
        self.err = torch.empty(nw, global_map.n, dtype=torch.float32, device=dev)
        gs.gs_render_error(r.proj, global_map.n, r.bins, wviews, r.image, window_images,
                           r.n_contrib, self.err)
        if eps is None:
            emax = self.err.max(dim=0).values
            pos = emax[emax > 0]
            eps = float(torch.quantile(pos, eps_quantile).item()) if pos.numel() else 0.0
        self.eps = float(eps)
        n = global_map.n + local_map.n
        self.active = torch.ones(n, dtype=torch.uint8, device=dev)   # inserted ones stay on
        self.n_selected = torch.zeros(1, dtype=torch.int32, device=dev)
        gs.gs_active_set(self.err, global_map.n, nw, self.eps, self.active[:global_map.n],
                         n_active=self.n_selected)
        del r
        # stop-gradient targets of E_pc: renders of M_{t-1} at the past poses
        targets = [window_images.reshape(-1)]
        if npast:
            pviews = gs.Views(self.past_cams, dev)
            rp = Rasterizer(global_map.n, pviews)
            targets.append(rp.forward(global_map, self.bg).clone())
            del rp
        self.targets = torch.cat(targets)
        # insertion, then the batched step over window + past views
        self.map = insert(global_map, local_map, insert_opacity)
        self.views = gs.Views(self.window_cams + self.past_cams, dev)
        self.step_ = BatchedStep(self.map, self.views, self.targets, lrs=lrs or DEFAULT_LR, bg=bg,
                                 active=self.active, iso_weight=iso_weight, use_graph=use_graph,
                                 pose=pose_lr is not None)
        self.pose_lr = pose_lr
        if pose_lr is not None:
            V = self.views.n_views
            self.pose_m = torch.zeros(V, 6, dtype=torch.float32, device=dev)
            self.pose_v = torch.zeros(V, 6, dtype=torch.float32, device=dev)
            self.pose_step = torch.zeros(1, dtype=torch.int32, device=dev)
            mask = torch.zeros(V, dtype=torch.uint8, device=dev)
            mask[:nw] = 1                                  # past poses are fixed
            self.pose_mask = mask
            self.step_.post_body = self._pose_update
            self.step_.extra_state = [self.views.dev, self.pose_m, self.pose_v, self.pose_step]

    def _pose_update(self):
        gs.gs_pose_adam_step(self.views, self.step_.grads.xi, self.pose_m, self.pose_v,
                             self.pose_step, self.pose_lr[0], self.pose_lr[1], BETA1, BETA2, EPS,
                             self.pose_mask)

    def iterate(self, iters: int):
        for _ in range(iters):
            self.step_.step()

    def active_fraction(self) -> float:
        return float(self.active.float().mean().item())

    def finish(self):
        """Pruning; returns (M_t, keep mask over M'_t)."""
        return prune(self.map, self.prune_opacity)
