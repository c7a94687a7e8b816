"""Batched replay of keyframe views, and the plain per-view path.

GEVO re-renders past keyframes from the map instead of storing them, and the
global mapping stage optimises against several such views at once: the
current window plus four past viewpoints whose targets are renders of the
previous map (Sec. III-B2, the E_pc term and Eq. 3).  ``BatchedStep`` runs
one mapping iteration over a whole batch of views of possibly different
sizes:

    gs_preprocess    every Gaussian projected into all V views (map read once)
    gs_bin_sort      one sort over the global tile ids of all views
                     (capacity mode: no host synchronisation)
    gs_render_fwd    one compositing grid over every tile of every view
    gs_l1_loss_grad  photometric L1 gradient per view
    gs_render_bwd    one reverse-walk grid, then the projection backward
                     summed over views (overwrite mode) plus pose tangents
    gs_adam_step_dev one capture-safe Adam update per parameter group,
                     skipped on binning overflow

captured once as a HIP graph and replayed with a single launch.  The key
capacity is fixed at capture; ``step_checked`` reads the device key count
after a replay and, on overflow, grows the capacity, re-captures and redoes
the step (the guarded optimiser made the overflowed replay a no-op).

``PlainStep`` is the reference point: the same kernels at V = 1, called once
per view with the synchronous key-count readback, gradients accumulated over
views, then the same Adam updates.
"""
from __future__ import annotations

import gc
from typing import Dict, Optional, Sequence

import torch

from . import gs
from .rasterizer import Rasterizer

GROUPS = ("means", "log_scales", "quats", "opacity_logits", "sh")
DEFAULT_LR: Dict[str, float] = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3,
                                    opacity_logits=5e-2, sh=2.5e-3)
BETA1, BETA2, EPS = 0.9, 0.999, 1e-15


class _AdamState:
    def __init__(self, g: gs.Gaussians, lrs: Dict[str, float]):
        self.params = g.tensors()
        self.m = [torch.zeros_like(t) for t in self.params]
        self.v = [torch.zeros_like(t) for t in self.params]
        self.lrs = [float(lrs[k]) for k in GROUPS]
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=g.means.device)

    def snapshot(self):
        return [t.clone() for t in self.params + self.m + self.v + [self.step_dev]]

    def restore(self, snap):
        for dst, src in zip(self.params + self.m + self.v + [self.step_dev], snap):
            dst.copy_(src)

    def apply(self, grads: gs.Grads, guard_n_keys=None, guard_capacity: int = 0,
              active: Optional[torch.Tensor] = None):
        """One Adam step of every group in a single launch (graph-capture safe);
        with ``active`` (uint8 per Gaussian) only the active Gaussians move."""
        gl = [grads.means, grads.log_scales, grads.quats, grads.opacity_logits, grads.sh]
        key = tuple(t.data_ptr() for t in gl)
        if getattr(self, "_groups_key", None) != key:
            self._groups = gs.adam_groups(list(zip(self.params, gl, self.m, self.v, self.lrs)))
            self._groups_key = key
        if active is None:
            gs.gs_adam_step_groups_dev(self._groups, BETA1, BETA2, EPS, self.step_dev,
                                       guard_n_keys=guard_n_keys, guard_capacity=guard_capacity)
        else:
            gs.gs_adam_step_groups_masked_dev(self._groups, BETA1, BETA2, EPS, self.step_dev, active,
                                              active.numel(), guard_n_keys=guard_n_keys,
                                              guard_capacity=guard_capacity)


class BatchedStep:
    def __init__(self, g: gs.Gaussians, views: gs.Views, targets: torch.Tensor, *,
                 lrs: Optional[Dict[str, float]] = None, capacity: Optional[int] = None,
                 headroom: float = 1.25, bg: Sequence[float] = (0.0, 0.0, 0.0),
                 optimize: bool = True, pose: bool = True, use_graph: bool = True,
                 active: Optional[torch.Tensor] = None, iso_weight: float = 0.0):
        """active: optional uint8 per-Gaussian mask; only active Gaussians are
        updated (the selective optimisation of the global stage).  iso_weight:
        weight of the isotropic regulariser added to the photometric loss (0:
        none)."""
        self.g, self.views, self.bg = g, views, tuple(bg)
        self.active = active
        self.iso_weight = float(iso_weight)
        self.n = g.n
        self.targets = targets
        self.optimize, self.pose, self.use_graph = optimize, pose, use_graph
        self.headroom = headroom
        V, dev = views.n_views, g.means.device
        P = views.n_pixels
        self.n_pixels = P
        self.proj = gs.Projected.empty(V, self.n, dev)
        self.grads = gs.Grads.zeros_like(g, V)
        self.image = torch.zeros(3 * P, dtype=torch.float32, device=dev)
        self.final_T = torch.zeros(P, dtype=torch.float32, device=dev)
        self.n_contrib = torch.zeros(P, dtype=torch.int32, device=dev)
        self.dL = torch.zeros(3 * P, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.iso_loss = torch.zeros(1, dtype=torch.float64, device=dev)
        # handed to every backward as clear (GS_BWD_KEEP_CLEAR): zeroed once here
        self.bwd_ws = gs.workspace(gs.gs_render_bwd_workspace_size(self.n, views), dev).zero_()
        self.l1_ws = gs.workspace(gs.gs_render_fwd_l1_workspace_size(views), dev)
        self.adam = _AdamState(g, lrs or DEFAULT_LR)
        self.n_tiles = views.n_tiles
        if capacity is None:
            capacity = self.measure_keys()
            capacity = int(capacity * headroom) + 4096
        self._alloc_bins(capacity)
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.recaptures = 0
        # optional work appended to every iteration (inside the graph), and
        # device state it modifies, restored after the warm-up of a capture
        self.post_body = None
        self.extra_state = []

    # -- buffers ------------------------------------------------------------
    def _alloc_bins(self, capacity: int):
        capacity = int(min(capacity, 0xFFFFFFFF))
        dev = self.g.means.device
        self.bins = gs.Bins.empty(capacity, self.n_tiles, dev, keys=False)   # never read here
        self.sort_ws = gs.workspace(gs.gs_bin_sort_workspace_size(self.n, self.views, capacity), dev)

    def measure_keys(self) -> int:
        """Key count of the current map (one synchronous binning pass)."""
        gs.gs_preprocess(self.g, self.views, self.proj)
        probe = gs.Bins.empty(1, self.n_tiles, self.g.means.device, keys=False)
        ws = gs.workspace(gs.gs_bin_sort_workspace_size(self.n, self.views, 1), self.g.means.device)
        try:
            return int(gs.gs_bin_sort(self.proj, self.n, self.views, probe, ws, sync=True))
        except gs.GsError as e:
            if e.status != gs.GS_ERR_CAPACITY:
                raise
            return int(e.required)

    # -- one iteration ------------------------------------------------------
    def _body(self):
        gs.gs_preprocess(self.g, self.views, self.proj)
        gs.gs_bin_sort(self.proj, self.n, self.views, self.bins, self.sort_ws, sync=False)
        gs.gs_render_fwd_l1(self.proj, self.n, self.bins, self.views, self.bg, self.image,
                            self.final_T, self.n_contrib, self.targets, self.dL, self.loss,
                            self.l1_ws)
        flags = (gs.GS_BWD_OVERWRITE | gs.GS_BWD_KEEP_CLEAR
                 | (0 if self.pose else gs.GS_BWD_NO_POSE))
        gs.gs_render_bwd(self.g, self.proj, self.bins, self.views, self.bg, self.dL, self.final_T,
                         self.n_contrib, self.grads, flags, self.bwd_ws)
        if self.iso_weight:
            gs.gs_iso_loss_grad(self.g.log_scales, self.iso_weight, self.grads.log_scales,
                                self.iso_loss)
        if self.optimize:
            self.adam.apply(self.grads, self.bins.n_keys, self.bins.capacity, self.active)
        if self.post_body is not None:
            self.post_body()

    def capture(self):
        """Warm up eagerly (state restored afterwards), then capture one step."""
        snap = self.adam.snapshot()
        extra = [t.clone() for t in self.extra_state]
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._body()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.adam.restore(snap)
        for dst, src in zip(self.extra_state, extra):
            dst.copy_(src)
        torch.cuda.synchronize()
        # Collect unreachable cycles now: a dead step found by the collector
        # during the capture would free its graph's memory pool, and freeing
        # device memory is not allowed while a stream is capturing.
        # The collector stays off during the capture, so that no cycle found
        # mid-capture can free memory either.
        gc.collect()
        enabled = gc.isenabled()
        gc.disable()
        try:
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph):
                self._body()
        finally:
            if enabled:
                gc.enable()
        torch.cuda.synchronize()

    def step(self):
        if self.use_graph:
            if self.graph is None:
                self.capture()
            self.graph.replay()
        else:
            self._body()

    def key_count(self) -> int:
        return int(self.bins.n_keys.cpu().view(torch.int32).item()) & 0xFFFFFFFF

    def overflowed(self) -> bool:
        return self.key_count() > self.bins.capacity

    def step_checked(self) -> bool:
        """One step; on binning overflow grow, re-capture and redo.  Returns
        True if a re-capture happened."""
        self.step()
        if not self.overflowed():
            return False
        need = self.key_count()
        self._alloc_bins(int(need * self.headroom) + 4096)
        self.graph = None
        self.recaptures += 1
        self.step()
        return True

    def images(self):
        return self.views.split_images(self.image)


class PlainStep:
    """Per-view reference path: V calls of the V = 1 pipeline (each with its
    key-count readback), gradients accumulated over views, then Adam."""

    def __init__(self, g: gs.Gaussians, cams, targets: Sequence[torch.Tensor], *,
                 lrs: Optional[Dict[str, float]] = None, bg: Sequence[float] = (0.0, 0.0, 0.0),
                 optimize: bool = True, pose: bool = True):
        self.g, self.bg = g, tuple(bg)
        self.targets = [t.reshape(-1).contiguous() for t in targets]
        self.views = [gs.Views([c]) for c in cams]
        self.rasts = [Rasterizer(g.n, v) for v in self.views]
        self.grads = gs.Grads.zeros_like(g, 1)
        self.xi = torch.zeros(len(cams), 6, dtype=torch.float32, device=g.means.device)
        self.dL = [torch.empty_like(t) for t in self.targets]
        self.adam = _AdamState(g, lrs or DEFAULT_LR)
        self.optimize, self.pose = optimize, pose

    def step(self):
        self.xi.zero_()
        for k, (v, r, t, dl) in enumerate(zip(self.views, self.rasts, self.targets, self.dL)):
            r.forward_l1(self.g, t, dl, bg=self.bg)
            grads = gs.Grads(self.grads.means, self.grads.log_scales, self.grads.quats,
                             self.grads.opacity_logits, self.grads.sh, self.xi[k:k + 1])
            flags = (gs.GS_BWD_OVERWRITE if k == 0 else 0) | (0 if self.pose else gs.GS_BWD_NO_POSE)
            r.backward(self.g, dl, grads, flags, self.bg)
        if self.optimize:
            self.adam.apply(self.grads)
