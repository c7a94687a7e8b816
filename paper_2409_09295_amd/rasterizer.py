"""Plain (per-call) rendering path over the C ABI.

``Rasterizer`` owns the device buffers of one view batch (projected splats,
tile keys, workspaces, images) and sequences the entry points:

    forward:  gs_preprocess -> gs_bin_sort (one 4-byte key-count readback) ->
              gs_render_fwd
    backward: gs_render_bwd (per-splat screen-space gradients, then the
              projection backward and pose partials)

The key capacity grows geometrically when gs_bin_sort reports
GS_ERR_CAPACITY, so the steady state issues exactly one synchronisation
(the key count) per forward.
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import gs


class Rasterizer:
    def __init__(self, n: int, views: gs.Views, capacity: Optional[int] = None, device="cuda",
                 with_depth: bool = False):
        self.n = int(n)
        self.views = views
        self.device = device
        V = views.n_views
        self.proj = gs.Projected.empty(V, self.n, device)
        self.n_tiles = views.n_tiles
        self.n_pixels = views.n_pixels
        cap = capacity if capacity is not None else max(1 << 16, 4 * self.n * V)
        self._alloc_bins(cap)
        self.image = torch.empty(3 * self.n_pixels, dtype=torch.float32, device=device)
        self.final_T = torch.empty(self.n_pixels, dtype=torch.float32, device=device)
        self.n_contrib = torch.empty(self.n_pixels, dtype=torch.int32, device=device)
        self.depth = torch.empty(self.n_pixels, dtype=torch.float32, device=device) if with_depth else None
        self.bwd_ws = gs.workspace(gs.gs_render_bwd_workspace_size(self.n, views), device)
        self.n_keys = 0

    def _alloc_bins(self, capacity: int):
        capacity = int(min(capacity, 0xFFFFFFFF))
        self.bins = gs.Bins.empty(capacity, self.n_tiles, self.device, keys=False)   # never read here
        self.sort_ws = gs.workspace(gs.gs_bin_sort_workspace_size(self.n, self.views, capacity), self.device)

    def _project_and_bin(self, g: gs.Gaussians):
        if g.n != self.n:
            raise ValueError("Gaussian count changed")
        gs.gs_preprocess(g, self.views, self.proj)
        while True:
            try:
                self.n_keys = gs.gs_bin_sort(self.proj, self.n, self.views, self.bins, self.sort_ws, sync=True)
                break
            except gs.GsError as e:
                if e.status != gs.GS_ERR_CAPACITY or e.required <= self.bins.capacity:
                    raise
                self._alloc_bins(int(e.required * 1.25) + 1024)

    def forward(self, g: gs.Gaussians, bg: Sequence[float] = (0.0, 0.0, 0.0)) -> torch.Tensor:
        """Renders every view; returns the packed image buffer [V][3][H][W]."""
        self._project_and_bin(g)
        gs.gs_render_fwd(self.proj, self.n, self.bins, self.views, bg, self.image, self.final_T,
                         self.n_contrib, self.depth)
        return self.image

    def forward_l1(self, g: gs.Gaussians, target: torch.Tensor, dL_dimage: torch.Tensor,
                   loss: Optional[torch.Tensor] = None,
                   bg: Sequence[float] = (0.0, 0.0, 0.0)) -> torch.Tensor:
        """forward() plus the L1 photometric gradient against ``target`` (and
        the loss) in the same compositing pass."""
        self._project_and_bin(g)
        if getattr(self, "_l1_ws", None) is None:
            self._l1_ws = gs.workspace(gs.gs_render_fwd_l1_workspace_size(self.views), self.device)
        gs.gs_render_fwd_l1(self.proj, self.n, self.bins, self.views, bg, self.image, self.final_T,
                            self.n_contrib, target, dL_dimage, loss, self._l1_ws)
        return self.image

    def backward(self, g: gs.Gaussians, dL_dimage: torch.Tensor, grads: gs.Grads, flags: int = 0,
                 bg: Sequence[float] = (0.0, 0.0, 0.0)) -> None:
        """Accumulates gradients of the last forward into ``grads``."""
        gs.gs_render_bwd(g, self.proj, self.bins, self.views, bg, dL_dimage, self.final_T,
                         self.n_contrib, grads, flags, self.bwd_ws)
