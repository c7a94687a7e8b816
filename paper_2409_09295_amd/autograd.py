"""Differentiable rendering with camera-pose gradients (torch.autograd).

GEVO's local and global mapping objectives minimise a photometric loss over
both the map and the keyframe poses T_k (Eq. 2 and Eq. 3), and tracking
optimises the pose alone.  ``GSRender`` exposes the C-ABI renderer as a
``torch.autograd.Function``:

    render = GSRender(cams, n, sh_degree, recompute=False)
    images = render(means, log_scales, quats, opacity_logits, sh, xi)   # packed [V][3][H][W]
    loss(images).backward()   # grads for the five parameter groups and xi

``xi`` is a (V, 6) tangent (rho, phi) of a left perturbation
T_cw <- Exp(xi) T_cw, evaluated at xi = 0: its gradient is the pose gradient
at the current cameras (``apply_pose_step`` moves the cameras along it).  A
nonzero ``xi`` is rejected (the image would otherwise belong to other
poses than the gradient), and so is a backward after ``set_cameras`` has
changed the poses its forward rendered.

Between forward and backward only the per-pixel blend state is kept: the
final transmittance and the index of the last blended splat (8 bytes per
pixel), independent of how many splats a pixel blends; the backward
recovers every splat's transmittance by walking the list in reverse.  The
projected splats and tile lists are the renderer's reusable buffers; with
``recompute=True`` (or when another forward has reused them) the backward
re-runs projection and binning, which reproduce them exactly.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import gs, scenes


class _State:
    def __init__(self, cams: Sequence[scenes.Camera], n: int, sh_degree: int, bg, device):
        self.views = gs.Views(list(cams), device)
        self.n = n
        self.sh_degree = sh_degree
        self.bg = tuple(float(x) for x in bg)
        self.device = device
        V = self.views.n_views
        self.proj = gs.Projected.empty(V, n, device)
        self.n_tiles = self.views.n_tiles
        self._alloc_bins(max(1 << 16, 4 * n * V))
        self.bwd_ws = gs.workspace(gs.gs_render_bwd_workspace_size(n, self.views), device)
        self.generation = 0          # bumps whenever proj/bins are rebuilt
        self.cam_generation = 0      # bumps whenever the poses change

    def _alloc_bins(self, capacity: int):
        capacity = int(min(capacity, 0xFFFFFFFF))
        self.bins = gs.Bins.empty(capacity, self.n_tiles, self.device, keys=False)   # never read here
        self.sort_ws = gs.workspace(gs.gs_bin_sort_workspace_size(self.n, self.views, capacity),
                                    self.device)

    def project_and_bin(self, g: gs.Gaussians) -> int:
        gs.gs_preprocess(g, self.views, self.proj)
        while True:
            try:
                n_keys = gs.gs_bin_sort(self.proj, self.n, self.views, self.bins, self.sort_ws, sync=True)
                break
            except gs.GsError as e:
                if e.status != gs.GS_ERR_CAPACITY or e.required <= self.bins.capacity:
                    raise
                self._alloc_bins(int(e.required * 1.25) + 1024)
        self.generation += 1
        return n_keys


def _gaussians(state: _State, means, log_scales, quats, opacity_logits, sh) -> gs.Gaussians:
    f = lambda t: t.detach().contiguous()
    return gs.Gaussians(f(means), f(log_scales), f(quats), f(opacity_logits), f(sh), state.sh_degree)


class _GSRenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, xi, state: _State, recompute: bool):
        if xi.shape != (state.views.n_views, 6):
            raise ValueError(f"xi must have shape ({state.views.n_views}, 6)")
        if bool(torch.count_nonzero(xi).item()):
            raise ValueError("xi is the tangent at the current poses and must be zero; move the "
                             "cameras with apply_pose_step or set_cameras instead")
        g = _gaussians(state, means, log_scales, quats, opacity_logits, sh)
        state.project_and_bin(g)
        P = state.views.n_pixels
        image = torch.empty(3 * P, dtype=torch.float32, device=state.device)
        final_T = torch.empty(P, dtype=torch.float32, device=state.device)
        n_contrib = torch.empty(P, dtype=torch.int32, device=state.device)
        gs.gs_render_fwd(state.proj, state.n, state.bins, state.views, state.bg, image, final_T, n_contrib)
        ctx.state = state
        ctx.recompute = recompute
        ctx.generation = state.generation
        ctx.cam_generation = state.cam_generation
        ctx.save_for_backward(means, log_scales, quats, opacity_logits, sh, final_T, n_contrib)
        return image

    @staticmethod
    def backward(ctx, dL_dimage):
        means, log_scales, quats, opacity_logits, sh, final_T, n_contrib = ctx.saved_tensors
        state: _State = ctx.state
        if state.cam_generation != ctx.cam_generation:
            raise RuntimeError("the cameras changed between this forward and its backward; the "
                               "saved blend state belongs to the old poses")
        g = _gaussians(state, means, log_scales, quats, opacity_logits, sh)
        if ctx.recompute or state.generation != ctx.generation:
            state.project_and_bin(g)
            ctx.generation = state.generation
        V = state.views.n_views
        grads = gs.Grads(torch.empty_like(g.means), torch.empty_like(g.log_scales),
                         torch.empty_like(g.quats), torch.empty_like(g.opacity_logits),
                         torch.empty_like(g.sh), torch.empty(V, 6, dtype=torch.float32, device=g.means.device))
        gs.gs_render_bwd(g, state.proj, state.bins, state.views, state.bg, dL_dimage.contiguous(),
                         final_T, n_contrib, grads, gs.GS_BWD_OVERWRITE, state.bwd_ws)
        return (grads.means, grads.log_scales, grads.quats, grads.opacity_logits, grads.sh, grads.xi,
                None, None)


class GSRender:
    """Differentiable renderer for a fixed set of cameras (image sizes fixed;
    poses may be updated with ``set_cameras``/``apply_pose_step``)."""

    def __init__(self, cams: Sequence[scenes.Camera], n: int, sh_degree: int,
                 bg: Sequence[float] = (0.0, 0.0, 0.0), recompute: bool = False, device="cuda"):
        self.cams = list(cams)
        self.recompute = recompute
        self.state = _State(self.cams, n, sh_degree, bg, device)

    @property
    def views(self) -> gs.Views:
        return self.state.views

    def __call__(self, means, log_scales, quats, opacity_logits, sh, xi=None) -> torch.Tensor:
        if xi is None:
            xi = torch.zeros(self.state.views.n_views, 6, dtype=torch.float32, device=means.device)
        return _GSRenderFn.apply(means, log_scales, quats, opacity_logits, sh, xi, self.state,
                                 self.recompute)

    def images(self, packed: torch.Tensor):
        return self.state.views.split_images(packed)

    def set_cameras(self, cams: Sequence[scenes.Camera]):
        self.cams = list(cams)
        self.state.views.update_poses(self.cams)
        self.state.cam_generation += 1

    def apply_pose_step(self, delta: np.ndarray):
        """T_cw <- Exp(delta_v) T_cw for every view (delta: (V, 6), rho then phi)."""
        new = []
        for c, d in zip(self.cams, np.asarray(delta, np.float64).reshape(-1, 6)):
            T = se3_exp(d) @ np.vstack([np.hstack([c.R, np.asarray(c.t).reshape(3, 1)]), [0, 0, 0, 1]])
            new.append(scenes.Camera(T[:3, :3], T[:3, 3], c.fx, c.fy, c.cx, c.cy, c.width, c.height))
        self.set_cameras(new)


def se3_exp(xi: np.ndarray) -> np.ndarray:
    """4x4 exponential of the twist (rho, phi) (closed form: Rodrigues and the
    left Jacobian)."""
    rho, phi = np.asarray(xi[:3], np.float64), np.asarray(xi[3:], np.float64)
    th = float(np.linalg.norm(phi))
    K = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    if th < 1e-9:
        R = np.eye(3) + K
        Vm = np.eye(3) + 0.5 * K
    else:
        R = np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K
        Vm = np.eye(3) + (1 - np.cos(th)) / th ** 2 * K + (th - np.sin(th)) / th ** 3 * K @ K
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = Vm @ rho
    return T
