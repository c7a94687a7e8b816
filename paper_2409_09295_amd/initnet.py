"""Learned Gaussian initialiser and its plain counterpart.

GEVO creates new Gaussians from a depth image of the newest keyframe; its
depth comes from a photometric cost volume over the keyframe window (Eq. 1,
Sec. III-A1) reduced by belief propagation (Sec. III-A2).  This module holds

* ``plain_depth``: the cost volume of Eq. 1 at 1/4 resolution, reduced by
  winner-take-all (``gs_cost_volume_wta``), upsampled 4x by repetition: the
  fallback initialiser and the reference the learned one is measured against;
* ``UNet``: a 4-level U-Net (32/64/128/256 channels, two 3x3 conv + ReLU per
  level, 2x2 average pooling, nearest upsampling with skip concatenation, a
  1x1 head) that maps one RGB keyframe to per-pixel log depth and log scale.
  Activations and weights are BF16, accumulation FP32 on MFMA, FP32 master
  weights updated by ``gs_adam_step``; every layer runs in the library's
  kernels (``gs_nn_*``);
* training data rendered by the library's own rasterizer: (image, depth)
  pairs with depth = sum(w z) / (1 - T_final) where the render is at least
  half opaque;
* ``propose``: per-pixel Gaussians (means, log-scales) from a depth image.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import gs, scenes
from .rasterizer import Rasterizer

IN_CH = 8
CHANNELS = (32, 64, 128, 256)


def layer_specs(ch=CHANNELS):
    c0, c1, c2, c3 = ch
    return [("e0a", IN_CH, c0), ("e0b", c0, c0), ("e1a", c0, c1), ("e1b", c1, c1),
            ("e2a", c1, c2), ("e2b", c2, c2), ("e3a", c2, c3), ("e3b", c3, c3),
            ("d2a", c3 + c2, c2), ("d2b", c2, c2), ("d1a", c2 + c1, c1), ("d1b", c1, c1),
            ("d0a", c1 + c0, c0), ("d0b", c0, c0)]


def unet_flops(h: int, w: int, ch=CHANNELS) -> float:
    """Multiply-adds x 2 of the 3x3 convolutions of one forward pass."""
    res = {"e0": 1, "e1": 2, "e2": 4, "e3": 8, "d2": 4, "d1": 2, "d0": 1}
    tot = 0.0
    for name, cin, cout in layer_specs(ch):
        s = res[name[:2]]
        tot += 2.0 * 9 * cin * cout * (h // s) * (w // s)
    return tot


class UNet:
    def __init__(self, seed: int = 0, device="cuda", ch=CHANNELS, depth_prior: float = 3.0,
                 fx_prior: float = 525.0):
        self.device = device
        self.ch = ch
        self.specs = layer_specs(ch)
        g = torch.Generator().manual_seed(seed)
        self.params: Dict[str, torch.Tensor] = {}
        for name, cin, cout in self.specs:
            fan = 9 * (3 if name == "e0a" else cin)
            w = torch.randn(9, cout, cin, generator=g) * math.sqrt(2.0 / fan)
            if name == "e0a":
                w[:, :, 3:] = 0.0                    # input padding channels
            self.params[name + ".w"] = w.to(device)
            self.params[name + ".b"] = torch.zeros(cout, device=device)
        self.params["head.w"] = (torch.randn(2, ch[0], generator=g) * 0.01).to(device)
        self.params["head.b"] = torch.tensor([math.log(depth_prior), math.log(depth_prior / fx_prior)],
                                             device=device)
        self.grads = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.m = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.params.items()}
        self.step_count = 0
        self.wb: Dict[str, torch.Tensor] = {}
        self.wt: Dict[str, torch.Tensor] = {}
        for name, cin, cout in self.specs:
            self.wb[name] = torch.empty(9, cout, cin, dtype=torch.bfloat16, device=device)
            self.wt[name] = torch.empty(9, cin, cout, dtype=torch.bfloat16, device=device)
        self.refresh()
        self._bufs = None
        self._shape = None

    # -- weights --------------------------------------------------------------
    def refresh(self):
        """BF16 forward weights and flipped backward-data weights from the FP32 masters."""
        for name, cin, cout in self.specs:
            gs.gs_nn_f32_to_bf16(self.params[name + ".w"], self.wb[name])
            gs.gs_nn_flip_weights(self.wb[name], cout, cin, self.wt[name])

    def state_dict(self):
        return {k: v.detach().cpu() for k, v in self.params.items()}

    def load_state_dict(self, sd):
        for k, v in sd.items():
            self.params[k].copy_(v.to(self.device))
        self.refresh()

    # -- buffers ----------------------------------------------------------------
    def _alloc(self, n: int, h: int, w: int):
        if self._shape == (n, h, w):
            return self._bufs
        if h % 8 or w % 8:
            raise ValueError("image height and width must be multiples of 8")
        c0, c1, c2, c3 = self.ch
        A = lambda s, c: gs.Act.empty(n, h // s, w // s, c, self.device, zero=True)
        b = {}
        b["x"] = A(1, IN_CH)
        for lvl, s, c in (("e0", 1, c0), ("e1", 2, c1), ("e2", 4, c2), ("e3", 8, c3)):
            b[lvl + "a"] = A(s, c)
            b[lvl + "b"] = A(s, c)
        b["p0"], b["p1"], b["p2"] = A(2, c0), A(4, c1), A(8, c2)
        b["u2"], b["u1"], b["u0"] = A(4, c3), A(2, c2), A(1, c1)
        for lvl, s, c in (("d2", 4, c2), ("d1", 2, c1), ("d0", 1, c0)):
            b[lvl + "a"] = A(s, c)
            b[lvl + "b"] = A(s, c)
        # gradient buffers (w.r.t. layer outputs)
        for key in list(b.keys()):
            if key != "x":
                b["g_" + key] = A(*{"e0": (1,), "e1": (2,), "e2": (4,), "e3": (8,), "d2": (4,),
                                    "d1": (2,), "d0": (1,), "p0": (2,), "p1": (4,), "p2": (8,),
                                    "u2": (4,), "u1": (2,), "u0": (1,)}[key[:2]], b[key].c)
        b["g_cat2"] = A(4, c3 + c2)
        b["g_cat1"] = A(2, c2 + c1)
        b["g_cat0"] = A(1, c1 + c0)
        b["pred"] = torch.zeros(n, 2, h, w, device=self.device)
        b["dpred"] = torch.zeros(n, 2, h, w, device=self.device)
        b["loss"] = torch.zeros(1, dtype=torch.float64, device=self.device)
        b["loss_ws"] = torch.zeros(4, dtype=torch.int32, device=self.device)
        self._bufs, self._shape = b, (n, h, w)
        return b

    # -- forward / backward -------------------------------------------------------
    def _conv(self, name, x1, x2, y):
        _, cin, cout = next(s for s in self.specs if s[0] == name)
        gs.gs_nn_conv3x3(x1, x2, None, self.wb[name], cout, self.params[name + ".b"], True, y)

    def forward(self, rgb: torch.Tensor) -> torch.Tensor:
        """rgb: planar float32 [n, 3, h, w] -> prediction [n, 2, h, w]
        (log depth, log scale)."""
        n, _, h, w = rgb.shape
        b = self._alloc(n, h, w)
        gs.gs_nn_rgb_to_nhwc(rgb.contiguous(), b["x"])
        self._conv("e0a", b["x"], None, b["e0a"])
        self._conv("e0b", b["e0a"], None, b["e0b"])
        gs.gs_nn_avgpool2(b["e0b"], b["p0"])
        self._conv("e1a", b["p0"], None, b["e1a"])
        self._conv("e1b", b["e1a"], None, b["e1b"])
        gs.gs_nn_avgpool2(b["e1b"], b["p1"])
        self._conv("e2a", b["p1"], None, b["e2a"])
        self._conv("e2b", b["e2a"], None, b["e2b"])
        gs.gs_nn_avgpool2(b["e2b"], b["p2"])
        self._conv("e3a", b["p2"], None, b["e3a"])
        self._conv("e3b", b["e3a"], None, b["e3b"])
        gs.gs_nn_upsample2(b["e3b"], b["u2"])
        self._conv("d2a", b["u2"], b["e2b"], b["d2a"])
        self._conv("d2b", b["d2a"], None, b["d2b"])
        gs.gs_nn_upsample2(b["d2b"], b["u1"])
        self._conv("d1a", b["u1"], b["e1b"], b["d1a"])
        self._conv("d1b", b["d1a"], None, b["d1b"])
        gs.gs_nn_upsample2(b["d1b"], b["u0"])
        self._conv("d0a", b["u0"], b["e0b"], b["d0a"])
        self._conv("d0b", b["d0a"], None, b["d0b"])
        gs.gs_nn_head(b["d0b"], self.params["head.w"], self.params["head.b"], b["pred"])
        return b["pred"]

    def _layer_bwd(self, name, x1, x2, y, gy, gx):
        """Gradients of conv+ReLU layer `name` given gy = dL/dy (y its output):
        weight/bias gradients, and gx = dL/d(input) unless gx is None."""
        _, cin, cout = next(s for s in self.specs if s[0] == name)
        gs.gs_nn_conv3x3_wgrad(x1, x2, gy, y, self.grads[name + ".w"], self.grads[name + ".b"])
        if gx is not None:
            gs.gs_nn_conv3x3(gy, None, y, self.wt[name], cin, None, False, gx)

    def backward(self, dpred: torch.Tensor) -> None:
        """Accumulates parameter gradients for the last forward."""
        b = self._bufs
        c0, c1, c2, c3 = self.ch
        gs.gs_nn_head_bwd(b["d0b"], self.params["head.w"], dpred.contiguous(), b["g_d0b"],
                          self.grads["head.w"], self.grads["head.b"])
        self._layer_bwd("d0b", b["d0a"], None, b["d0b"], b["g_d0b"], b["g_d0a"])
        self._layer_bwd("d0a", b["u0"], b["e0b"], b["d0a"], b["g_d0a"], b["g_cat0"])
        gs.gs_nn_upsample2_bwd(b["g_cat0"].slice(0, c1), b["g_d1b"])
        self._layer_bwd("d1b", b["d1a"], None, b["d1b"], b["g_d1b"], b["g_d1a"])
        self._layer_bwd("d1a", b["u1"], b["e1b"], b["d1a"], b["g_d1a"], b["g_cat1"])
        gs.gs_nn_upsample2_bwd(b["g_cat1"].slice(0, c2), b["g_d2b"])
        self._layer_bwd("d2b", b["d2a"], None, b["d2b"], b["g_d2b"], b["g_d2a"])
        self._layer_bwd("d2a", b["u2"], b["e2b"], b["d2a"], b["g_d2a"], b["g_cat2"])
        gs.gs_nn_upsample2_bwd(b["g_cat2"].slice(0, c3), b["g_e3b"])
        self._layer_bwd("e3b", b["e3a"], None, b["e3b"], b["g_e3b"], b["g_e3a"])
        self._layer_bwd("e3a", b["p2"], None, b["e3a"], b["g_e3a"], b["g_p2"])
        gs.gs_nn_avgpool2_bwd(b["g_p2"], b["g_cat2"].slice(c3, c2), b["g_e2b"])
        self._layer_bwd("e2b", b["e2a"], None, b["e2b"], b["g_e2b"], b["g_e2a"])
        self._layer_bwd("e2a", b["p1"], None, b["e2a"], b["g_e2a"], b["g_p1"])
        gs.gs_nn_avgpool2_bwd(b["g_p1"], b["g_cat1"].slice(c2, c1), b["g_e1b"])
        self._layer_bwd("e1b", b["e1a"], None, b["e1b"], b["g_e1b"], b["g_e1a"])
        self._layer_bwd("e1a", b["p0"], None, b["e1a"], b["g_e1a"], b["g_p0"])
        gs.gs_nn_avgpool2_bwd(b["g_p0"], b["g_cat0"].slice(c1, c0), b["g_e0b"])
        self._layer_bwd("e0b", b["e0a"], None, b["e0b"], b["g_e0b"], b["g_e0a"])
        self._layer_bwd("e0a", b["x"], None, b["e0a"], b["g_e0a"], None)

    def zero_grad(self):
        for g in self.grads.values():
            g.zero_()

    def adam(self, lr: float = 1e-3):
        self.step_count += 1
        for k, p in self.params.items():
            gs.gs_adam_step(p, self.grads[k], self.m[k], self.v[k], lr, 0.9, 0.999, 1e-8, self.step_count)
        self.refresh()

    def loss_and_grad(self, pred: torch.Tensor, depth: torch.Tensor, fx: float) -> torch.Tensor:
        b = self._bufs
        gs.gs_nn_depth_loss(pred, depth.contiguous(), fx, b["dpred"], b["loss"], b["loss_ws"])
        return b["dpred"]

    def predict_depth(self, rgb: torch.Tensor) -> torch.Tensor:
        return torch.exp(self.forward(rgb)[:, 0]).clone()

    def buffer_bytes(self) -> int:
        """Bytes of the activation, gradient and prediction buffers of the
        last batch shape."""
        if self._bufs is None:
            return 0
        tot = 0
        for v in self._bufs.values():
            t = v.t if isinstance(v, gs.Act) else v
            tot += t.numel() * t.element_size()
        return tot


# ---------------------------------------------------------------------------
# data: renders of the map with their depth
# ---------------------------------------------------------------------------

def conv_throughput(n: int = 4, h: int = 480, w: int = 640, reps: int = 5, seed: int = 0) -> dict:
    """Forward and forward + backward time of the U-Net on n random h x w
    images (HIP events around each pass), with the convolutions' rate:
    forward flops as counted by unet_flops, backward twice that (data and
    weight gradients)."""
    net = UNet(seed=seed)
    g = torch.Generator(device="cuda").manual_seed(seed)
    rgb = torch.rand(n, 3, h, w, device="cuda", generator=g)
    dpred = torch.randn(n, 2, h, w, device="cuda", generator=g) * 1e-3
    net.forward(rgb)
    net.backward(dpred)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    fwd = bwd = 0.0
    for _ in range(reps):
        ev[0].record()
        net.forward(rgb)
        ev[1].record()
        net.backward(dpred)
        ev[2].record()
        torch.cuda.synchronize()
        fwd += ev[0].elapsed_time(ev[1]) / reps
        bwd += ev[1].elapsed_time(ev[2]) / reps
    fl = unet_flops(h, w) * n
    return {"images": n, "height": h, "width": w, "fwd_ms": fwd, "bwd_ms": bwd,
            "fwd_tflops": fl / (fwd * 1e-3) / 1e12,
            "fwd_bwd_tflops": 3 * fl / ((fwd + bwd) * 1e-3) / 1e12}


def render_dataset(gmap: scenes.GaussianMap, cams: Sequence[scenes.Camera], batch: int = 16,
                   device="cuda") -> Tuple[torch.Tensor, torch.Tensor]:
    """(rgb [n, 3, h, w], depth [n, h, w]) rendered by the rasterizer; depth
    = sum(w z) / (1 - T_final) where 1 - T_final >= 0.5, else 0."""
    g = gs.Gaussians.from_map(gmap, device)
    W, H = cams[0].width, cams[0].height
    rgbs, depths = [], []
    for i in range(0, len(cams), batch):
        chunk = cams[i:i + batch]
        views = gs.Views(chunk, device)
        r = Rasterizer(g.n, views, device=device, with_depth=True)
        img = r.forward(g)
        alpha = 1.0 - r.final_T
        d = torch.where(alpha >= 0.5, r.depth / alpha.clamp(min=1e-6), torch.zeros_like(alpha))
        rgbs.append(img.view(len(chunk), 3, H, W).clone())
        depths.append(d.view(len(chunk), H, W).clone())
    return torch.cat(rgbs), torch.cat(depths)


def trajectory_cams(n: int, seed: int, boxes, W: int, H: int, per_path: int = 50) -> List[scenes.Camera]:
    """n views along seeded room trajectories (a new path every `per_path`
    views, so long sequences cover the whole room); focal length 525 px at
    640 px width, scaled to W."""
    f = 525.0 * W / 640.0
    poses = []
    k = 0
    while len(poses) < n:
        m = min(per_path, n - len(poses))
        poses += scenes.room_trajectory(m, seed * 1000 + k, boxes)
        k += 1
    return [scenes.Camera(R, t, f, f, W / 2, H / 2, W, H) for R, t in poses]


# ---------------------------------------------------------------------------
# plain initialiser and evaluation
# ---------------------------------------------------------------------------

BP_LAMBDA, BP_TRUNC, BP_ITERS, BP_INVALID = 0.01, 0.08, 30, 1.0


def plain_depth(keyframes: torch.Tensor, cams: Sequence[scenes.Camera], device="cuda",
                method: str = "wta") -> torch.Tensor:
    """Eq. 1 cost volume for the last keyframe, reduced per pixel by
    winner-take-all (``method="wta"``; 0 where no hypothesis had a valid
    view) or by belief propagation under the truncated linear smoothness
    prior (``"bp"``, Sec. III-A2), upsampled 4x by repetition: [h, w]."""
    k, _, H, W = keyframes.shape
    views = gs.Views(list(cams), device)
    ws = gs.workspace(gs.gs_cost_volume_workspace_size(k, H, W), device)
    low = torch.empty(H // 4, W // 4, device=device)
    if method == "wta":
        gs.gs_cost_volume_wta(keyframes.contiguous(), views, None, low, ws)
    elif method == "bp":
        cost = torch.empty(64, H // 4, W // 4, device=device)
        gs.gs_cost_volume_wta(keyframes.contiguous(), views, cost, low, ws)
        bws = gs.workspace(gs.gs_bp_workspace_size(H // 4, W // 4), device)
        gs.gs_bp_labels(cost, H // 4, W // 4, BP_LAMBDA, BP_TRUNC, BP_ITERS, BP_INVALID, None, low, bws)
    else:
        raise ValueError(f"unknown method {method}")
    return low.repeat_interleave(4, 0).repeat_interleave(4, 1)


def learned_depth(net: "UNet", keyframes: torch.Tensor, cams: Sequence[scenes.Camera],
                  device="cuda") -> Tuple[torch.Tensor, Optional[torch.Tensor], bool]:
    """Depth and log-scale of the newest keyframe from the network
    (Sec. III-A1); when any of its outputs is not finite, the plain
    initialiser's depth (Eq. 1, winner-take-all) over the window instead.
    Returns (depth [h, w], log-scale [h, w] or None, whether the network's
    output was used)."""
    pred = net.forward(keyframes[-1:].contiguous())[0]
    if bool(torch.isfinite(pred).all()):
        return torch.exp(pred[0]).clone(), pred[1].clone(), True
    return plain_depth(keyframes, cams, device), None, False


def abs_rel(pred: torch.Tensor, gt: torch.Tensor) -> float:
    """Mean |pred - gt| / gt over pixels with gt > 0 (pred <= 0 counts as error 1)."""
    m = gt > 0
    err = torch.where(pred > 0, (pred - gt).abs() / gt.clamp(min=1e-6), torch.ones_like(gt))
    return float(err[m].mean())


def rmse(pred: torch.Tensor, gt: torch.Tensor) -> float:
    """Root mean square of (pred - gt) in metres over pixels with gt > 0
    (a pixel without a prediction, pred <= 0, counts as predicting 0)."""
    m = gt > 0
    return float(((pred.clamp(min=0) - gt)[m] ** 2).mean().sqrt())


def propose(depth: torch.Tensor, cam: scenes.Camera, stride: int = 4,
            log_scale: Optional[torch.Tensor] = None):
    """Gaussians at every `stride`-th pixel of a depth image: means on the
    back-projected rays (world frame) and isotropic log-scales, the pixel
    footprint log(depth / fx) (or the given per-pixel log_scale map) plus
    log(stride).  Returns (means [3, m], log_scales [3, m])."""
    H, W = depth.shape
    ys, xs = torch.meshgrid(torch.arange(stride // 2, H, stride, device=depth.device),
                            torch.arange(stride // 2, W, stride, device=depth.device), indexing="ij")
    d = depth[ys, xs]
    keep = d > 0
    foot = log_scale[ys, xs][keep] if log_scale is not None else None
    d, xs, ys = d[keep], xs[keep].float() + 0.5, ys[keep].float() + 0.5
    Xc = torch.stack([(xs - cam.cx) / cam.fx * d, (ys - cam.cy) / cam.fy * d, d])
    R = torch.as_tensor(np.asarray(cam.R), dtype=torch.float32, device=depth.device)
    t = torch.as_tensor(np.asarray(cam.t), dtype=torch.float32, device=depth.device)
    means = R.T @ (Xc - t[:, None])
    if foot is None:
        foot = torch.log(d / cam.fx)
    ls = (foot + math.log(stride)).expand(3, -1)
    return means.contiguous(), ls.contiguous()


@dataclasses.dataclass
class InitReport:
    train_pairs: int
    heldout: int
    resolution: Tuple[int, int]
    epochs: int
    net_absrel: float
    plain_absrel: float
    net_rmse: float
    plain_rmse: float
    final_loss: float
    train_seconds: float
    conv_tflops: float


def train_and_compare(n_gauss: int = 200000, W: int = 128, H: int = 96, n_train: int = 600,
                    n_heldout: int = 12, window: int = 8, epochs: int = 15, batch: int = 8,
                    lr: float = 2e-3, seed: int = 0, sh_degree: int = 3, device="cuda",
                    log=None) -> Tuple[UNet, InitReport]:
    """Renders a procedural room, trains the U-Net on (render, depth) pairs and
    compares its depth AbsRel and RMSE with the plain initialiser's on
    held-out trajectory views (each with the `window` preceding keyframes as
    its window)."""
    gmap, boxes = scenes.procedural_room(n_gauss, seed, sh_degree=sh_degree)
    train_cams = trajectory_cams(n_train, seed + 101, boxes, W, H)
    test_cams = trajectory_cams(n_heldout + window, seed + 202, boxes, W, H)
    rgb, depth = render_dataset(gmap, train_cams, device=device)
    trgb, tdepth = render_dataset(gmap, test_cams, device=device)
    fx = train_cams[0].fx
    net = UNet(seed=seed, device=device, fx_prior=fx)
    perm_gen = torch.Generator().manual_seed(seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = float("nan")
    steps = 0
    for ep in range(epochs):
        perm = torch.randperm(n_train, generator=perm_gen)
        tot = 0.0
        for i in range(0, n_train - batch + 1, batch):
            idx = perm[i:i + batch].to(device)
            x = rgb.index_select(0, idx).contiguous()
            d = depth.index_select(0, idx).contiguous()
            pred = net.forward(x)
            dpred = net.loss_and_grad(pred, d, fx)
            net.zero_grad()
            net.backward(dpred)
            net.adam(lr * (0.1 ** (ep / max(epochs - 1, 1))))
            tot += float(net._bufs["loss"].item())
            steps += 1
        last = tot / max(1, n_train // batch)
        if log:
            log(f"epoch {ep}: loss {last:.4f}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    flops = 3.0 * unet_flops(H, W) * steps * batch
    net_err, plain_err, net_sq, plain_sq = [], [], [], []
    for j in range(n_heldout):
        k = j + window - 1                          # held-out view, with window - 1 predecessors
        gt = tdepth[k]
        pd = net.predict_depth(trgb[k:k + 1].contiguous())[0]
        net_err.append(abs_rel(pd, gt))
        net_sq.append(rmse(pd, gt) ** 2)
        pl = plain_depth(trgb[j:k + 1].contiguous(), test_cams[j:k + 1], device)
        plain_err.append(abs_rel(pl, gt))
        plain_sq.append(rmse(pl, gt) ** 2)
    rep = InitReport(n_train, n_heldout, (W, H), epochs, float(np.mean(net_err)),
                     float(np.mean(plain_err)), float(np.sqrt(np.mean(net_sq))),
                     float(np.sqrt(np.mean(plain_sq))), last, secs, flops / secs / 1e12)
    return net, rep


def main(argv=None) -> None:
    """Train and evaluate the initialiser at a chosen size and print one JSON
    line; the defaults are the full-size run: 640 x 480, 5,000 training
    renders of a 1,000,000-Gaussian room, 500 held-out views."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--gaussians", type=int, default=1000000)
    ap.add_argument("--width", type=int, default=640)
    ap.add_argument("--height", type=int, default=480)
    ap.add_argument("--train", type=int, default=5000)
    ap.add_argument("--heldout", type=int, default=500)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    import sys
    t0 = time.perf_counter()
    _, rep = train_and_compare(a.gaussians, a.width, a.height, a.train, a.heldout, epochs=a.epochs,
                               batch=a.batch, lr=a.lr, seed=a.seed,
                               log=lambda m: print(m, file=sys.stderr, flush=True))
    out = dataclasses.asdict(rep)
    out.update(gaussians=a.gaussians, batch=a.batch, total_seconds=time.perf_counter() - t0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
