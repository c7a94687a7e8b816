"""FP64 CPU oracle for the learned and plain Gaussian initialisers.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).  It
shares no code with the HIP library.  Tensors are float64 torch CPU tensors
in NHWC layout ([n, h, w, c]) unless stated.

Plain initialiser: the photometric cost volume of Eq. 1 (Sec. III-A1) over a
keyframe window, 64 hypotheses spaced evenly over 0.25-25 m, on 1/4
resolution intensity images, reduced per pixel by winner-take-all or by
loopy min-sum belief propagation under a truncated linear smoothness prior
(Sec. III-A2).

Network pieces: 3x3 convolution with zero padding (written as an explicit
sum over the nine taps), 2x2 average pooling, nearest 2x upsampling, ReLU,
a 1x1 head and the depth loss; gradients by reverse-mode differentiation.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional

import numpy as np
import torch

DT = torch.float64
N_HYP = 64
D_MIN, D_MAX = 0.25, 25.0


# ---------------------------------------------------------------------------
# network pieces
# ---------------------------------------------------------------------------

def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest even), returned as float64."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def conv3x3(x: torch.Tensor, w: torch.Tensor, bias: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x [n, h, w, cin], w [9, cout, cin] (tap = 3 dy + dx) -> [n, h, w, cout]:
    y[p] = bias + sum over taps of w[tap] @ x[p + (dy - 1, dx - 1)], zero outside."""
    n, h, wd, cin = x.shape
    xp = torch.nn.functional.pad(x, (0, 0, 1, 1, 1, 1))          # pad w then h
    y = torch.zeros((n, h, wd, w.shape[1]), dtype=x.dtype)
    for tap in range(9):
        dy, dx = tap // 3, tap % 3
        y = y + xp[:, dy:dy + h, dx:dx + wd, :] @ w[tap].T
    if bias is not None:
        y = y + bias
    return y


def avgpool2(x: torch.Tensor) -> torch.Tensor:
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(dim=(2, 4))


def upsample2(x: torch.Tensor) -> torch.Tensor:
    return x.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)


def head(f: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """f [n, h, w, c], w [2, c] -> [n, 2, h, w]."""
    return (f @ w.T + b).permute(0, 3, 1, 2)


def depth_loss(pred: torch.Tensor, depth: torch.Tensor, fx: float) -> torch.Tensor:
    """mean over pixels with depth > 0 of |pred0 - log d| + |pred1 - log(d/fx)|."""
    valid = depth > 0
    d = torch.where(valid, depth, torch.ones_like(depth))
    e = (pred[:, 0] - torch.log(d)).abs() + (pred[:, 1] - torch.log(d / fx)).abs()
    return (e * valid).sum() / max(int(valid.sum()), 1)


CHANNELS = (32, 64, 128, 256)


def unet_layers(in_ch: int = 8, ch=CHANNELS):
    """(name, cin, cout) of the 14 convolutions of the 4-level U-Net."""
    c0, c1, c2, c3 = ch
    return [("e0a", in_ch, c0), ("e0b", c0, c0), ("e1a", c0, c1), ("e1b", c1, c1),
            ("e2a", c1, c2), ("e2b", c2, c2), ("e3a", c2, c3), ("e3b", c3, c3),
            ("d2a", c3 + c2, c2), ("d2b", c2, c2), ("d1a", c2 + c1, c1), ("d1b", c1, c1),
            ("d0a", c1 + c0, c0), ("d0b", c0, c0)]


class Bf16Store(torch.autograd.Function):
    """A tensor held in bfloat16: the value rounded to the nearest bfloat16
    (ties to even) going forward, and the gradient flowing back rounded the
    same way (the network keeps activations and their gradients in BF16,
    with FP32 accumulation in between)."""

    @staticmethod
    def forward(ctx, x):
        return x.to(torch.float32).to(torch.bfloat16).to(x.dtype)

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.float32).to(torch.bfloat16).to(g.dtype)


def bf16_store(x: torch.Tensor) -> torch.Tensor:
    return Bf16Store.apply(x)


def unet_forward(x: torch.Tensor, p: Dict[str, torch.Tensor], store=None) -> torch.Tensor:
    """x [n, h, w, in_ch]; p maps '<layer>.w' [9, cout, cin], '<layer>.b' [cout],
    'head.w' [2, c0], 'head.b' [2].  Encoder: two conv+ReLU per level, 2x2
    average pooling between levels; decoder: nearest upsampling, concatenation
    [upsampled, skip], two conv+ReLU; 1x1 head.

    store (optional, e.g. bf16_store) is applied to every tensor the network
    holds between layers: each conv+ReLU output, each pooled and upsampled
    map, and each skip input of a concatenation (which rounds the gradient
    that flows back into it on its own)."""
    q = store if store is not None else (lambda t: t)
    r = torch.relu
    c = lambda name, t: q(r(conv3x3(t, p[name + ".w"], p[name + ".b"])))
    e0 = c("e0b", c("e0a", x))
    e1 = c("e1b", c("e1a", q(avgpool2(e0))))
    e2 = c("e2b", c("e2a", q(avgpool2(e1))))
    e3 = c("e3b", c("e3a", q(avgpool2(e2))))
    d2 = c("d2b", c("d2a", torch.cat([q(upsample2(e3)), q(e2)], dim=3)))
    d1 = c("d1b", c("d1a", torch.cat([q(upsample2(d2)), q(e1)], dim=3)))
    d0 = c("d0b", c("d0a", torch.cat([q(upsample2(d1)), q(e0)], dim=3)))
    return head(d0, p["head.w"], p["head.b"])


# ---------------------------------------------------------------------------
# plain initialiser
# ---------------------------------------------------------------------------

def hypotheses() -> np.ndarray:
    return D_MIN + (D_MAX - D_MIN) * np.arange(N_HYP) / (N_HYP - 1)


def luma_down4(rgb: np.ndarray) -> np.ndarray:
    """rgb [3, H, W] -> intensity 0.299 R + 0.587 G + 0.114 B averaged over 4x4 blocks."""
    rgb = np.asarray(rgb, np.float64)
    I = 0.299 * rgb[0] + 0.587 * rgb[1] + 0.114 * rgb[2]
    H, W = I.shape
    return I.reshape(H // 4, 4, W // 4, 4).mean(axis=(1, 3))


def _bilinear(img: np.ndarray, x: np.ndarray, y: np.ndarray):
    Hl, Wl = img.shape
    ok = (x >= 0) & (y >= 0) & (x <= Wl - 1) & (y <= Hl - 1)
    xs = np.where(ok, x, 0.0)
    ys = np.where(ok, y, 0.0)
    x0 = np.floor(xs).astype(np.int64)
    y0 = np.floor(ys).astype(np.int64)
    x1 = np.minimum(x0 + 1, Wl - 1)
    y1 = np.minimum(y0 + 1, Hl - 1)
    fx = xs - x0
    fy = ys - y0
    v = ((1 - fy) * ((1 - fx) * img[y0, x0] + fx * img[y0, x1])
         + fy * ((1 - fx) * img[y1, x0] + fx * img[y1, x1]))
    return v, ok


def cost_volume(keyframes: List[np.ndarray], cams) -> np.ndarray:
    """Eq. 1: V(u, d) = mean over source views i of |I_ref(u) - I_i(pi(u, d, T))|
    for the last keyframe as reference, at 1/4 resolution; views whose sample
    falls outside the image or behind the camera are left out of the mean
    (+inf when none remains).  Returns [64, H/4, W/4]."""
    low = [luma_down4(k) for k in keyframes]
    ref = cams[-1]
    Hl, Wl = low[-1].shape
    jj, ii = np.meshgrid(np.arange(Hl), np.arange(Wl), indexing="ij")
    u = 4.0 * ii + 2.0
    v = 4.0 * jj + 2.0
    rx = (u - ref.cx) / ref.fx
    ry = (v - ref.cy) / ref.fy
    Rr, tr = np.asarray(ref.R, np.float64), np.asarray(ref.t, np.float64)
    out = np.empty((N_HYP, Hl, Wl))
    for h, d in enumerate(hypotheses()):
        Xc = np.stack([rx * d, ry * d, np.full_like(rx, d)], -1)      # camera frame of the reference
        Xw = (Xc - tr) @ Rr                                            # R^T (Xc - t)
        acc = np.zeros((Hl, Wl))
        cnt = np.zeros((Hl, Wl))
        for k, cam in enumerate(cams[:-1]):
            P = Xw @ np.asarray(cam.R, np.float64).T + np.asarray(cam.t, np.float64)
            front = P[..., 2] > 1e-6
            z = np.where(front, P[..., 2], 1.0)
            us = cam.fx * P[..., 0] / z + cam.cx
            vs = cam.fy * P[..., 1] / z + cam.cy
            val, ok = _bilinear(low[k], (us - 2.0) / 4.0, (vs - 2.0) / 4.0)
            ok &= front
            acc += np.where(ok, np.abs(low[-1] - val), 0.0)
            cnt += ok
        out[h] = np.where(cnt > 0, acc / np.maximum(cnt, 1), np.inf)
    return out


def wta_depth(cost: np.ndarray) -> np.ndarray:
    """First hypothesis of minimum cost; 0 where every cost is +inf."""
    idx = np.argmin(cost, axis=0)
    d = hypotheses()[idx]
    return np.where(np.isfinite(cost.min(axis=0)), d, 0.0)


# ---------------------------------------------------------------------------
# belief propagation over the cost volume (Sec. III-A2)
# ---------------------------------------------------------------------------

BP_LAMBDA = 0.01        # smoothness cost per hypothesis step (the paper gives none)
BP_TRUNC = 0.08         # truncation of the smoothness cost
BP_ITERS = 30           # synchronous message-passing iterations
BP_INVALID = 1.0        # data cost of a hypothesis no source view sees


def bp_messages_step(D, m, lam, trunc):
    """One synchronous min-sum iteration on the 4-connected grid.

    D [L, H, W] data costs; m [4, L, H, W] the messages each pixel received
    in the last iteration, from its left (0), right (1), upper (2) and lower
    (3) neighbour.  A pixel sends to a neighbour the minimum over its own
    labels l of D(l) plus the messages it received from its other three
    neighbours plus the smoothness cost min(lam |l - l'|, trunc), for every
    label l' of the receiver, shifted so that its minimum is 0.  Written out
    as the definition (an explicit minimum over l for each l')."""
    L, H, W = D.shape
    lab = np.arange(L)
    S = np.minimum(lam * np.abs(lab[:, None] - lab[None, :]), trunc)       # [l, l']
    total = D + m.sum(axis=0)
    new = np.zeros_like(m)

    def send(h):
        out = np.empty_like(h)
        for lp in range(L):
            out[lp] = (h + S[:, lp][:, None, None]).min(axis=0)
        return out - out.min(axis=0, keepdims=True)

    # to the right neighbour: excludes what came from the right
    new[0][:, :, 1:] = send(total - m[1])[:, :, :-1]
    new[1][:, :, :-1] = send(total - m[0])[:, :, 1:]          # to the left
    new[2][:, 1:, :] = send(total - m[3])[:, :-1, :]          # downwards
    new[3][:, :-1, :] = send(total - m[2])[:, 1:, :]          # upwards
    return new


def belief_propagation(cost, lam=BP_LAMBDA, trunc=BP_TRUNC, iters=BP_ITERS, invalid=BP_INVALID):
    """Loopy min-sum belief propagation (Felzenszwalb and Huttenlocher's
    formulation, Sec. III-A2) over a cost volume [L, H, W]: +inf entries (no
    valid source view) cost ``invalid``; messages start at 0 and are updated
    synchronously ``iters`` times; the label of a pixel is the first minimum of
    its belief, the data cost plus the four incoming messages.  Returns
    (labels [H, W], beliefs [L, H, W])."""
    D = np.where(np.isfinite(cost), np.asarray(cost, np.float64), invalid)
    m = np.zeros((4,) + D.shape)
    for _ in range(iters):
        m = bp_messages_step(D, m, lam, trunc)
    belief = D + m.sum(axis=0)
    return np.argmin(belief, axis=0), belief


def bp_depth(cost, **kw) -> np.ndarray:
    labels, _ = belief_propagation(cost, **kw)
    return hypotheses()[labels]
