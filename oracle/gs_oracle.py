"""FP64 CPU oracle for the differentiable tile-based 3D Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library: it reads seeded inputs (numpy arrays, camera records) and
computes everything itself in float64 with plain PyTorch CPU tensor ops.

What it computes (the renderer R(M, T) whose images the paper re-renders in
place of stored keyframes, Sec. I and the E_pc loss in Sec. III-B2; the
renderer itself is the Gaussian-splatting rasterizer the paper builds on, so
the steps below follow the published EWA-splatting/3DGS mathematics):

  activations      s = exp(log_scale), q/|q|, o = sigmoid(logit)
  covariance       Sigma = (R(q) S)(R(q) S)^T
  view transform   p = R_cw mu + t_cw; culled when p_z <= Z_NEAR
  projection       u = fx x/z + cx, v = fy y/z + cy (pixel centres at i + 1/2)
  EWA              J with x/z, y/z clamped to +-GUARD * W/(2 fx) (resp. H/(2 fy)),
                   Sigma2 = J R_cw Sigma R_cw^T J^T, Sigma' = Sigma2 + DILATION I,
                   conic Q = Sigma'^-1
  extent           r = ceil(3 sqrt(lambda_max(Sigma')))
  tile rect        tiles holding a pixel centre inside [u-r, u+r] x [v-r, v+r]
  colour           real SH (Condon-Shortley phase, ordered l, m=-l..l) at the
                   unit direction camera-centre -> mean, + 1/2, clamped at >= 0
  keys             (global tile, float32 bits of p_z), ties to the lower index
  compositing      per pixel, front to back over its tile's list:
                   power = -1/2 d^T Q d (skip if > 0), alpha = min(0.99, o e^power)
                   (skip if < 1/255), stop before T would fall below 1e-4,
                   C = sum alpha_i T_i c_i + T_final bg; w(g, u) = alpha T is the
                   blending weight the paper's per-Gaussian error uses (Sec. III-B2)
  gradients        exact derivatives of the above by reverse-mode differentiation,
                   including a left-perturbation 6-DoF pose tangent xi = (rho, phi),
                   T_cw <- Exp(xi) T_cw at xi = 0 (the pose is optimised in the
                   local and global objectives, Eq. 2 and Eq. 3)
  Adam             standard bias-corrected Adam (the paper does not name its
                   optimiser)
  rendering error  E_k(g) = sum_u w(g, u) |R(M, T_k)(u) - C_k(u)| per Gaussian and
                   view, and the active set {g : max_k E_k(g) > eps} united with
                   the newly inserted Gaussians (selective optimisation, Sec. III-B2)
  global stage     insertion of the local map at opacity 0.2, the isotropic
                   regulariser, pruning below opacity 0.7 (Sec. III-B2)

Readings where the paper is silent are the constants below; every one of
them is listed with its reason in the design notes.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

DT = torch.float64

Z_NEAR = 0.2          # near-plane cull (camera-frame z)
DILATION = 0.3        # screen-space covariance dilation, px^2
ALPHA_MAX = 0.99      # opacity clamp
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4          # early-termination transmittance
GUARD = 1.3           # frustum guard on x/z, y/z inside the Jacobian
EXTENT_SIGMAS = 3.0   # r = ceil(3 sqrt(lambda_max))

# Bands used to flag float32 decisions that can legitimately go either way
# (see near_threshold handling in render()).
BAND_REL = 2e-5       # relative band on alpha vs 1/255, o e^power vs 0.99, T' vs 1e-4
BAND_TERMS = 2.4e-7   # plus this times |Q00| dx^2 + 2 |Q01 dx dy| + |Q11| dy^2 on the two
                      # alpha decisions: float32 evaluation of the exponent rounds each
                      # of its terms, so its absolute error scales with their magnitudes
                      # (not with the exponent itself) for an elongated splat
BAND_DEPTH = 1e-12    # relative depth difference under which two splats may swap
                      # (the kernel rounds a float64 depth once, so only depths
                      # tied at float64 precision can order differently)
BAND_EXTENT = 2e-6    # relative band on 3 sqrt(lambda_max) near an integer
BAND_PX = 4e-6        # relative band on u -/+ r - 1/2 near an integer


# ---------------------------------------------------------------------------
# small linear-algebra pieces
# ---------------------------------------------------------------------------

def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of unit quaternions q = (w, x, y, z), shape (4, N) -> (N, 3, 3).
    Built as the matrix of v -> q v q* (Hamilton product)."""
    w, x, y, z = q[0], q[1], q[2], q[3]
    R = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)
    return R


def hat(v: torch.Tensor) -> torch.Tensor:
    z = torch.zeros((), dtype=v.dtype)
    return torch.stack([torch.stack([z, -v[2], v[1]]),
                        torch.stack([v[2], z, -v[0]]),
                        torch.stack([-v[1], v[0], z])])


def se3_exp(xi: torch.Tensor) -> torch.Tensor:
    """4x4 matrix exponential of the twist xi = (rho, phi)."""
    M = torch.zeros((4, 4), dtype=xi.dtype)
    M = M + torch.nn.functional.pad(hat(xi[3:]), (0, 1, 0, 1))
    M = M + torch.nn.functional.pad(xi[:3].reshape(3, 1), (3, 0, 0, 1))
    return torch.linalg.matrix_exp(M)


# ---------------------------------------------------------------------------
# real spherical harmonics, generic definition
# ---------------------------------------------------------------------------

def sh_basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Real spherical harmonics at unit directions d (N, 3) -> (N, (degree+1)^2).

    Y_l^m = K_l^|m| P~_l^|m|(z) * {sqrt2 Re (x+iy)^m  (m > 0), 1 (m = 0),
    sqrt2 Im (x+iy)^|m| (m < 0)} with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
    and P~_l^m(z) = P_l^m(z) / (1 - z^2)^(m/2), where P_l^m carries the
    Condon-Shortley phase; P~ follows the standard three-term recurrence.
    Index k = l^2 + l + m."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    K = (degree + 1) ** 2
    out = [None] * K
    # Re/Im of (x + i y)^m
    cm = [torch.ones_like(x)]
    sm = [torch.zeros_like(x)]
    for m in range(1, degree + 1):
        c_prev, s_prev = cm[-1], sm[-1]
        cm.append(c_prev * x - s_prev * y)
        sm.append(s_prev * x + c_prev * y)
    for m in range(0, degree + 1):
        # P~_m^m, P~_{m+1}^m, ...
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        P = {m: torch.full_like(z, ((-1.0) ** m) * dfact)}
        if m + 1 <= degree:
            P[m + 1] = z * (2 * m + 1) * P[m]
        for l in range(m + 2, degree + 1):
            P[l] = ((2 * l - 1) * z * P[l - 1] - (l + m - 1) * P[l - 2]) / (l - m)
        for l in range(m, degree + 1):
            Klm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                out[l * l + l] = Klm * P[l]
            else:
                out[l * l + l + m] = math.sqrt(2.0) * Klm * P[l] * cm[m]
                out[l * l + l - m] = math.sqrt(2.0) * Klm * P[l] * sm[m]
    return torch.stack(out, dim=1)


# ---------------------------------------------------------------------------
# per-view projection (differentiable)
# ---------------------------------------------------------------------------

def _t(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a, np.float64), dtype=DT)


def project_view(means, log_scales, quats, opacity_logits, sh, sh_degree, R, t, cam):
    """Per-Gaussian screen-space quantities for one camera.

    means (3,N), log_scales (3,N), quats (4,N), opacity_logits (N,), sh (3,K,N)
    are float64 tensors (possibly requiring grad); R (3,3), t (3,) the
    world->camera pose tensors; cam supplies fx, fy, cx, cy, width, height.
    Returns a dict of tensors; integer/boolean entries carry no gradient."""
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    W, H = int(cam.width), int(cam.height)
    N = means.shape[1]
    finite = (torch.isfinite(means).all(0) & torch.isfinite(log_scales).all(0)
              & torch.isfinite(quats).all(0) & torch.isfinite(opacity_logits)
              & torch.isfinite(sh).reshape(-1, N).all(0))
    qn = torch.linalg.vector_norm(quats, dim=0)
    ok_q = qn > 0
    safe_q = torch.where(ok_q & finite, quats / torch.where(qn > 0, qn, torch.ones_like(qn)),
                         torch.tensor([1.0, 0, 0, 0], dtype=DT)[:, None].expand(4, N))
    s = torch.exp(torch.where(finite[None], log_scales, torch.zeros_like(log_scales)))
    o = torch.sigmoid(torch.where(finite, opacity_logits, torch.zeros_like(opacity_logits)))
    mu = torch.where(finite[None], means, torch.zeros_like(means))

    p = (R @ mu).T + t                     # (N, 3) camera frame
    z = p[:, 2]
    in_front = z > Z_NEAR
    zs = torch.where(in_front, z, torch.ones_like(z))
    u = fx * p[:, 0] / zs + cx
    v = fy * p[:, 1] / zs + cy

    limx = GUARD * (W / (2.0 * fx))
    limy = GUARD * (H / (2.0 * fy))
    tx = torch.clamp(p[:, 0] / zs, -limx, limx)
    ty = torch.clamp(p[:, 1] / zs, -limy, limy)
    zero = torch.zeros_like(zs)
    J = torch.stack([torch.stack([fx / zs, zero, -fx * tx / zs], -1),
                     torch.stack([zero, fy / zs, -fy * ty / zs], -1)], -2)   # (N,2,3)

    Rq = quat_to_rotmat(safe_q)                                   # (N,3,3)
    M = Rq * s.T[:, None, :]                                      # R S
    Sigma = M @ M.transpose(1, 2)
    Sig_cam = R @ Sigma @ R.T
    S2 = J @ Sig_cam @ J.transpose(1, 2)                          # (N,2,2)
    a = S2[:, 0, 0] + DILATION
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + DILATION
    det = a * c - b * b
    det_ok = det > 0
    dets = torch.where(det_ok, det, torch.ones_like(det))
    conic = torch.stack([c / dets, -b / dets, a / dets], -1)      # Q00, Q01, Q11

    mid = 0.5 * (a + c)
    lam = mid + torch.sqrt(torch.clamp(mid * mid - det, min=0.0))
    ext = EXTENT_SIGMAS * torch.sqrt(lam.detach())
    radius = torch.ceil(ext).to(torch.int64)

    # colour from SH at the direction camera centre -> mean
    cam_c = -(R.T @ t)
    dvec = mu.T - cam_c
    dnorm = torch.linalg.vector_norm(dvec, dim=1, keepdim=True)
    dirs = dvec / dnorm
    Y = sh_basis(dirs, sh_degree)                                  # (N, K)
    rgb_raw = torch.einsum("ckn,nk->nc", sh, Y) + 0.5
    rgb = torch.clamp(rgb_raw, min=0.0)

    visible = finite & ok_q & in_front & det_ok & (radius > 0)
    return dict(u=u, v=v, z=z, conic=conic, opacity=o, rgb=rgb, radius=radius,
                visible=visible, ext=ext.detach(), fx_x_over_z=(fx * p[:, 0] / zs).detach(),
                fy_y_over_z=(fy * p[:, 1] / zs).detach())


# ---------------------------------------------------------------------------
# binning (integer stage)
# ---------------------------------------------------------------------------

def tile_grid(cam, tile_size: int):
    return (int(cam.width) + tile_size - 1) // tile_size, (int(cam.height) + tile_size - 1) // tile_size


def tile_rects(u, v, r, W: int, H: int, ts: int):
    """Half-open tile rectangles [x0, x1) x [y0, y1) of the tiles that hold a
    pixel centre i + 1/2 with |i + 1/2 - u| <= r (and the same in y).
    u, v float64 arrays, r int array (0 = culled).  Returns int64 arrays and
    the tile count."""
    u = np.asarray(u, np.float64)
    v = np.asarray(v, np.float64)
    r = np.asarray(r, np.int64)
    with np.errstate(invalid="ignore"):
        ilo = np.ceil(u - r - 0.5)
        ihi = np.floor(u + r - 0.5)
        jlo = np.ceil(v - r - 0.5)
        jhi = np.floor(v + r - 0.5)
    empty = ~((ilo <= ihi) & (jlo <= jhi) & (ihi >= 0) & (ilo <= W - 1)
              & (jhi >= 0) & (jlo <= H - 1) & (r > 0) & np.isfinite(u) & np.isfinite(v))
    ilo = np.where(empty, 0, np.clip(ilo, 0, W - 1)).astype(np.int64)
    ihi = np.where(empty, 0, np.clip(ihi, 0, W - 1)).astype(np.int64)
    jlo = np.where(empty, 0, np.clip(jlo, 0, H - 1)).astype(np.int64)
    jhi = np.where(empty, 0, np.clip(jhi, 0, H - 1)).astype(np.int64)
    x0 = ilo // ts
    x1 = ihi // ts + 1
    y0 = jlo // ts
    y1 = jhi // ts + 1
    x0[empty] = x1[empty] = y0[empty] = y1[empty] = 0
    count = (x1 - x0) * (y1 - y0)
    return x0, x1, y0, y1, count


def bin_splats(xy: Sequence[np.ndarray], depth_f32: Sequence[np.ndarray],
               radius: Sequence[np.ndarray], cams, tile_size: int):
    """Tile keys, values and per-tile ranges for V views.

    xy[v] (N, 2) float (used in float64), depth_f32[v] (N,) float32,
    radius[v] (N,) int.  Keys are (global tile << 32) | bits(depth); values are
    v * N + i; emission is Gaussian-major in index order with each rectangle
    row-major, and the sorted order is ascending (key, value).  Returns
    (keys uint64, values uint32, ranges uint32 (T_total, 2), tile_base list)."""
    keys_all = []
    vals_all = []
    bases = []
    base = 0
    V = len(cams)
    N = np.asarray(radius[0]).shape[0]
    for vi, cam in enumerate(cams):
        TX, TY = tile_grid(cam, tile_size)
        bases.append(base)
        x = np.asarray(xy[vi], np.float64)
        x0, x1, y0, y1, cnt = tile_rects(x[:, 0], x[:, 1], radius[vi], cam.width, cam.height, tile_size)
        dbits = np.asarray(depth_f32[vi], np.float32).view(np.uint32).astype(np.uint64)
        sel = np.nonzero(cnt > 0)[0]                 # visible Gaussians, index order
        c = cnt[sel]
        owner = np.repeat(sel, c)                    # Gaussian of each emitted key
        j = np.arange(int(c.sum())) - np.repeat(np.cumsum(c) - c, c)   # position in its rect
        wdt = (x1 - x0)[owner]
        tx = x0[owner] + j % wdt                     # rectangle walked row-major
        ty = y0[owner] + j // wdt
        tiles = (base + ty * TX + tx).astype(np.uint64)
        keys_all.append((tiles << np.uint64(32)) | dbits[owner])
        vals_all.append((vi * N + owner).astype(np.uint64))
        base += TX * TY
    if keys_all:
        keys = np.concatenate(keys_all)
        vals = np.concatenate(vals_all)
    else:
        keys = np.zeros(0, np.uint64)
        vals = np.zeros(0, np.uint64)
    emitted = (keys.copy(), vals.astype(np.uint32))
    order = np.lexsort((vals, keys))
    keys = keys[order]
    vals = vals[order].astype(np.uint32)
    T_total = base
    ranges = np.zeros((T_total, 2), np.uint32)
    if keys.size:
        tiles = (keys >> np.uint64(32)).astype(np.int64)
        starts = np.searchsorted(tiles, np.arange(T_total), side="left")
        ends = np.searchsorted(tiles, np.arange(T_total), side="right")
        nonempty = ends > starts
        ranges[nonempty, 0] = starts[nonempty]
        ranges[nonempty, 1] = ends[nonempty]
    return keys, vals, ranges, bases, emitted


# ---------------------------------------------------------------------------
# compositing (differentiable per tile)
# ---------------------------------------------------------------------------

def _composite_tile(px, py, S, bg, with_mask, depth=None, depth_band=BAND_DEPTH):
    """px, py (P,) pixel centres; S (L, 9) rows u, v, Q00, Q01, Q11, o, r, g, b
    in list order.  Returns colour (P,3), T_final (P,), n_contrib (P,), weights
    (P,L), near-threshold mask (P,) and optional depth sum (P,)."""
    L = S.shape[0]
    P = px.shape[0]
    if L == 0:
        C = bg[None, :].expand(P, 3).clone()
        return (C, torch.ones(P, dtype=DT), torch.zeros(P, dtype=torch.int64),
                torch.zeros((P, 0), dtype=DT), torch.zeros(P, dtype=torch.bool),
                torch.zeros(P, dtype=DT))
    dx = px[:, None] - S[None, :, 0]
    dy = py[:, None] - S[None, :, 1]
    q0, q1, q2 = S[None, :, 2], S[None, :, 3], S[None, :, 4]
    power = -0.5 * (q0 * dx * dx + q2 * dy * dy) - q1 * dx * dy
    raw = S[None, :, 5] * torch.exp(power)
    alpha = torch.clamp(raw, max=ALPHA_MAX)
    keep = (power <= 0) & (alpha >= ALPHA_MIN)
    a = torch.where(keep, alpha, torch.zeros_like(alpha))
    one_m = 1.0 - a
    T_incl = torch.cumprod(one_m, dim=1)
    T_excl = torch.cat([torch.ones((P, 1), dtype=DT), T_incl[:, :-1]], dim=1)
    stop_here = keep & (T_incl.detach() < T_MIN)
    idx = torch.arange(L)
    big = torch.full((P, L), L, dtype=torch.int64)
    s = torch.where(stop_here, idx[None, :].expand(P, L), big).min(dim=1).values   # stop index (L = none)
    active = keep & (idx[None, :] < s[:, None])
    w = torch.where(active, a * T_excl, torch.zeros_like(a))
    C = w @ S[:, 6:9]
    T_fin = torch.where(s < L, T_excl.gather(1, torch.clamp(s, max=L - 1)[:, None])[:, 0], T_incl[:, -1])
    C = C + T_fin[:, None] * bg[None, :]
    last = torch.where(active, idx[None, :].expand(P, L) + 1, torch.zeros_like(big)).max(dim=1).values
    dsum = (w @ depth) if depth is not None else torch.zeros(P, dtype=DT)
    mask = torch.zeros(P, dtype=torch.bool)
    if with_mask:
        with torch.no_grad():
            evaluated = idx[None, :] <= s[:, None]
            rr = raw.detach()
            pw = power.detach()
            terms = (q0 * dx * dx).abs() + (q2 * dy * dy).abs() + 2 * (q1 * dx * dy).abs()
            band = BAND_REL + BAND_TERMS * terms
            near = ((rr - ALPHA_MIN).abs() < band * ALPHA_MIN) \
                | ((rr - ALPHA_MAX).abs() < band * ALPHA_MAX) \
                | ((pw > -1e-6 * terms.detach() - 1e-12) & (pw.abs() < 1e-3)) \
                | (keep & ((T_incl.detach() - T_MIN).abs() < BAND_REL * T_MIN))
            mask = (near & evaluated).any(dim=1)
            if depth is not None and depth_band is not None and L > 1:
                dz = (depth[1:] - depth[:-1]).abs() <= depth_band * depth[1:].abs()
                both = keep[:, 1:] & keep[:, :-1] & evaluated[:, 1:]
                mask |= (both & dz[None, :]).any(dim=1)
    return C, T_fin, last, w, mask, dsum


def _tile_pixels(cam, tile_size, tx, ty):
    xs = torch.arange(tx * tile_size, min((tx + 1) * tile_size, int(cam.width)), dtype=torch.int64)
    ys = torch.arange(ty * tile_size, min((ty + 1) * tile_size, int(cam.height)), dtype=torch.int64)
    yy, xx = torch.meshgrid(ys, xs, indexing="ij")
    return xx.reshape(-1), yy.reshape(-1)


def composite(rows: torch.Tensor, depth: torch.Tensor, vals: np.ndarray, ranges: np.ndarray,
              bases, cams, tile_size: int, bg, dL_dimage=None, with_mask=True,
              pixel_mask=None, tiles=None, depth_band=BAND_DEPTH):
    """Composite every tile of every view.

    rows: (V*N, 9) float64 (u, v, Q00, Q01, Q11, o, r, g, b), a leaf if
    gradients are wanted; depth (V*N,) float64.  dL_dimage: per-view (3,H,W)
    arrays or None.  Per-tile backward accumulates into rows.grad.
    pixel_mask: optional per-view (H, W) bool arrays of pixels to flag.
    depth_band: relative depth gap under which two consecutive splats may be
    ordered differently by a float32 depth (None when depths are given
    exactly, as for render_splats).
    tiles: optional per-view collections of (ty, tx) to composite; pixels of
    other tiles are left NaN (image, T_final, depth) / -1 (n_contrib).
    Returns per-view lists: image (3,H,W), T_final, n_contrib (list position
    of the last blended splat), n_blended (number of splats blended), depth,
    mask."""
    bg_t = _t(bg)
    out = []
    for vi, cam in enumerate(cams):
        W, H = int(cam.width), int(cam.height)
        TX, TY = tile_grid(cam, tile_size)
        fill = np.nan if tiles is not None else 0.0
        img = np.full((3, H, W), fill)
        Tf = np.full((H, W), np.nan if tiles is not None else 1.0)
        nc = np.full((H, W), -1 if tiles is not None else 0, np.int64)
        nu = np.full((H, W), -1 if tiles is not None else 0, np.int64)
        dimg = np.full((H, W), fill)
        msk = np.zeros((H, W), bool)
        g = None if dL_dimage is None else _t(dL_dimage[vi])
        want = None if tiles is None else set(tiles[vi])
        for ty in range(TY):
            for tx in range(TX):
                if want is not None and (ty, tx) not in want:
                    continue
                gt = bases[vi] + ty * TX + tx
                s0, s1 = int(ranges[gt, 0]), int(ranges[gt, 1])
                xx, yy = _tile_pixels(cam, tile_size, tx, ty)
                idx = torch.as_tensor(vals[s0:s1].astype(np.int64))
                S = rows.index_select(0, idx) if s1 > s0 else rows[:0]
                dep = depth.index_select(0, idx).detach() if s1 > s0 else depth[:0].detach()
                C, T_fin, last, w, mask, dsum = _composite_tile(
                    xx.to(DT) + 0.5, yy.to(DT) + 0.5, S, bg_t, with_mask, dep, depth_band)
                if g is not None and rows.requires_grad and s1 > s0:
                    gC = g[:, yy, xx].T
                    (C * gC).sum().backward()
                img[:, yy.numpy(), xx.numpy()] = C.detach().numpy().T
                Tf[yy.numpy(), xx.numpy()] = T_fin.detach().numpy()
                nc[yy.numpy(), xx.numpy()] = last.numpy()
                nu[yy.numpy(), xx.numpy()] = (w.detach() > 0).sum(dim=1).numpy()
                dimg[yy.numpy(), xx.numpy()] = dsum.detach().numpy()
                m = mask.numpy()
                if pixel_mask is not None:
                    m = m | pixel_mask[vi][yy.numpy(), xx.numpy()]
                msk[yy.numpy(), xx.numpy()] = m
        out.append(dict(image=img, T_final=Tf, n_contrib=nc, n_blended=nu, depth=dimg, mask=msk))
    return out


# ---------------------------------------------------------------------------
# stage-wise entry points
# ---------------------------------------------------------------------------

def render_splats(splats, tile_size: int = 16, bg=(0.0, 0.0, 0.0), with_mask=True):
    """Composite given screen-space splats (a scenes.SplatSet, float32 inputs
    read as float64).  Returns (per-view results, keys, values, ranges)."""
    V, N = splats.radius.shape
    keys, vals, ranges, bases, _ = bin_splats(
        [splats.xy[v] for v in range(V)], [splats.rgb_depth[v, :, 3] for v in range(V)],
        [splats.radius[v] for v in range(V)], splats.cams, tile_size)
    rows = torch.cat([_t(splats.xy.reshape(V * N, 2)),
                      _t(splats.conic_opacity.reshape(V * N, 4)),
                      _t(splats.rgb_depth.reshape(V * N, 4)[:, :3])], dim=1)
    depth = _t(splats.rgb_depth.reshape(V * N, 4)[:, 3])
    res = composite(rows, depth, vals, ranges, bases, splats.cams, tile_size, bg, None, with_mask,
                    depth_band=None)
    return res, keys, vals, ranges


def _ambiguous_pixels(P, cam, tile_size):
    """Pixels whose splat list could differ under float32 rounding of a
    splat's extent, projected centre or near-plane test: for every such
    splat, the pixels of the tiles it may or may not cover at which it would
    be blended (raw alpha within the band of 1/255 or above).  Returns an
    (H, W) bool array."""
    TX, TY = tile_grid(cam, tile_size)
    W, H = int(cam.width), int(cam.height)
    flag = np.zeros((H, W), bool)
    u = P["u"].detach().numpy()
    v = P["v"].detach().numpy()
    ext = P["ext"].numpy()
    rad = P["radius"].numpy()
    vis = P["visible"].numpy()
    z = P["z"].detach().numpy()
    conic = P["conic"].detach().numpy()
    opac = P["opacity"].detach().numpy()
    with np.errstate(invalid="ignore"):
        ext_amb = np.abs(ext - np.round(ext)) < BAND_EXTENT * np.maximum(ext, 1.0)
        z_amb = np.abs(z - Z_NEAR) < 1e-5 * max(Z_NEAR, 1.0)
        bu = BAND_PX * np.maximum.reduce([np.ones_like(u), np.abs(u), np.abs(P["fx_x_over_z"].numpy())])
        bv = BAND_PX * np.maximum.reduce([np.ones_like(v), np.abs(v), np.abs(P["fy_y_over_z"].numpy())])
        r_lo = np.where(ext_amb, np.round(ext), rad)
        r_hi = np.where(ext_amb, np.round(ext) + 1, rad)
        edge_amb = np.zeros_like(ext_amb)
        for val in (u - rad - 0.5, u + rad - 0.5):
            edge_amb |= np.abs(val - np.round(val)) < bu
        for val in (v - rad - 0.5, v + rad - 0.5):
            edge_amb |= np.abs(val - np.round(val)) < bv
    cand = np.nonzero((vis | z_amb) & (ext_amb | z_amb | edge_amb) & np.isfinite(u) & np.isfinite(v))[0]
    for i in cand:
        if z_amb[i]:
            r_big = int(max(rad[i], 1)) + 1
            x0, x1, y0, y1, c = tile_rects(u[i:i + 1], v[i:i + 1], np.array([r_big]), W, H, tile_size)
            if c[0] > 0:
                flag[y0[0] * tile_size:y1[0] * tile_size, x0[0] * tile_size:x1[0] * tile_size] = True
            continue
        big = tile_rects(np.array([u[i] - bu[i], u[i] + bu[i]]), np.array([v[i] - bv[i], v[i] + bv[i]]),
                         np.array([r_hi[i], r_hi[i]]), W, H, tile_size)
        small = tile_rects(np.array([u[i] - bu[i], u[i] + bu[i]]), np.array([v[i] - bv[i], v[i] + bv[i]]),
                           np.array([max(r_lo[i], 0), max(r_lo[i], 0)]), W, H, tile_size)
        if big[4].max() == 0:
            continue
        region = np.zeros((TY, TX), bool)
        region[big[2].min():big[3].max(), big[0].min():big[1].max()] = True
        if small[4].min() > 0:
            ix0, ix1 = small[0].max(), small[1].min()
            iy0, iy1 = small[2].max(), small[3].min()
            if ix1 > ix0 and iy1 > iy0:
                region[iy0:iy1, ix0:ix1] = False
        q0, q1, q2 = conic[i]
        for ty, tx in zip(*np.nonzero(region)):
            ys = np.arange(ty * tile_size, min((ty + 1) * tile_size, H))
            xs = np.arange(tx * tile_size, min((tx + 1) * tile_size, W))
            dy = ys[:, None] + 0.5 - v[i]
            dx = xs[None, :] + 0.5 - u[i]
            power = -0.5 * (q0 * dx * dx + q2 * dy * dy) - q1 * dx * dy
            raw = opac[i] * np.exp(np.minimum(power, 0.0))
            hit = raw >= ALPHA_MIN * (1.0 - BAND_REL)
            flag[ys[0]:ys[-1] + 1, xs[0]:xs[-1] + 1] |= hit
    return flag


def render(gmap, cams, tile_size: int = 16, bg=(0.0, 0.0, 0.0), dL_dimage=None,
           with_mask=True, want_pose_grad=True, tiles=None):
    """Full pipeline from Gaussian parameters (scenes.GaussianMap, float32
    arrays read as float64) for a list of cameras.

    Returns dict(views=[per-view image, T_final, n_contrib, depth, mask],
    proj=[per-view projected numpy arrays], keys/values/ranges of the
    binning, and, if dL_dimage is given, grads: means, log_scales, quats,
    opacity_logits, sh (same layouts as the inputs) and xi (V, 6))."""
    want_grad = dL_dimage is not None
    leaves = [_t(a).requires_grad_(want_grad) for a in gmap.arrays()]
    means, log_scales, quats, ologit, sh = leaves
    N = gmap.n
    V = len(cams)
    xis = [torch.zeros(6, dtype=DT, requires_grad=want_grad and want_pose_grad) for _ in cams]
    projs = []
    outs = []
    for vi, cam in enumerate(cams):
        R0 = _t(np.asarray(cam.R, np.float64).reshape(3, 3))
        t0 = _t(np.asarray(cam.t, np.float64).reshape(3))
        if want_grad and want_pose_grad:
            T = se3_exp(xis[vi]) @ torch.cat([torch.cat([R0, t0[:, None]], 1),
                                              torch.tensor([[0, 0, 0, 1.0]], dtype=DT)], 0)
            R, t = T[:3, :3], T[:3, 3]
        else:
            R, t = R0, t0
        P = project_view(means, log_scales, quats, ologit, sh, gmap.sh_degree, R, t, cam)
        projs.append(P)
        o = torch.where(P["visible"], P["opacity"], torch.zeros_like(P["opacity"]))
        outs.append(torch.cat([P["u"][:, None], P["v"][:, None], P["conic"], o[:, None], P["rgb"]], 1))
    rows_graph = torch.cat(outs, 0)                                     # (V*N, 9)
    rows = rows_graph.detach().clone().requires_grad_(want_grad)
    depth = torch.cat([P["z"].detach() for P in projs])
    radius = [torch.where(P["visible"], P["radius"], torch.zeros_like(P["radius"])).numpy() for P in projs]
    xy = [torch.stack([P["u"], P["v"]], 1).detach().numpy() for P in projs]
    dz = [P["z"].detach().numpy().astype(np.float32) for P in projs]
    keys, vals, ranges, bases, _ = bin_splats(xy, dz, radius, cams, tile_size)
    tmask = [_ambiguous_pixels(P, cam, tile_size) for P, cam in zip(projs, cams)] if with_mask else None
    res = composite(rows, depth, vals, ranges, bases, cams, tile_size, bg, dL_dimage, with_mask, tmask,
                    tiles)
    result = dict(views=res, keys=keys, values=vals, ranges=ranges, bases=bases,
                  proj=[{k: (val.detach().numpy() if torch.is_tensor(val) else val) for k, val in P.items()}
                        for P in projs])
    if want_grad:
        if rows.grad is None:
            rows.grad = torch.zeros_like(rows)
        torch.autograd.backward([rows_graph], [rows.grad])
        zero = lambda x: (x.grad if x.grad is not None else torch.zeros_like(x)).numpy()
        result["grads"] = dict(means=zero(means), log_scales=zero(log_scales), quats=zero(quats),
                               opacity_logits=zero(ologit), sh=zero(sh),
                               xi=np.stack([zero(x) for x in xis]) if want_pose_grad else np.zeros((V, 6)))
        result["grad2d"] = rows.grad.numpy().reshape(V, N, 9)
    return result


def gradient_term_mass(gmap, cams, dL_dimage, gauss_ids, tile_size: int = 16, bg=(0.0, 0.0, 0.0),
                       tiles=None):
    """Absolute first-order mass of the per-pixel terms whose sum is each map
    gradient of the Gaussians ``gauss_ids``: for a parameter theta of
    Gaussian g,

        mass(theta) = sum over views and pixels u of
                      sum_k |d row_k / d theta| |d (C(u) . dL/dC(u)) / d row_k|

    with row = g's screen-space splat (u, v, conic, opacity, colour).  The
    gradient itself is the same sum without the absolute values; when its
    terms cancel, mass / |gradient| is the factor by which rounding of the
    terms is amplified.  Also returns the longest list position walked by any
    pixel where one of the Gaussians contributes.  Test infrastructure: it
    bounds float32 rounding of ill-conditioned gradient elements and is not a
    reference value.  Returns (dict group -> array (len(ids), components),
    walk)."""
    ids = [int(i) for i in gauss_ids]
    K = (gmap.sh_degree + 1) ** 2
    comps = dict(means=3, log_scales=3, quats=4, opacity_logits=1, sh=3 * K)
    mass = {k: np.zeros((len(ids), c)) for k, c in comps.items()}
    walk = 0
    leaves = [_t(a) for a in gmap.arrays()]
    bg_t = _t(bg)
    for vi, cam in enumerate(cams):
        R = _t(np.asarray(cam.R, np.float64).reshape(3, 3))
        t = _t(np.asarray(cam.t, np.float64).reshape(3))
        P = project_view(*leaves, gmap.sh_degree, R, t, cam)
        o = torch.where(P["visible"], P["opacity"], torch.zeros_like(P["opacity"]))
        rows = torch.cat([P["u"][:, None], P["v"][:, None], P["conic"], o[:, None], P["rgb"]], 1)
        rows = rows.detach()
        radius = torch.where(P["visible"], P["radius"], torch.zeros_like(P["radius"])).numpy()
        xy = torch.stack([P["u"], P["v"]], 1).detach().numpy()
        _, vals, ranges, _, _ = bin_splats([xy], [P["z"].detach().numpy().astype(np.float32)],
                                           [radius], [cam], tile_size)
        # d row / d theta of each listed Gaussian (a single-Gaussian projection)
        jac = {}
        for j, gi in enumerate(ids):
            if not bool(P["visible"][gi]):
                continue
            sl = [a[..., gi:gi + 1].clone().requires_grad_(True) for a in leaves]
            Pg = project_view(*sl, gmap.sh_degree, R, t, cam)
            row = torch.cat([Pg["u"], Pg["v"], Pg["conic"][0], Pg["opacity"], Pg["rgb"][0]])
            J = []
            for k in range(9):
                gk = torch.autograd.grad(row[k], sl, retain_graph=True, allow_unused=True)
                J.append(torch.cat([(x if x is not None else torch.zeros_like(a)).reshape(-1)
                                    for x, a in zip(gk, sl)]))
            jac[gi] = torch.stack(J).abs().numpy()                  # (9, n_params)
        if not jac:
            continue
        TX, TY = tile_grid(cam, tile_size)
        g = _t(dL_dimage[vi])
        want = None if tiles is None else set(tiles[vi])
        for ty in range(TY):
            for tx in range(TX):
                if want is not None and (ty, tx) not in want:
                    continue
                gt = ty * TX + tx
                s0, s1 = int(ranges[gt, 0]), int(ranges[gt, 1])
                lst = vals[s0:s1].astype(np.int64)
                here = [(j, gi, int(np.nonzero(lst == gi)[0][0])) for j, gi in enumerate(ids)
                        if gi in jac and (lst == gi).any()]
                if not here:
                    continue
                xx, yy = _tile_pixels(cam, tile_size, tx, ty)
                S = rows[torch.as_tensor(lst)].clone().requires_grad_(True)
                C, _, last, _, _, _ = _composite_tile(xx.to(DT) + 0.5, yy.to(DT) + 0.5, S, bg_t, False)
                f = (C * g[:, yy, xx].T).sum(dim=1)
                gr = torch.autograd.grad(f, S, grad_outputs=torch.eye(f.shape[0], dtype=DT),
                                         is_grads_batched=True)[0]          # (P, L, 9)
                for j, gi, pos in here:
                    sp = gr[:, pos, :].abs()
                    if float(sp.sum()) == 0.0:
                        continue
                    walk = max(walk, int(last.max()))
                    m = sp.sum(dim=0).numpy() @ jac[gi]                   # (n_params,)
                    off = 0
                    for k, c in comps.items():
                        mass[k][j] += m[off:off + c]
                        off += c
    return mass, walk


# ---------------------------------------------------------------------------
# per-Gaussian rendering error and the active set (selective optimisation)
# ---------------------------------------------------------------------------

def render_error(gmap, cams, targets, tile_size: int = 16, bg=(0.0, 0.0, 0.0), pixel_mask=None,
                 tiles=None):
    """Per-Gaussian rendering error of the global stage's active-set selection
    (Sec. III-B2), for every view k of ``cams``:

        E_k(g) = sum over pixels u of w(g, u) |R(M, T_k)(u) - C_k(u)|

    w(g, u) = alpha_g(u) T_g(u) is g's blending weight at u, R(M, T_k) the
    render of the map from view k (this oracle's own) and C_k = targets[k]
    (3, H, W).  The paper leaves the reduction over colour channels open; the
    RGB residual's |.| is read as its L1 norm (sum over the channels).
    pixel_mask: optional per-view (H, W) bool arrays of pixels to leave out
    (their residual counts as 0).  tiles: optional per-view collections of
    (ty, tx): only those tiles' pixels are summed (the others count as 0).

    Returns dict(err (V, N), weight (V, N): sum over u of w(g, u),
    images: per-view (3, H, W) renders, T_final: per-view (H, W))."""
    V, N = len(cams), gmap.n
    res = render(gmap, cams, tile_size, bg, with_mask=False, want_pose_grad=False)
    rows = []
    for P in res["proj"]:
        o = np.where(P["visible"], P["opacity"], 0.0)
        rows.append(np.concatenate([P["u"][:, None], P["v"][:, None], P["conic"], o[:, None],
                                    P["rgb"]], 1))
    rows = _t(np.concatenate(rows, 0))
    bg_t = _t(bg)
    err = np.zeros(V * N)
    wsum = np.zeros(V * N)
    vals, ranges, bases = res["values"], res["ranges"], res["bases"]
    for vi, cam in enumerate(cams):
        TX, TY = tile_grid(cam, tile_size)
        tgt = _t(targets[vi])
        want = None if tiles is None else set(tiles[vi])
        for ty in range(TY):
            for tx in range(TX):
                if want is not None and (ty, tx) not in want:
                    continue
                gt = bases[vi] + ty * TX + tx
                s0, s1 = int(ranges[gt, 0]), int(ranges[gt, 1])
                if s1 <= s0:
                    continue
                xx, yy = _tile_pixels(cam, tile_size, tx, ty)
                idx = vals[s0:s1].astype(np.int64)
                S = rows.index_select(0, torch.as_tensor(idx))
                C, _, _, w, _, _ = _composite_tile(xx.to(DT) + 0.5, yy.to(DT) + 0.5, S, bg_t, False)
                e = (C - tgt[:, yy, xx].T).abs().sum(dim=1)          # (P,) L1 over channels
                if pixel_mask is not None:
                    e = torch.where(torch.as_tensor(pixel_mask[vi][yy.numpy(), xx.numpy()]),
                                    torch.zeros_like(e), e)
                err[idx] += (w.T @ e).numpy()                          # a Gaussian appears once per tile
                wsum[idx] += w.sum(dim=0).numpy()
    return dict(err=err.reshape(V, N), weight=wsum.reshape(V, N),
                images=[v["image"] for v in res["views"]], T_final=[v["T_final"] for v in res["views"]])


def active_set(err: np.ndarray, eps: float, always: Optional[np.ndarray] = None) -> np.ndarray:
    """E_t = {g : max over the window's views k of E_k(g) > eps}, united with
    the Gaussians flagged in ``always`` (the newly inserted local map), as a
    bool array over the Gaussians (Sec. III-B2)."""
    err = np.asarray(err, np.float64)
    mask = err.max(axis=0) > eps if err.shape[0] else np.zeros(err.shape[1], bool)
    if always is not None:
        mask = mask | (np.asarray(always) != 0)
    return mask


# ---------------------------------------------------------------------------
# global stage: insertion, isotropic regulariser, pruning
# ---------------------------------------------------------------------------

INSERT_OPACITY = 0.2     # opacity of the local map when it enters the global map
PRUNE_OPACITY = 0.7      # Gaussians below this opacity are pruned after optimisation
ISO_WEIGHT = 10.0        # weight of the isotropic regulariser (the paper gives none)


def logit(p: float) -> float:
    return math.log(p / (1.0 - p))


def insert(global_map, local_map, opacity: float = INSERT_OPACITY):
    """Pre-optimised global map M'_t = M_{t-1} united with the local map M~_t
    (Sec. III-B2): the previous global map's Gaussians first, then the local
    map's, whose opacity is lowered to ``opacity`` (its logit) before the
    insertion.  Returns the five parameter arrays (float64) and the flags of
    the inserted Gaussians."""
    out = []
    for k, (a, b) in enumerate(zip(global_map.arrays(), local_map.arrays())):
        b = np.asarray(b, np.float64)
        if k == 3:
            b = np.full(b.shape, logit(opacity))
        out.append(np.concatenate([np.asarray(a, np.float64), b], axis=-1))
    new = np.r_[np.zeros(global_map.n, np.uint8), np.ones(local_map.n, np.uint8)]
    return out, new


def iso_loss_grad(log_scales, weight: float = ISO_WEIGHT):
    """Isotropic regulariser E_iso (Eq. 2 and Eq. 3; the paper states only that
    it keeps Gaussians from becoming elongated or thin): the mean over all
    Gaussians and their three axes of |s_j - mean_k s_k|, s = exp(log_scale),
    times ``weight``.  Returns (E_iso, dE_iso/dlog_scales (3, N))."""
    ls = _t(log_scales).requires_grad_(True)
    s = torch.exp(ls)
    # s_j - (s_0 + s_1 + s_2) / 3 written as a third of s_j's differences to the
    # other two: the same value, exactly 0 when the three scales are equal
    d = torch.stack([(s[0] - s[1]) + (s[0] - s[2]), (s[1] - s[0]) + (s[1] - s[2]),
                     (s[2] - s[0]) + (s[2] - s[1])]) / 3.0
    E = weight * d.abs().mean()
    E.backward()
    return float(E.detach()), ls.grad.numpy()


def prune_keep(opacity_logits, min_opacity: float = PRUNE_OPACITY):
    """Gaussians kept by the opacity rule of the pruning step (Sec. III-B2):
    opacity sigmoid(logit) not below ``min_opacity``.  The occupancy rule
    (Gaussian mixture regression on free-space Gaussians) is not part of this
    reading."""
    o = 1.0 / (1.0 + np.exp(-np.asarray(opacity_logits, np.float64)))
    return o >= min_opacity


def pose_adam_step(R, t, g, m, v, lr_trans, lr_rot, beta1, beta2, eps, step):
    """The pose step of the mapping objectives (which minimise over the
    keyframe poses T_k, Eq. 2 and Eq. 3): one bias-corrected Adam step on the
    left-perturbation tangent xi = (rho, phi) from its gradient g (6,), with
    rate lr_trans on rho and lr_rot on phi, then T <- Exp(delta) T.  Returns
    the new (R, t, m, v) in float64."""
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    lr = np.r_[[lr_trans] * 3, [lr_rot] * 3]
    delta = -lr * (m / (1 - beta1 ** step)) / (np.sqrt(v / (1 - beta2 ** step)) + eps)
    E = se3_exp(torch.as_tensor(delta)).numpy()
    T = np.eye(4)
    T[:3, :3] = np.asarray(R, np.float64).reshape(3, 3)
    T[:3, 3] = np.asarray(t, np.float64).reshape(3)
    Tn = E @ T
    return Tn[:3, :3], Tn[:3, 3], m, v


# ---------------------------------------------------------------------------
# loss gradient and optimiser
# ---------------------------------------------------------------------------

def l1_loss_grad(image: np.ndarray, target: np.ndarray):
    """L = mean |C - C*| over 3 H W; returns (L, dL/dC) with sign(0) = 0."""
    diff = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    n = diff.size
    return float(np.abs(diff).sum() / n), np.sign(diff) / n


def adam_step(p, g, m, v, lr, beta1, beta2, eps, step, mask=None):
    """One bias-corrected Adam step in float64; entries with mask == 0 are
    left untouched.  Returns new (p, m, v)."""
    p = np.asarray(p, np.float64).copy()
    g = np.asarray(g, np.float64)
    m = np.asarray(m, np.float64).copy()
    v = np.asarray(v, np.float64).copy()
    sel = np.ones(p.shape, bool) if mask is None else (np.asarray(mask) != 0)
    m_new = beta1 * m + (1 - beta1) * g
    v_new = beta2 * v + (1 - beta2) * g * g
    mhat = m_new / (1 - beta1 ** step)
    vhat = v_new / (1 - beta2 ** step)
    p_new = p - lr * mhat / (np.sqrt(vhat) + eps)
    p[sel] = p_new[sel]
    m[sel] = m_new[sel]
    v[sel] = v_new[sel]
    return p, m, v
