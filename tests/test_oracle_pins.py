"""Pins of the FP64 oracle against closed forms, library routines, brute force
and invariants (CPU only).  Each test targets a mistake that would otherwise
slip through: a wrong SH sign or index, a transposed rotation, a wrong tile
edge, a dropped transmittance factor."""
import math

import numpy as np
import pytest
import scipy.special as sps
import torch

from oracle import gs_oracle as O
from paper_2409_09295_amd import scenes


# ---------------------------------------------------------------------------
# spherical harmonics
# ---------------------------------------------------------------------------

def _scipy_real_sh(d, degree):
    """Real SH from scipy's complex SH (Condon-Shortley phase included):
    m > 0: sqrt2 Re Y_l^m, m < 0: sqrt2 Im Y_l^|m|, m = 0: Y_l^0."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    out = np.zeros((d.shape[0], (degree + 1) ** 2))
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = sps.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                val = math.sqrt(2) * Y.real
            elif m < 0:
                val = math.sqrt(2) * Y.imag
            else:
                val = Y.real
            out[:, l * l + l + m] = val
    return out


def test_sh_matches_scipy():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ours = O.sh_basis(torch.as_tensor(d), 3).numpy()
    ref = _scipy_real_sh(d, 3)
    np.testing.assert_allclose(ours, ref, rtol=0, atol=1e-12)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi integrates products of
    # degree <= 6 exactly.
    xg, wg = np.polynomial.legendre.leggauss(12)
    phis = np.linspace(0, 2 * np.pi, 24, endpoint=False)
    zz, pp = np.meshgrid(xg, phis, indexing="ij")
    ww = np.repeat(wg[:, None], len(phis), 1) * (2 * np.pi / len(phis))
    st = np.sqrt(1 - zz ** 2)
    d = np.stack([st * np.cos(pp), st * np.sin(pp), zz], -1).reshape(-1, 3)
    Y = O.sh_basis(torch.as_tensor(d), 3).numpy()
    G = (Y * ww.reshape(-1, 1)).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_sign_convention_degree1():
    # Degree 1 is (-y, z, -x) * sqrt(3 / (4 pi)) in this ordering.
    d = np.array([[0.36, -0.48, 0.8]])
    Y = O.sh_basis(torch.as_tensor(d), 1).numpy()[0]
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y, [0.5 / math.sqrt(math.pi), -c1 * -0.48, c1 * 0.8, -c1 * 0.36], atol=1e-15)


# ---------------------------------------------------------------------------
# rotation and pose exponential
# ---------------------------------------------------------------------------

def _hamilton(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def test_quat_rotation_matches_hamilton_product():
    rng = np.random.default_rng(2)
    q = rng.normal(size=(4, 20))
    q /= np.linalg.norm(q, axis=0)
    R = O.quat_to_rotmat(torch.as_tensor(q)).numpy()
    for i in range(20):
        v = rng.normal(size=3)
        qc = q[:, i] * np.array([1, -1, -1, -1])
        rot = _hamilton(_hamilton(q[:, i], np.r_[0.0, v]), qc)[1:]
        np.testing.assert_allclose(R[i] @ v, rot, atol=1e-13)
        np.testing.assert_allclose(np.linalg.det(R[i]), 1.0, atol=1e-13)


def test_se3_exp_rotation_part_is_rodrigues():
    phi = np.array([0.3, -0.2, 0.5])
    rho = np.array([0.1, 0.2, -0.3])
    T = O.se3_exp(torch.as_tensor(np.r_[rho, phi])).numpy()
    th = np.linalg.norm(phi)
    k = phi / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    Rr = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K
    np.testing.assert_allclose(T[:3, :3], Rr, atol=1e-13)
    # translation part: left Jacobian times rho
    Jl = np.eye(3) + (1 - math.cos(th)) / th * K + (th - math.sin(th)) / th * K @ K
    np.testing.assert_allclose(T[:3, 3], Jl @ rho, atol=1e-13)


# ---------------------------------------------------------------------------
# single Gaussian closed form
# ---------------------------------------------------------------------------

def _single(s, z, f, W, H, o_logit, f0, cx=None, cy=None, xy=(0.0, 0.0)):
    g = scenes.GaussianMap(
        means=np.array([[xy[0]], [xy[1]], [z]], np.float32),
        log_scales=np.full((3, 1), math.log(s), np.float32),
        quats=np.array([[1.0], [0.0], [0.0], [0.0]], np.float32),
        opacity_logits=np.array([o_logit], np.float32),
        sh=np.array(f0, np.float32).reshape(3, 1, 1), sh_degree=0)
    cam = scenes.Camera(np.eye(3), np.zeros(3), f, f, W / 2 if cx is None else cx,
                        H / 2 if cy is None else cy, W, H)
    return g, cam


@pytest.mark.parametrize("s,z,o_logit", [(0.05, 3.0, 0.5), (0.02, 2.0, 3.0), (0.2, 5.0, -1.0)])
def test_single_gaussian_closed_form(s, z, o_logit):
    W, H, f = 64, 48, 100.0
    f0 = [0.7, -0.3, 1.2]
    g, cam = _single(np.float32(s), np.float32(z), f, W, H, o_logit, f0)
    s, z = math.exp(float(g.log_scales[0, 0])), float(np.float32(z))
    res = O.render(g, [cam], tile_size=16, bg=(0.1, 0.2, 0.3))
    view = res["views"][0]
    P = res["proj"][0]
    var = (f * s / z) ** 2 + 0.3
    np.testing.assert_allclose(P["conic"][0], [1 / var, 0.0, 1 / var], rtol=1e-12, atol=1e-15)
    r = math.ceil(3 * math.sqrt(var))
    assert P["radius"][0] == r
    o = 1 / (1 + math.exp(-float(np.float32(o_logit))))
    col = np.array([float(np.float32(c)) for c in f0]) / (2 * math.sqrt(math.pi)) + 0.5
    col = np.maximum(col, 0)
    bg = np.array([0.1, 0.2, 0.3])
    # brute-force tile membership: tiles holding a pixel centre inside [u +- r]
    u, v = W / 2, H / 2
    touched = np.zeros((H // 16 + 1, W // 16 + 1), bool)
    for j in range(H):
        for i in range(W):
            if abs(i + 0.5 - u) <= r and abs(j + 0.5 - v) <= r:
                touched[j // 16, i // 16] = True
    for j in range(H):
        for i in range(W):
            d2 = (i + 0.5 - u) ** 2 + (j + 0.5 - v) ** 2
            a = min(0.99, o * math.exp(-0.5 * d2 / var))
            if not touched[j // 16, i // 16] or a < 1 / 255:
                expect = bg
            else:
                expect = a * col + (1 - a) * bg
            np.testing.assert_allclose(view["image"][:, j, i], expect, rtol=0, atol=1e-13)


def test_projection_off_axis_closed_form():
    # mean at (x, y, z) with identity camera: u = f x / z + cx
    g, cam = _single(0.05, 4.0, 120.0, 80, 60, 0.0, [0, 0, 0], xy=(0.5, -0.25))
    res = O.render(g, [cam])
    P = res["proj"][0]
    np.testing.assert_allclose(P["u"][0], 120.0 * 0.5 / 4.0 + 40.0, rtol=1e-7)
    np.testing.assert_allclose(P["v"][0], 120.0 * -0.25 / 4.0 + 30.0, rtol=1e-7)


def test_near_plane_cull():
    g, cam = _single(0.05, 0.19, 100.0, 32, 32, 2.0, [1, 1, 1])
    res = O.render(g, [cam])
    assert res["proj"][0]["visible"][0] == False  # noqa: E712
    assert len(res["keys"]) == 0
    np.testing.assert_array_equal(res["views"][0]["image"], 0.0)


# ---------------------------------------------------------------------------
# binning vs brute force
# ---------------------------------------------------------------------------

def test_tile_rects_brute_force():
    rng = np.random.default_rng(5)
    W, H, ts = 70, 45, 16
    n = 400
    u = rng.uniform(-30, W + 30, n)
    v = rng.uniform(-30, H + 30, n)
    r = rng.integers(0, 25, n)
    # include exact half-integer edges
    u[:20] = np.round(u[:20]) + 0.5
    x0, x1, y0, y1, cnt = O.tile_rects(u, v, r, W, H, ts)
    for k in range(n):
        touched = set()
        if r[k] > 0:
            for j in range(H):
                for i in range(W):
                    if abs(i + 0.5 - u[k]) <= r[k] and abs(j + 0.5 - v[k]) <= r[k]:
                        touched.add((j // ts, i // ts))
        rect = {(ty, tx) for ty in range(y0[k], y1[k]) for tx in range(x0[k], x1[k])}
        assert rect == touched, k
        assert cnt[k] == len(touched)


def test_sorted_keys_match_python_sorted():
    cams = [scenes.pinhole(100, 70, 80.0), scenes.pinhole(48, 40, 40.0)]
    sp = scenes.random_splats(300, cams, seed=3, depth_ties=0.3)
    V, N = sp.radius.shape
    keys, vals, ranges, bases, emitted = O.bin_splats(
        [sp.xy[v] for v in range(V)], [sp.rgb_depth[v, :, 3] for v in range(V)],
        [sp.radius[v] for v in range(V)], cams, 16)
    # brute force: tuples (global tile, depth bits, value)
    tuples = []
    base = 0
    for vi, cam in enumerate(cams):
        TX, TY = O.tile_grid(cam, 16)
        for i in range(N):
            r = sp.radius[vi, i]
            if r <= 0:
                continue
            u, v = float(sp.xy[vi, i, 0]), float(sp.xy[vi, i, 1])
            tiles = set()
            for j in range(cam.height):
                for x in range(cam.width):
                    if abs(x + 0.5 - u) <= r and abs(j + 0.5 - v) <= r:
                        tiles.add((j // 16) * TX + x // 16)
            db = int(np.float32(sp.rgb_depth[vi, i, 3]).view(np.uint32))
            for t in tiles:
                tuples.append((base + t, db, vi * N + i))
        base += TX * TY
    tuples.sort()
    assert len(tuples) == len(keys)
    np.testing.assert_array_equal(keys, np.array([(t << 32) | d for t, d, _ in tuples], np.uint64))
    np.testing.assert_array_equal(vals, np.array([x for _, _, x in tuples], np.uint32))
    # ranges by brute force
    tl = np.array([t for t, _, _ in tuples])
    for t in range(base):
        idx = np.nonzero(tl == t)[0]
        if idx.size:
            assert tuple(ranges[t]) == (idx[0], idx[-1] + 1)
        else:
            assert tuple(ranges[t]) == (0, 0)


# ---------------------------------------------------------------------------
# compositing invariants
# ---------------------------------------------------------------------------

def _tile_lists(keys, vals, ranges):
    return [vals[s:e] for s, e in ranges]


def test_blend_weights_and_transmittance_invariants():
    cams = [scenes.pinhole(96, 64, 80.0)]
    sp = scenes.random_splats(600, cams, seed=7)
    res, keys, vals, ranges = O.render_splats(sp, 16, bg=(0.0, 0.0, 0.0))
    V, N = sp.radius.shape
    rows = torch.cat([torch.as_tensor(sp.xy.reshape(-1, 2), dtype=O.DT),
                      torch.as_tensor(sp.conic_opacity.reshape(-1, 4), dtype=O.DT),
                      torch.as_tensor(sp.rgb_depth.reshape(-1, 4)[:, :3], dtype=O.DT)], 1)
    cam = cams[0]
    TX, TY = O.tile_grid(cam, 16)
    for ty in range(TY):
        for tx in range(TX):
            s0, s1 = ranges[ty * TX + tx]
            idx = torch.as_tensor(vals[s0:s1].astype(np.int64))
            xx, yy = O._tile_pixels(cam, 16, tx, ty)
            C, T_fin, last, w, mask, _ = O._composite_tile(
                xx.to(O.DT) + 0.5, yy.to(O.DT) + 0.5, rows[idx], torch.zeros(3, dtype=O.DT), False)
            # sum of blend weights + final transmittance = 1
            np.testing.assert_allclose(w.sum(1).numpy() + T_fin.numpy(), 1.0, atol=1e-12)
            assert (T_fin.numpy() >= O.T_MIN).all()
            # colour bounded by the convex combination
            cmax = rows[idx][:, 6:9].max().item() if len(idx) else 0.0
            assert (C.numpy() <= cmax * (1 - T_fin.numpy()[:, None]) + 1e-12).all()
            assert (last.numpy() <= len(idx)).all()
            # transmittance before each list entry is non-increasing
            if len(idx):
                Tb = 1.0 - torch.cumsum(w, 1)
                assert (Tb[:, 1:] <= Tb[:, :-1] + 1e-15).all()


def test_index_permutation_invariance():
    cams = [scenes.pinhole(64, 48, 60.0)]
    sp = scenes.random_splats(200, cams, seed=11)
    res1, *_ = O.render_splats(sp, 16)
    perm = np.random.default_rng(0).permutation(200)
    sp2 = scenes.SplatSet(sp.xy[:, perm], sp.conic_opacity[:, perm], sp.rgb_depth[:, perm],
                          sp.radius[:, perm], cams)
    res2, *_ = O.render_splats(sp2, 16)
    np.testing.assert_allclose(res1[0]["image"], res2[0]["image"], atol=1e-14)


def test_disjoint_splats_order_invariance():
    # two splats far apart: swapping their depths leaves the image unchanged
    cams = [scenes.pinhole(64, 32, 60.0)]
    xy = np.array([[[12.0, 16.0], [50.0, 16.0]]], np.float32)
    co = np.array([[[0.5, 0.0, 0.5, 0.9], [0.3, 0.1, 0.4, 0.7]]], np.float32)
    rd1 = np.array([[[1.0, 0.2, 0.1, 2.0], [0.1, 0.9, 0.3, 3.0]]], np.float32)
    rd2 = rd1.copy()
    rd2[0, :, 3] = [3.0, 2.0]
    rad = np.array([[8, 8]], np.int32)
    a, *_ = O.render_splats(scenes.SplatSet(xy, co, rd1, rad, cams), 16)
    b, *_ = O.render_splats(scenes.SplatSet(xy, co, rd2, rad, cams), 16)
    np.testing.assert_allclose(a[0]["image"], b[0]["image"], atol=1e-15)


def test_two_overlapping_splats_closed_form():
    # two coincident isotropic splats at different depths: C = a1 c1 + (1-a1) a2 c2
    cams = [scenes.pinhole(32, 32, 60.0)]
    xy = np.array([[[16.0, 16.0], [16.0, 16.0]]], np.float32)
    co = np.array([[[0.05, 0.0, 0.05, 0.6], [0.02, 0.0, 0.02, 0.8]]], np.float32)
    rd = np.array([[[1.0, 0.0, 0.0, 3.0], [0.0, 1.0, 0.0, 2.0]]], np.float32)
    rad = np.array([[12, 12]], np.int32)
    res, *_ = O.render_splats(scenes.SplatSet(xy, co, rd, rad, cams), 16)
    img = res[0]["image"]
    for (i, j) in [(16, 16), (10, 20), (3, 29)]:
        d2 = (i + 0.5 - 16) ** 2 + (j + 0.5 - 16) ** 2
        a_front = min(0.99, float(np.float32(0.8)) * math.exp(-0.5 * float(np.float32(0.02)) * d2))
        a_back = min(0.99, float(np.float32(0.6)) * math.exp(-0.5 * float(np.float32(0.05)) * d2))
        fr = a_front if a_front >= 1 / 255 else 0.0
        bk = a_back if a_back >= 1 / 255 else 0.0
        expect = np.array([0, 1, 0]) * fr + (1 - fr) * bk * np.array([1, 0, 0])
        np.testing.assert_allclose(img[:, j, i], expect, atol=1e-13)


def test_early_termination_excludes_stopping_splat():
    # five opaque coincident splats: 1 - 0.99 = 0.01, 0.01^2 = 1e-4 (not below),
    # the third would give 1e-6 < 1e-4 and must not be composited
    cams = [scenes.pinhole(16, 16, 20.0)]
    n = 5
    xy = np.full((1, n, 2), 8.5, np.float32)
    co = np.tile(np.array([1e-4, 0.0, 1e-4, 1.0], np.float32), (1, n, 1))
    rd = np.zeros((1, n, 4), np.float32)
    rd[0, :, 3] = np.arange(1, n + 1)
    rd[0, :, 0] = [1.0, 0.5, 0.25, 0.125, 0.0625]
    rad = np.full((1, n), 3, np.int32)
    res, *_ = O.render_splats(scenes.SplatSet(xy, co, rd, rad, cams), 16)
    v = res[0]
    a = min(0.99, math.exp(-0.5 * float(np.float32(1e-4)) * 0.0))
    T2 = (1 - a) ** 2
    if T2 >= 1e-4:
        expect = a * 1.0 + (1 - a) * a * 0.5
        assert v["n_contrib"][8, 8] == 2
    np.testing.assert_allclose(v["image"][0, 8, 8], expect, atol=1e-13)
    np.testing.assert_allclose(v["T_final"][8, 8], T2, rtol=1e-12)


# ---------------------------------------------------------------------------
# gradients vs central finite differences
# ---------------------------------------------------------------------------

def _tiny_scene(seed, n=4, W=32, H=32, degree=3):
    g = scenes.random_cloud(n, degree, seed, box=((-0.4, 0.4), (-0.4, 0.4), (1.5, 2.5)),
                            log_scale_mu=-2.5, log_scale_sigma=0.3)
    rng = np.random.default_rng(seed + 100)
    cam = scenes.perturb_pose(scenes.Camera(np.eye(3), np.zeros(3), 40.0, 40.0, W / 2, H / 2, W, H),
                              rng, max_deg=3, max_m=0.05)
    return g, cam


def _loss(g, cam, wimg):
    res = O.render(g, [cam], with_mask=False)
    return float((res["views"][0]["image"] * wimg).sum())


def _set(g, group, idx, val):
    arrs = {k: getattr(g, k).astype(np.float64).copy() for k in
            ("means", "log_scales", "quats", "opacity_logits", "sh")}
    arrs[group][idx] = val
    return scenes.GaussianMap(arrs["means"], arrs["log_scales"], arrs["quats"],
                              arrs["opacity_logits"], arrs["sh"], g.sh_degree)


def _fd(fun, h):
    return (fun(h) - fun(-h)) / (2 * h)


@pytest.mark.parametrize("seed", [0, 1])
def test_param_gradients_vs_finite_differences(seed):
    g, cam = _tiny_scene(seed)
    rng = np.random.default_rng(seed + 7)
    wimg = rng.normal(size=(3, cam.height, cam.width))
    # float64 copies so the FD perturbation is not rounded away
    g64 = _set(g, "means", (0, 0), float(g.means[0, 0]))
    res = O.render(g64, [cam], dL_dimage=[wimg], with_mask=False)
    grads = res["grads"]
    checked = 0
    for group in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        arr = getattr(g64, group)
        for idx in np.ndindex(arr.shape):
            base = float(arr[idx])
            f = lambda h: _loss(_set(g64, group, idx, base + h), cam, wimg)
            d1 = _fd(f, 1e-6)
            d10 = _fd(f, 1e-5)
            if abs(d1 - d10) > 1e-4 * max(1.0, abs(d1)):
                continue  # a kink (tile edge, clamp, skip threshold) inside the stencil
            ga = float(grads[group][idx])
            assert abs(ga - d1) <= 1e-6 * max(1.0, abs(d1)) + 2e-7, (group, idx, ga, d1)
            checked += 1
    assert checked > 100


@pytest.mark.parametrize("seed", [0, 3])
def test_pose_gradient_vs_finite_differences(seed):
    g, cam = _tiny_scene(seed)
    rng = np.random.default_rng(seed + 9)
    wimg = rng.normal(size=(3, cam.height, cam.width))
    res = O.render(g, [cam], dL_dimage=[wimg], with_mask=False)
    gx = res["grads"]["xi"][0]

    def moved(k, h):
        xi = np.zeros(6)
        xi[k] = h
        T = O.se3_exp(torch.as_tensor(xi)).numpy()
        return scenes.Camera(T[:3, :3] @ cam.R, T[:3, :3] @ cam.t + T[:3, 3], cam.fx, cam.fy,
                             cam.cx, cam.cy, cam.width, cam.height)

    for k in range(6):
        f = lambda h: _loss(g, moved(k, h), wimg)
        d1 = _fd(f, 1e-6)
        d10 = _fd(f, 1e-5)
        assert abs(d1 - d10) <= 1e-4 * max(1.0, abs(d1))
        assert abs(gx[k] - d1) <= 1e-6 * max(1.0, abs(d1)) + 2e-7, (k, gx[k], d1)


def test_pose_translation_equals_moving_all_means():
    # t <- t + rho moves every camera-frame point by rho, as does mu <- mu + R^T rho
    # (the SH view direction depends only on the camera-frame point), so
    # dL/drho = R sum_g dL/dmu_g.
    g, cam = _tiny_scene(4, n=5)
    wimg = np.random.default_rng(3).normal(size=(3, cam.height, cam.width))
    res = O.render(g, [cam], dL_dimage=[wimg], with_mask=False)
    gm = res["grads"]["means"].sum(axis=1)
    np.testing.assert_allclose(res["grads"]["xi"][0][:3], np.asarray(cam.R) @ gm, rtol=1e-10, atol=1e-13)


# ---------------------------------------------------------------------------
# loss gradient and Adam
# ---------------------------------------------------------------------------

def test_l1_grad_sign_and_scale():
    img = np.array([[[0.5, 0.2], [0.1, 0.9]]] * 3)
    tgt = np.array([[[0.4, 0.2], [0.3, 0.1]]] * 3)
    L, g = O.l1_loss_grad(img, tgt)
    np.testing.assert_allclose(L, (0.1 + 0 + 0.2 + 0.8) / 4)
    np.testing.assert_array_equal(g[0], np.array([[1, 0], [-1, 1]]) / 12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    lr, eps = 0.01, 1e-15
    p1, m1, v1 = O.adam_step(p, g, np.zeros(100), np.zeros(100), lr, 0.9, 0.999, eps, 1)
    # step 1: m_hat = g, v_hat = g^2 -> p - lr g / (|g| + eps)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-14)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-14)
    mask = (np.arange(100) % 3 == 0).astype(np.uint8)
    p2, m2, v2 = O.adam_step(p, g, np.zeros(100), np.zeros(100), lr, 0.9, 0.999, eps, 1, mask)
    np.testing.assert_array_equal(p2[mask == 0], p[mask == 0])
    np.testing.assert_allclose(p2[mask == 1], p1[mask == 1])


def test_alpha_band_covers_float32_exponent_rounding():
    """The near-threshold band on the alpha decisions (relative BAND_REL plus
    BAND_TERMS times |Q00| dx^2 + 2 |Q01 dx dy| + |Q11| dy^2) bounds the
    relative error of o e^power when the exponent is evaluated in float32 by
    either association of its terms, for splats elongated up to 40:1 sampled
    far along their major axis where the terms cancel most."""
    rng = np.random.default_rng(7)
    f32 = np.float32
    l2e = f32(1.4426950408889634)
    worst = 0.0
    for _ in range(2000):
        s1, s2 = np.exp(rng.uniform(np.log(0.6), np.log(24.0), 2))
        th = rng.uniform(0, np.pi)
        cs, sn = np.cos(th), np.sin(th)
        i1, i2 = 1 / s1 ** 2, 1 / s2 ** 2
        q = np.array([cs * cs * i1 + sn * sn * i2, cs * sn * (i1 - i2), sn * sn * i1 + cs * cs * i2],
                     np.float32)
        mx, my = rng.uniform(0, 1200, 2).astype(np.float32)
        major = (cs, sn) if s1 > s2 else (-sn, cs)
        t = rng.uniform(-3, 3) * max(s1, s2)
        px = f32(np.floor(mx + t * major[0]) + 0.5)
        py = f32(np.floor(my + t * major[1]) + 0.5)
        dx, dy = f32(px - mx), f32(py - my)
        a, b, c = f32(-0.5) * l2e * q[0], -l2e * q[1], f32(-0.5) * l2e * q[2]
        fma = lambda x, y, z: f32(np.float64(x) * np.float64(y) + np.float64(z))
        p_a = fma(dx, fma(a, dx, b * dy), (c * dy) * dy)
        p_b = fma(dy, fma(c, dy, b * dx), (a * dx) * dx)
        dx64, dy64 = np.float64(px) - np.float64(mx), np.float64(py) - np.float64(my)
        q64 = q.astype(np.float64)
        exact = -0.5 * (q64[0] * dx64 ** 2 + 2 * q64[1] * dx64 * dy64 + q64[2] * dy64 ** 2)
        terms = abs(q64[0]) * dx64 ** 2 + 2 * abs(q64[1] * dx64 * dy64) + abs(q64[2]) * dy64 ** 2
        band = O.BAND_REL + O.BAND_TERMS * terms
        for p in (p_a, p_b):
            rel = abs(np.expm1(np.float64(p) / 1.4426950408889634 - exact))
            worst = max(worst, rel / band)
            assert rel <= band, (rel, band, terms)
    assert worst > 0.01, worst   # the bound is exercised, not vacuous


# ---------------------------------------------------------------------------
# off-axis EWA Jacobian and the camera rotation of Sigma
# ---------------------------------------------------------------------------

def _rot_from_quat_scipy(q_wxyz):
    from scipy.spatial.transform import Rotation
    w, x, y, z = q_wxyz
    return Rotation.from_quat([x, y, z, w]).as_matrix()      # scipy orders (x, y, z, w)


def test_ewa_covariance_matches_finite_difference_jacobian():
    """Sigma' of project_view equals J Wc Sigma Wc^T J^T + 0.3 I with J taken
    from central differences of the pinhole map p -> (fx x/z + cx, fy y/z + cy),
    at off-axis points under a rotated camera.  Inside the 1.3 guard the
    Jacobian is the map's own; outside it, the map's Jacobian at the camera
    point moved onto the guard (x/z, y/z clamped, z kept).  Sigma comes from
    scipy's rotation of the quaternion.  A sign flip in the x/z (y/z) column,
    a missing clamp or Wc^T Sigma Wc in place of Wc Sigma Wc^T fails here."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(12)
    W, H, fx, fy, cx, cy = 320, 240, 260.0, 250.0, 150.0, 130.0
    Wc = Rotation.from_rotvec([0.3, -0.5, 0.2]).as_matrix()
    tc = np.array([0.2, -0.1, 0.4])
    n = 60
    # camera-frame points: x/z, y/z spread to 2.2x the guard limits
    lx, ly = 1.3 * W / (2 * fx), 1.3 * H / (2 * fy)
    z = rng.uniform(1.0, 5.0, n)
    p = np.stack([rng.uniform(-2.2, 2.2, n) * lx * z, rng.uniform(-2.2, 2.2, n) * ly * z, z])
    mu = Wc.T @ (p - tc[:, None])
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0)
    ls = rng.normal(-2.0, 0.6, size=(3, n))
    P = O.project_view(torch.as_tensor(mu), torch.as_tensor(ls), torch.as_tensor(q),
                       torch.zeros(n, dtype=torch.float64), torch.zeros((3, 1, n), dtype=torch.float64),
                       0, torch.as_tensor(Wc), torch.as_tensor(tc),
                       scenes.Camera(Wc, tc, fx, fy, cx, cy, W, H))
    conic = P["conic"].numpy()

    def proj(pt):
        return np.array([fx * pt[0] / pt[2] + cx, fy * pt[1] / pt[2] + cy])

    inside = 0
    for i in range(n):
        tx = np.clip(p[0, i] / p[2, i], -lx, lx)
        ty = np.clip(p[1, i] / p[2, i], -ly, ly)
        inside += (abs(p[0, i] / p[2, i]) < lx) and (abs(p[1, i] / p[2, i]) < ly)
        base = np.array([tx * p[2, i], ty * p[2, i], p[2, i]])
        J = np.zeros((2, 3))
        for k in range(3):
            h = 1e-5 * p[2, i]
            e = np.zeros(3)
            e[k] = h
            J[:, k] = (proj(base + e) - proj(base - e)) / (2 * h)
        Rq = _rot_from_quat_scipy(q[:, i])
        S = Rq @ np.diag(np.exp(2 * ls[:, i])) @ Rq.T
        Sp = J @ Wc @ S @ Wc.T @ J.T + 0.3 * np.eye(2)
        a, b, c = conic[i]
        got = np.linalg.inv(np.array([[a, b], [b, c]]))
        np.testing.assert_allclose(got, Sp, rtol=1e-7, atol=1e-9 * np.abs(Sp).max(), err_msg=str(i))
    assert 5 < inside < n - 5          # both branches of the guard are exercised


def test_render_is_equivariant_under_camera_rotation():
    """At SH degree 0 (view-independent colour) the map seen from (R, t)
    renders exactly like the rotated map (mu -> R mu, q -> q_R (x) q) seen from
    (I, t): both put every Gaussian at the same camera-frame point with the
    same camera-frame covariance R Sigma R^T.  A camera rotation applied as
    R^T Sigma R breaks this."""
    from scipy.spatial.transform import Rotation
    gmap = scenes.random_cloud(400, 0, seed=13, box=((-1.5, 1.5), (-1.0, 1.0), (2.0, 5.0)))
    Rc = Rotation.from_rotvec([0.25, -0.35, 0.15]).as_matrix()
    t = np.array([0.1, -0.05, 0.3])
    # a map whose camera-frame points under (Rc, t) equal gmap's under (I, t)
    mu_a = Rc.T @ gmap.means.astype(np.float64)
    qa = np.stack([_hamilton(_quat_of(Rc.T), gmap.quats[:, i].astype(np.float64))
                   for i in range(gmap.n)], 1)
    rot = scenes.GaussianMap(mu_a, gmap.log_scales.astype(np.float64), qa,
                             gmap.opacity_logits.astype(np.float64), gmap.sh.astype(np.float64), 0)
    W, H, f = 96, 72, 80.0
    cam_r = scenes.Camera(Rc, t, f, f, W / 2, H / 2, W, H)
    cam_i = scenes.Camera(np.eye(3), t, f, f, W / 2, H / 2, W, H)
    a = O.render(rot, [cam_r], bg=(0.1, 0.2, 0.3))
    b = O.render(gmap, [cam_i], bg=(0.1, 0.2, 0.3))
    m = ~(a["views"][0]["mask"] | b["views"][0]["mask"])
    assert m.mean() > 0.95
    np.testing.assert_allclose(a["views"][0]["image"][:, m], b["views"][0]["image"][:, m], atol=1e-10)
    np.testing.assert_allclose(a["proj"][0]["conic"], b["proj"][0]["conic"], rtol=1e-9, atol=1e-12)


def _quat_of(R):
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(R).as_quat()
    return np.array([w, x, y, z])


# ---------------------------------------------------------------------------
# per-Gaussian rendering error (selective optimisation)
# ---------------------------------------------------------------------------

def _covered_pixels(u, v, r, W, H, ts=16):
    """Pixels of the tiles that hold a pixel centre inside [u +- r] x [v +- r],
    by enumeration."""
    tiles = set()
    for j in range(H):
        for i in range(W):
            if abs(i + 0.5 - u) <= r and abs(j + 0.5 - v) <= r:
                tiles.add((j // ts, i // ts))
    cov = np.zeros((H, W), bool)
    for (ty, tx) in tiles:
        cov[ty * ts:(ty + 1) * ts, tx * ts:(tx + 1) * ts] = True
    return cov


@pytest.mark.parametrize("s,z,o_logit,W,H", [(0.2, 3.0, 1.0, 32, 24), (0.03, 2.0, 2.5, 80, 64)])
def test_render_error_single_gaussian_closed_form(s, z, o_logit, W, H):
    """One on-axis isotropic Gaussian, black background, black target: the
    render is c alpha(u), so E = sum_c c_c * sum over covered pixels of
    alpha(u)^2, with alpha(u) = min(0.99, o exp(-|d|^2 / (2 var))) where at
    least 1/255, var = (f s / z)^2 + 0.3."""
    f = 100.0
    f0 = [0.7, -0.3, 1.2]
    g, cam = _single(np.float32(s), np.float32(z), f, W, H, o_logit, f0)
    s, z = math.exp(float(g.log_scales[0, 0])), float(np.float32(z))
    o = 1 / (1 + math.exp(-float(np.float32(o_logit))))
    var = (f * s / z) ** 2 + 0.3
    r = math.ceil(3 * math.sqrt(var))
    c = np.maximum(np.asarray(g.sh[:, 0, 0], np.float64) * 0.5 / math.sqrt(math.pi) + 0.5, 0.0)
    cov = _covered_pixels(W / 2, H / 2, r, W, H)
    jj, ii = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    a = np.minimum(0.99, o * np.exp(-((ii - W / 2) ** 2 + (jj - H / 2) ** 2) / (2 * var)))
    a = np.where((a >= 1 / 255) & cov, a, 0.0)
    expect = c.sum() * (a * a).sum()
    res = O.render_error(g, [cam], [np.zeros((3, H, W))])
    np.testing.assert_allclose(res["err"][0, 0], expect, rtol=1e-12)
    np.testing.assert_allclose(res["weight"][0, 0], a.sum(), rtol=1e-12)


def test_render_error_occlusion_two_gaussians():
    """A splat behind another on the axis: its weight is alpha_b (1 - alpha_f)
    per pixel, and with target t the residual is |c_f a_f + c_b a_b (1 - a_f) - t|
    summed over channels (black background, every pixel covered)."""
    W, H, f = 32, 24, 100.0
    g = scenes.GaussianMap(
        means=np.array([[0.0, 0.0], [0.0, 0.0], [3.0, 4.0]], np.float32),
        log_scales=np.log(np.array([[0.25, 0.35]] * 3, np.float32)),
        quats=np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0]], np.float32),
        opacity_logits=np.array([0.3, 1.5], np.float32),
        sh=np.array([[0.4, -0.6], [0.1, 0.9], [-1.0, 0.5]], np.float32).reshape(3, 1, 2), sh_degree=0)
    cam = scenes.Camera(np.eye(3), np.zeros(3), f, f, W / 2, H / 2, W, H)
    rng = np.random.default_rng(3)
    tgt = rng.random((3, H, W))
    jj, ii = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    alph, col = [], []
    for k in range(2):
        s = math.exp(float(g.log_scales[0, k]))
        z = float(g.means[2, k])
        var = (f * s / z) ** 2 + 0.3
        assert math.ceil(3 * math.sqrt(var)) >= W / 2   # the rectangle covers the image
        o = 1 / (1 + math.exp(-float(g.opacity_logits[k])))
        a = np.minimum(0.99, o * np.exp(-((ii - W / 2) ** 2 + (jj - H / 2) ** 2) / (2 * var)))
        alph.append(np.where(a >= 1 / 255, a, 0.0))
        col.append(np.maximum(g.sh[:, 0, k].astype(np.float64) * 0.5 / math.sqrt(math.pi) + 0.5, 0))
    wf, wb = alph[0], alph[1] * (1 - alph[0])
    img = col[0][:, None, None] * wf + col[1][:, None, None] * wb
    e = np.abs(img - tgt).sum(axis=0)
    res = O.render_error(g, [cam], [tgt])
    np.testing.assert_allclose(res["err"][0], [(wf * e).sum(), (wb * e).sum()], rtol=1e-11)
    np.testing.assert_allclose(res["images"][0], img, atol=1e-12)


def test_render_error_weights_sum_to_coverage():
    """Summed over the Gaussians, E_k equals sum_u (1 - T_final(u)) e(u): the
    blending weights of a pixel add up to one minus its final transmittance
    (random cloud, two views, background and a random target)."""
    gmap = scenes.random_cloud(300, 0, seed=5)
    cams = [scenes.pinhole(64, 48, 60.0),
            scenes.perturb_pose(scenes.pinhole(48, 40, 50.0), np.random.default_rng(6))]
    rng = np.random.default_rng(7)
    tg = [rng.random((3, c.height, c.width)) for c in cams]
    res = O.render_error(gmap, cams, tg, bg=(0.2, 0.1, 0.3))
    for k in range(2):
        e = np.abs(res["images"][k] - tg[k]).sum(axis=0)
        np.testing.assert_allclose(res["err"][k].sum(), ((1 - res["T_final"][k]) * e).sum(), rtol=1e-10)
        np.testing.assert_allclose(res["weight"][k].sum(), (1 - res["T_final"][k]).sum(), rtol=1e-10)
    m = O.active_set(res["err"], float(np.median(res["err"].max(axis=0))))
    assert 0 < m.sum() < gmap.n
    always = np.zeros(gmap.n, np.uint8)
    always[:7] = 1
    m2 = O.active_set(res["err"], 1e30, always)
    np.testing.assert_array_equal(m2, always.astype(bool))


# ---------------------------------------------------------------------------
# global stage: insertion, isotropic regulariser, pruning
# ---------------------------------------------------------------------------

def test_iso_loss_closed_form():
    """Scales (a, a, b) with a > b: the three deviations from the mean are
    (a-b)/3, (a-b)/3, -2(a-b)/3, so E = weight/(3n) * 4(a-b)/3 for that
    Gaussian, and dE/dlog s = s * weight/(3n) * (sgn - mean sgn): 2/3 on the
    two large axes, -4/3 on the small one.  An isotropic Gaussian adds 0."""
    a, b, w = 0.3, 0.1, 10.0
    ls = np.log(np.array([[a, 0.2], [a, 0.2], [b, 0.2]]))
    E, g = O.iso_loss_grad(ls, w)
    c = w / (3 * 2)
    assert abs(E - c * 4 * (a - b) / 3) < 1e-15
    np.testing.assert_allclose(g[:, 0], [a * c * 2 / 3, a * c * 2 / 3, -b * c * 4 / 3], rtol=1e-12)
    np.testing.assert_allclose(g[:, 1], 0.0, atol=1e-17)


def test_insert_appends_the_local_map_at_opacity_0_2():
    gm = scenes.random_cloud(7, 1, seed=1)
    lm = scenes.random_cloud(4, 1, seed=2)
    arrs, new = O.insert(gm, lm)
    for k, (out, a, b) in enumerate(zip(arrs, gm.arrays(), lm.arrays())):
        assert out.shape[-1] == 11
        np.testing.assert_array_equal(out[..., :7], a)
        if k != 3:
            np.testing.assert_array_equal(out[..., 7:], b)
    np.testing.assert_allclose(1 / (1 + np.exp(-arrs[3][7:])), 0.2, rtol=1e-15)
    np.testing.assert_array_equal(new, [0] * 7 + [1] * 4)


def test_prune_keeps_opacity_at_least_0_7():
    lg = np.log(0.7 / 0.3)
    x = np.array([lg - 1e-9, lg + 1e-9, -3.0, 3.0, 0.0])
    np.testing.assert_array_equal(O.prune_keep(x), [False, True, False, True, False])


def test_pose_step_first_adam_step_closed_form():
    """First Adam step: m_hat / sqrt(v_hat) = sign(g), so the tangent step is
    -lr sign(g) per component.  A pure rho gradient then translates the camera
    by exactly that; a pure phi gradient about z rotates it by lr about z
    (rotating t with it)."""
    R = np.eye(3)
    t = np.array([0.3, -0.2, 1.0])
    z6 = np.zeros(6)
    Rn, tn, _, _ = O.pose_adam_step(R, t, [2.0, -1e-3, 0, 0, 0, 0], z6, z6, 0.01, 0.02, 0.9, 0.999,
                                    1e-15, 1)
    np.testing.assert_allclose(Rn, R, atol=1e-15)
    np.testing.assert_allclose(tn, t + [-0.01, 0.01, 0.0], atol=1e-13)
    Rn, tn, _, _ = O.pose_adam_step(R, t, [0, 0, 0, 0, 0, -5.0], z6, z6, 0.01, 0.02, 0.9, 0.999, 1e-15,
                                    1)
    c, s_ = math.cos(0.02), math.sin(0.02)
    Rz = np.array([[c, -s_, 0], [s_, c, 0], [0, 0, 1]])
    np.testing.assert_allclose(Rn, Rz, atol=1e-14)
    np.testing.assert_allclose(tn, Rz @ t, atol=1e-14)


def test_gradient_term_mass_bounds_the_gradient():
    """The term mass of a gradient element is at least its magnitude
    (triangle inequality), with equality when no term cancels: a lone
    Gaussian's opacity logit under a positive dL/dC on a black background
    (every pixel adds dC/do > 0)."""
    W, H, f = 48, 40, 60.0
    g, cam = _single(np.float32(0.1), np.float32(3.0), f, W, H, 0.4, [0.5, 0.2, 0.9])
    dl = [np.full((3, H, W), 1e-3)]
    res = O.render(g, [cam], dL_dimage=dl)
    mass, walk = O.gradient_term_mass(g, [cam], dl, [0])
    go = res["grads"]["opacity_logits"][0]
    assert go > 0
    np.testing.assert_allclose(mass["opacity_logits"][0, 0], go, rtol=1e-12)
    assert walk == 1
    # a random cloud: mass >= |grad| for every parameter of the listed Gaussians
    gm = scenes.random_cloud(200, 1, seed=3)
    cams = [scenes.pinhole(64, 48, 60.0)]
    rng = np.random.default_rng(4)
    dl = [rng.normal(size=(3, 48, 64)) * 1e-3]
    res = O.render(gm, cams, dL_dimage=dl)
    ids = [int(i) for i in np.nonzero(res["proj"][0]["visible"])[0][:12]]
    mass, walk = O.gradient_term_mass(gm, cams, dl, ids)
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        gk = res["grads"][k].reshape(-1, gm.n)[:, ids].T
        assert (mass[k] >= np.abs(gk) * (1 - 1e-9) - 1e-18).all(), k
    assert walk >= 1
