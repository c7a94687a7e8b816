"""Pins of the initialiser oracle (CPU only)."""
import math

import numpy as np
import torch

from oracle import nn_oracle as N
from paper_2409_09295_amd import scenes


def test_conv3x3_matches_torch_conv2d():
    rng = np.random.default_rng(0)
    x = torch.as_tensor(rng.normal(size=(2, 7, 9, 5)))
    w = torch.as_tensor(rng.normal(size=(9, 4, 5)))
    b = torch.as_tensor(rng.normal(size=4))
    ours = N.conv3x3(x, w, b)
    # library routine: NCHW cross-correlation with a [cout, cin, 3, 3] kernel
    k = w.reshape(3, 3, 4, 5).permute(2, 3, 0, 1)
    ref = torch.nn.functional.conv2d(x.permute(0, 3, 1, 2), k, b, padding=1).permute(0, 2, 3, 1)
    torch.testing.assert_close(ours, ref, rtol=1e-12, atol=1e-12)


def test_pool_and_upsample_are_adjoint_up_to_four():
    rng = np.random.default_rng(1)
    x = torch.as_tensor(rng.normal(size=(1, 6, 8, 3)))
    y = torch.as_tensor(rng.normal(size=(1, 3, 4, 3)))
    # <pool(x), y> = <x, up(y)> / 4
    lhs = (N.avgpool2(x) * y).sum()
    rhs = (x * N.upsample2(y)).sum() / 4
    assert abs(float(lhs - rhs)) < 1e-12


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159], np.float32)
    r = N.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0            # tie rounds to even
    assert r[2] == 1.0 + 2 ** -7   # above the tie rounds up
    assert r[3] == -2.5
    assert abs(r[4] - 3.140625) < 1e-12


def test_cost_volume_size_is_the_papers_4_7_mb():
    # 640 x 480 at 1/4 resolution, 64 hypotheses, float32 (Sec. III-A1)
    nbytes = N.N_HYP * (480 // 4) * (640 // 4) * 4
    assert round(nbytes / 2 ** 20, 1) == 4.7


def test_hypotheses_are_evenly_spaced():
    h = N.hypotheses()
    assert h[0] == 0.25 and abs(h[-1] - 25.0) < 1e-12 and len(h) == 64
    np.testing.assert_allclose(np.diff(h), (25 - 0.25) / 63)


def test_cost_volume_fronto_parallel_plane_recovers_depth():
    """A textured plane at depth D seen by a translating camera: the cost at
    the hypothesis nearest D is ~0 and WTA picks it."""
    W, H, f = 128, 96, 100.0
    D = N.hypotheses()[5]               # a depth exactly on the grid (2.21 m)
    rng = np.random.default_rng(3)
    tex = rng.random((3, 64, 64))

    def render_plane(cam_x):
        # pixel centre -> ray -> plane z = D in world (camera looks along +z)
        jj, ii = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
        X = (ii - W / 2) / f * D + cam_x
        Y = (jj - H / 2) / f * D
        # smooth periodic texture on the plane
        u = (X * 8) % 64
        v = (Y * 8) % 64
        img = np.zeros((3, H, W))
        for c in range(3):
            img[c] = 0.5 + 0.25 * np.sin(X * 6.0 + c) + 0.25 * np.cos(Y * 4.6 - c)
        return img

    xs = [-0.1 * k for k in range(7, -1, -1)]    # reference (last) at x = 0
    imgs = [render_plane(x) for x in xs]
    cams = [scenes.Camera(np.eye(3), np.array([-x, 0.0, 0.0]), f, f, W / 2, H / 2, W, H) for x in xs]
    cost = N.cost_volume(imgs, cams)
    d = N.wta_depth(cost)
    inner = d[4:-4, 4:-4]
    assert np.mean(np.abs(inner - D) < 1e-9) > 0.9


def test_head_hand_computed():
    """1x1 head on two pixels with three features: out[n, k, y, x] =
    sum_c f[n, y, x, c] w[k, c] + b[k], worked by hand; the output layout is
    [n, 2, h, w]."""
    f = torch.tensor([[[[1.0, 2.0, 3.0], [-1.0, 0.0, 0.5]]]], dtype=torch.float64)   # [1, 1, 2, 3]
    w = torch.tensor([[0.5, -1.0, 2.0], [1.0, 1.0, 1.0]], dtype=torch.float64)
    b = torch.tensor([0.25, -3.0], dtype=torch.float64)
    out = N.head(f, w, b)
    assert out.shape == (1, 2, 1, 2)
    np.testing.assert_allclose(out[0, :, 0, :].numpy(), [[4.75, 0.75], [3.0, -3.5]], atol=1e-15)


def test_depth_loss_hand_computed():
    """Three pixels, one without depth; fx = e^2 so log(d / fx) = log d - 2:
    residuals (0.5, 0.25) and (0.25, -0.5) give a mean of 0.75 over the two
    valid pixels, and gradients +-1/2 there, 0 at the invalid one."""
    e = math.e
    depth = torch.tensor([[[e, 0.0, 1.0]]], dtype=torch.float64)               # [1, 1, 3]
    pred = torch.tensor([[[[1.5, 7.0, 0.25]], [[-1.25, 9.0, -2.5]]]], dtype=torch.float64,
                        requires_grad=True)                                      # [1, 2, 1, 3]
    L = N.depth_loss(pred, depth, e * e)
    assert abs(float(L.detach()) - 0.75) < 1e-14
    L.backward()
    np.testing.assert_allclose(pred.grad[0, :, 0].numpy(), [[0.5, 0.0, 0.5], [-0.5, 0.0, -0.5]],
                               atol=1e-15)


def test_unet_forward_matches_library_layers():
    """The whole network against the same architecture assembled from
    torch.nn.functional library layers in NCHW (conv2d with padding 1,
    avg_pool2d, nearest interpolate, cat, relu, a 1x1 conv2d head)."""
    F = torch.nn.functional
    rng = np.random.default_rng(7)
    ch = (4, 8, 8, 16)
    p = {}
    for name, cin, cout in N.unet_layers(8, ch):
        p[name + ".w"] = torch.as_tensor(rng.normal(size=(9, cout, cin)) / math.sqrt(9 * cin))
        p[name + ".b"] = torch.as_tensor(rng.normal(size=cout) * 0.1)
    p["head.w"] = torch.as_tensor(rng.normal(size=(2, ch[0])))
    p["head.b"] = torch.as_tensor(rng.normal(size=2))
    x = torch.as_tensor(rng.normal(size=(2, 16, 24, 8)))
    ours = N.unet_forward(x, p)

    def conv(name, t):
        w = p[name + ".w"]
        k = w.reshape(3, 3, w.shape[1], w.shape[2]).permute(2, 3, 0, 1)
        return F.relu(F.conv2d(t, k, p[name + ".b"], padding=1))

    up = lambda t: F.interpolate(t, scale_factor=2, mode="nearest")
    xc = x.permute(0, 3, 1, 2)
    e0 = conv("e0b", conv("e0a", xc))
    e1 = conv("e1b", conv("e1a", F.avg_pool2d(e0, 2)))
    e2 = conv("e2b", conv("e2a", F.avg_pool2d(e1, 2)))
    e3 = conv("e3b", conv("e3a", F.avg_pool2d(e2, 2)))
    d2 = conv("d2b", conv("d2a", torch.cat([up(e3), e2], 1)))
    d1 = conv("d1b", conv("d1a", torch.cat([up(d2), e1], 1)))
    d0 = conv("d0b", conv("d0a", torch.cat([up(d1), e0], 1)))
    ref = F.conv2d(d0, p["head.w"][:, :, None, None], p["head.b"])
    torch.testing.assert_close(ours, ref, rtol=1e-10, atol=1e-10)


def test_bp_without_smoothness_is_winner_take_all():
    rng = np.random.default_rng(11)
    cost = rng.random((16, 7, 9))
    cost[:, 2, 3] = np.inf
    labels, _ = N.belief_propagation(cost, lam=0.0, trunc=0.0, iters=5)
    D = np.where(np.isfinite(cost), cost, N.BP_INVALID)
    np.testing.assert_array_equal(labels, np.argmin(D, axis=0))


def _chain_map(D, lam, trunc):
    """Exact minimum-energy labelling of a chain by dynamic programming."""
    L, n = D.shape
    S = np.minimum(lam * np.abs(np.arange(L)[:, None] - np.arange(L)[None, :]), trunc)
    acc = D[:, 0].copy()
    back = np.zeros((L, n), int)
    for x in range(1, n):
        tot = acc[:, None] + S                     # [previous label, label]
        back[:, x] = np.argmin(tot, axis=0)
        acc = tot.min(axis=0) + D[:, x]
    lab = np.zeros(n, int)
    lab[-1] = int(np.argmin(acc))
    for x in range(n - 1, 0, -1):
        lab[x - 1] = back[lab[x], x]
    return lab, acc.min()


def test_bp_on_a_chain_reaches_the_exact_map():
    """On a tree (a one-row image) min-sum belief propagation is exact once
    messages have crossed the chain: labels equal the dynamic-programming
    minimum of the same energy (data plus truncated linear smoothness)."""
    rng = np.random.default_rng(12)
    L, n = 12, 9
    D = rng.random((L, n)) * 0.3
    lam, trunc = 0.05, 0.2
    labels, belief = N.belief_propagation(D[:, None, :], lam=lam, trunc=trunc, iters=n + 1)
    ref, energy = _chain_map(D, lam, trunc)
    np.testing.assert_array_equal(labels[0], ref)
    # every belief's minimum is the minimum energy, up to the message shifts:
    # the chosen labelling's energy equals the exact minimum
    S = np.minimum(lam * np.abs(np.arange(L)[:, None] - np.arange(L)[None, :]), trunc)
    e = D[labels[0], np.arange(n)].sum() + sum(S[labels[0][x], labels[0][x + 1]] for x in range(n - 1))
    assert abs(e - energy) < 1e-12


def test_bp_smooths_an_outlier():
    """A constant-depth field with one pixel whose data prefer a far label by
    a margin smaller than the smoothness it would break: BP restores the
    neighbours' label, winner-take-all keeps the outlier."""
    L, H, W = 10, 5, 5
    D = np.full((L, H, W), 0.5)
    D[3] = 0.1
    D[8, 2, 2], D[3, 2, 2] = 0.05, 0.12
    labels, _ = N.belief_propagation(D, lam=0.05, trunc=0.3, iters=10)
    assert (labels == 3).all()
    assert np.argmin(D[:, 2, 2]) == 8


def test_bf16_store_rounds_values_and_gradients():
    """The storage rounding used by the network oracle agrees with the
    bit-level round-to-nearest-even of bf16_round, forward and backward, and
    leaves values already in bfloat16 unchanged."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal(4096) * 10.0 ** rng.integers(-3, 3, 4096)
    w = rng.standard_normal(4096)
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    y = N.bf16_store(xt)
    np.testing.assert_array_equal(y.detach().numpy(), N.bf16_round(x))
    (y * torch.tensor(w)).sum().backward()
    np.testing.assert_array_equal(xt.grad.numpy(), N.bf16_round(w))
    z = torch.tensor(N.bf16_round(x))
    np.testing.assert_array_equal(N.bf16_store(z).numpy(), z.numpy())
