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
