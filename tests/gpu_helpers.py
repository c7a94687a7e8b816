"""Helpers shared by the GPU parity tests (comparison and upload utilities)."""
import numpy as np
import torch


def u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def np_(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def random_dl(views_sizes, seed: int) -> np.ndarray:
    """Seeded dL/dimage, packed [V][3][H][W], scaled like a mean-reduced loss."""
    rng = np.random.default_rng(seed)
    parts = []
    for (w, h) in views_sizes:
        parts.append((rng.normal(size=(3, h, w)) / (3.0 * w * h)).reshape(-1))
    return np.concatenate(parts).astype(np.float32)


def assert_grad_close(name, g, ref, rel=1e-3, atol_frac=1e-5):
    """Elementwise |g - ref| <= rel |ref| + atol_frac max|ref|, and the group's
    ||g - ref||_2 <= rel ||ref||_2.  The absolute floor covers float32
    summation roundoff in elements whose per-pixel contributions cancel
    (their exact value is orders of magnitude below the group's largest)."""
    g = np.asarray(g, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    scale = np.abs(ref).max() if ref.size else 0.0
    if scale == 0.0:
        assert np.abs(g).max() == 0.0 if g.size else True, name
        return
    tol = rel * np.abs(ref) + atol_frac * scale
    err = np.abs(g - ref)
    bad = err > tol
    l2 = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    worst = int(np.argmax(err / tol))
    msg = (f"{name}: {bad.sum()} of {g.size} elements outside tolerance; relative L2 {l2:.3e}; "
           f"worst index {worst}: gpu {g[worst]:.6e} ref {ref[worst]:.6e} tol {tol[worst]:.3e}")
    assert not bad.any(), msg
    assert l2 <= rel, msg
    return l2
