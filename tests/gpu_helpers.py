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


def assert_grad_close(name, g, ref, rel=1e-3, floor=1e-3):
    """GPU gradient vs the FP64 oracle, the parity contract for gradients:
    per element |g - ref| <= rel * max(|ref|, floor * max|ref|) and, over the
    group, ||g - ref||_2 <= rel ||ref||_2.  The floor (1e-3 of the group's
    largest magnitude) covers elements that are sums of cancelling per-pixel
    terms, whose float32 value carries the summation's rounding of the terms
    rather than 1e-3 of its own (tiny) size.  Prints the worst element's
    ratio to its tolerance and the smallest floor that would have passed."""
    g = np.asarray(g, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    scale = np.abs(ref).max() if ref.size else 0.0
    if scale == 0.0:
        assert np.abs(g).max() == 0.0 if g.size else True, name
        return 0.0
    tol = rel * np.maximum(np.abs(ref), floor * scale)
    err = np.abs(g - ref)
    bad = err > tol
    l2 = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    worst = int(np.argmax(err / tol))
    need = float(np.max(err / (rel * scale)))   # floor under which every element passes
    print(f"  {name}: rel L2 {l2:.2e}, worst err/tol {err[worst] / tol[worst]:.3f}, "
          f"floor needed {need:.1e} (contract {floor:.0e})", flush=True)
    msg = (f"{name}: {bad.sum()} of {g.size} elements outside tolerance; relative L2 {l2:.3e}; "
           f"worst index {worst}: gpu {g[worst]:.6e} ref {ref[worst]:.6e} tol {tol[worst]:.3e}")
    assert not bad.any(), msg
    assert l2 <= rel, msg
    return l2


def assert_same_up_to_order(name, a, b, rel=1e-5, atol_frac=1e-5):
    """Two GPU results that differ only in the float32 order of their atomic
    additions: |a - b| <= rel |b| + atol_frac max|b| per element."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    scale = np.abs(b).max() if b.size else 0.0
    if scale == 0.0:
        assert np.abs(a).max() == 0.0 if a.size else True, name
        return
    err = np.abs(a - b)
    tol = rel * np.abs(b) + atol_frac * scale
    worst = int(np.argmax(err / tol))
    assert (err <= tol).all(), (f"{name}: {(err > tol).sum()} of {a.size} elements differ; worst "
                                f"index {worst}: {a[worst]:.6e} vs {b[worst]:.6e}")
