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


U32 = 2.0 ** -24   # float32 unit roundoff


def term_mass(gmap, cams, dls, tiles=None, bg=(0.0, 0.0, 0.0)):
    """mass_fn for assert_grad_close: the oracle's absolute first-order mass
    of the per-pixel terms of given gradient elements, and the longest list
    walk among their pixels."""
    from oracle import gs_oracle as O
    N = gmap.n

    def fn(group, flat):
        comp, gi = np.divmod(np.asarray(flat, np.int64), N)
        ids = sorted(set(gi.tolist()))
        mass, walk = O.gradient_term_mass(gmap, cams, dls, ids, bg=bg, tiles=tiles)
        row = {g: j for j, g in enumerate(ids)}
        return np.array([mass[group][row[int(g)], int(c)] for c, g in zip(comp, gi)]), walk

    return fn


def assert_grad_close(name, g, ref, rel=1e-3, floor=1e-3, mass_fn=None):
    """GPU gradient vs the FP64 oracle, the parity contract for gradients:
    per element |g - ref| <= rel * max(|ref|, floor * max|ref|) and, over the
    group, ||g - ref||_2 <= rel ||ref||_2.  The floor (1e-3 of the group's
    largest magnitude) covers elements that are sums of cancelling per-pixel
    terms.

    mass_fn (optional): an element outside that bound is still accepted when
    its terms cancel so strongly that float32 rounding alone explains the
    error: |g - ref| <= u (walk + 64) mass, where mass is the oracle's exact
    sum of the absolute values of the element's per-pixel terms (through the
    splat's screen-space parameters), u = 2^-24, and walk + 64 counts the
    roundings a term can collect (the transmittance recovered through up to
    `walk` splats of the reverse walk, then a 64-lane reduction).  Prints how
    many elements needed it.  The L2 bound has no exception."""
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
    extra = ""
    if bad.any() and mass_fn is not None:
        idx = np.nonzero(bad)[0]
        mass, walk = mass_fn(name, idx)
        bound = U32 * (walk + 64) * mass
        ok = err[idx] <= bound
        extra = (f", {len(idx)} outside the contract: {int(ok.sum())} within the float32 bound of "
                 f"their cancelling terms (terms/value up to "
                 f"{np.max(mass / np.maximum(np.abs(ref[idx]), 1e-300)):.0f}, walk {walk})")
        bad[idx[ok]] = False
    print(f"  {name}: rel L2 {l2:.2e}, worst err/tol {err[worst] / tol[worst]:.3f}{extra}", flush=True)
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


def f32(x: float) -> float:
    """A hyperparameter as the C ABI receives it (a float32), in float64."""
    return float(np.float32(x))
