"""Comparison helpers shared by the tests (no method arithmetic)."""
import numpy as np


def tiles_of_pixels(views, tile, pixel_mask):
    """Global tile ids (views concatenated) that contain any flagged pixel."""
    out = []
    tb = 0
    pb = 0
    for v in views:
        w, h = int(v["width"]), int(v["height"])
        gx, gy = (w + tile - 1) // tile, (h + tile - 1) // tile
        m = pixel_mask[pb:pb + w * h].reshape(h, w)
        ys, xs = np.nonzero(m)
        out.extend((tb + (ys // tile) * gx + xs // tile).tolist())
        tb += gx * gy
        pb += w * h
    return np.unique(np.asarray(out, dtype=np.int64))


def exempt_gaussians(proj, bins, views, tile, fragile):
    """[V, N] bool: the (view, Gaussian)s whose gradient a fragile pixel can move.

    A decision at a compositing threshold (alpha vs 1/255, T(1-alpha) vs 1e-4,
    o*G vs 0.99) or an L1 sign taken at a near-tie may differ between two
    float32 implementations; a pixel adds to a Gaussian's gradient only where
    it composites it, so a flip there moves the gradients of the Gaussians the
    pixel can composite (up to a loosened stop), which the oracle lists."""
    import oracle
    return oracle.pixel_support(proj, bins, views, tile, np.asarray(fragile).astype(np.uint8))


def checked_fraction(exempt_any, touched, floor, label=""):
    """Share of the gradient-carrying Gaussians that are checked (not exempt);
    printed, and asserted to be at least floor."""
    touched = np.asarray(touched, bool)
    checked = touched & ~np.asarray(exempt_any, bool)
    frac = checked.sum() / max(int(touched.sum()), 1)
    print(f"[gpu-test]   {label}checked {int(checked.sum())}/{int(touched.sum())} Gaussians with a "
          f"gradient ({frac:.3f})", flush=True)
    assert frac >= floor, f"only {frac:.3f} of the Gaussians with a gradient are checked"
    return frac


def masked_image_gradient(dLdC, fragile):
    """The image gradient with the fragile pixels' rows zeroed, float32 [P, 3]:
    given to both sides, no pixel whose decisions may differ adds to any
    gradient, so every Gaussian can be checked."""
    g = np.asarray(dLdC, np.float64).reshape(-1, 3).copy()
    g[np.asarray(fragile).reshape(-1) != 0] = 0.0
    return np.ascontiguousarray(g.astype(np.float32))


# float32 unit roundoff: the scale of the running error bounds the oracle returns
ROUND_U = 2.0 ** -24


def grad_close(got, ref, rtol=1e-3, floor=1e-2, mag=None):
    """Elementwise |got - ref| <= rtol * max(|ref|, floor * max|ref| per column)
    (+ ROUND_U * mag when a running error bound mag is given: a float32
    evaluation of a sum whose terms cancel can be held no closer than that)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max(axis=0, keepdims=True)
    tol = rtol * np.maximum(np.abs(ref), floor * scale)
    if mag is not None:
        tol = tol + ROUND_U * np.asarray(mag, np.float64)
    return np.abs(got - ref) <= tol
