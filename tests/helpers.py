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


def exempt_gaussians(ranges, vals, gid, views, tile, fragile, n):
    """[V, N] bool: Gaussians listed in a tile that holds a fragile pixel.

    A decision at a compositing threshold (alpha vs 1/255, T(1-alpha) vs 1e-4,
    o*G vs 0.99) or an L1 sign taken at a near-tie may differ between two
    float32 implementations; such a flip moves the gradient of every Gaussian
    composited at that pixel, so those Gaussians are checked separately."""
    ex = np.zeros((len(views), n), bool)
    tiles = tiles_of_pixels(views, tile, fragile.astype(bool))
    tb = np.cumsum([0] + [((int(v["width"]) + tile - 1) // tile) * ((int(v["height"]) + tile - 1) // tile)
                          for v in views])
    for t in tiles:
        vi = int(np.searchsorted(tb, t, side="right") - 1)
        s, e = ranges[t]
        ex[vi, gid[vals[s:e]]] = True
    return ex


def grad_close(got, ref, rtol=1e-3, floor=1e-2):
    """Elementwise |got - ref| <= rtol * max(|ref|, floor * max|ref| per column)."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max(axis=0, keepdims=True)
    return np.abs(got - ref) <= rtol * np.maximum(np.abs(ref), floor * scale)
