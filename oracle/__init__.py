"""CPU oracle for the 3DGS training hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it.

The arithmetic lives in ``oracle.c`` (plain loops, one Gaussian / one pixel at
a time); this module only compiles it with gcc, loads it with ctypes and
marshals numpy arrays.  ``double=False`` selects the float32-forward build
(the parity oracle), ``double=True`` the all-float64 build used by the
finite-difference and closed-form checks.

Pipeline (paper Sec. 2, Sec. 4): project -> scan -> emit keys -> stable sort
-> tile ranges -> compositing forward -> L1 gradient -> compositing backward
-> projection backward -> Adam.  ``train_step`` runs all of it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIBS = {False: os.path.join(_HERE, "liboracle_f32.so"),
         True: os.path.join(_HERE, "liboracle_f64.so")}
_loaded: dict = {}

# relative margins around the compositing thresholds inside which a decision
# taken in float32 may legitimately differ between two float32 implementations
# (alpha vs 1/255, o*G vs 0.99, T(1-alpha) vs 1e-4, the quadratic form vs 0),
# and the float32 error of the quadratic form per unit of its absolute terms
# (a few roundings of 2^-24 each, doubled for safety)
DEFAULT_MARGINS = (2e-5, 2e-5, 2e-4, 1e-5, 5e-7)
L1_SIGN_MARGIN = 1e-5


def build(force: bool = True) -> None:
    """Compile both oracle builds with gcc (no contraction, no fast-math)."""
    for dbl, out in _LIBS.items():
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
            continue
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", "-o", out + ".tmp", _SRC, "-lm"]
        if dbl:
            cmd.insert(1, "-DOR_DOUBLE")
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    _loaded.clear()


_P = C.c_void_p
_I64 = C.c_int64
_I = C.c_int
_D = C.c_double

_SIGS = {
    "or_project": (None, [_P, _P, _P, _P, _P, _I64, _P, _I, _I, _I, _P, _P, _P, _P, _P, _P, _P, _P,
                          _P]),
    "or_scan": (_I, [_P, _I64, _P]),
    "or_tile_bits": (_I, [_I]),
    "or_depth_bits": (_I, [_I]),
    "or_depth_key": (C.c_uint32, [C.c_float, _I]),
    "or_emit_keys": (None, [_P, _P, _P, _P, _P, _P, _I, _P, _I64, _P, _I, _I, _P, _P, _P]),
    "or_sort_segments": (None, [_P, _P, _P, _I]),
    "or_tile_ranges": (None, [_P, _P, _P, _I, _I, _P]),
    "or_raster_fwd": (None, [_P, _P, _P, _P, _P, _P, _P, _I64, _P, _I, _I, _P, _P,
                             _P, _P, _P, _P, _P, _P]),
    "or_l1": (_D, [_P, _P, _I64, _D, _P, _P, _P]),
    "or_pixel_support": (None, [_P, _P, _P, _P, _P, _P, _I64, _P, _I, _I, _P, _D, _D, _P]),
    "or_raster_bwd": (None, [_P, _P, _P, _P, _P, _P, _P, _P, _I64, _P, _I, _I, _P, _P, _P, _P, _P]),
    "or_project_bwd": (None, [_P, _P, _P, _P, _P, _I64, _P, _I, _I, _I, _P, _P]),
    "or_adam": (None, [_P, _P, _P, _P, _I64, _P, _D, _D, _D, _I]),
    "or_sh_basis": (None, [_P, _P]),
    "or_cov3d": (_I, [_P, _P, _P, _P]),
    "or_exp_param": (_D, [_D]),
    "or_log_spec": (_D, [_D]),
    "or_ellipse_tiles": (_I, [_D, _D, _D, _D, _D, _D, _I, _I, _I, _P]),
    "or_sigmoid": (_D, [_D]),
    "or_threads": (_I, []),
    "or_is_double": (_I, []),
}


def lib(double: bool = False):
    if double in _loaded:
        return _loaded[double]
    path = _LIBS[double]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(force=True)
    h = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(h, name)
        f.restype = res
        f.argtypes = args
    _loaded[double] = h
    return h


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "array must be C-contiguous"
    return a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _pin(a, double):
    """Parameters enter each build in its working precision."""
    return np.ascontiguousarray(a, dtype=np.float64 if double else np.float32)


def n_tiles(views, tile: int):
    return [((int(v["width"]) + tile - 1) // tile) * ((int(v["height"]) + tile - 1) // tile)
            for v in views]


def n_pixels(views):
    return [int(v["width"]) * int(v["height"]) for v in views]


def depth_bits(ntiles: int, double=False) -> int:
    return int(lib(double).or_depth_bits(ntiles))


# ---------------------------------------------------------------------------
# stage wrappers
# ---------------------------------------------------------------------------

@dataclass
class Projected:
    xy: np.ndarray       # [V, N, 2]
    conic: np.ndarray    # [V, N, 3]  (A, B, C)
    opacity: np.ndarray  # [V, N]
    rgb: np.ndarray      # [V, N, 3]
    depth: np.ndarray    # [V, N]
    radius: np.ndarray   # [V, N]
    cov2d: np.ndarray    # [V, N, 3]  (a, b, c)
    rect: np.ndarray     # [V, N, 4]  (x0, y0, x1, y1) int32: bounding tile box
    tiles: np.ndarray    # [V, N] uint32
    cull: int = 0        # 0: 3-sigma rectangle; 1: exact opacity-ellipse culling


CULL_RECT, CULL_ELLIPSE = 0, 1


def project(scene, views, tile: int, double: bool = False, cull: int = CULL_RECT) -> Projected:
    L = lib(double)
    means, ls, q, lo, sh = (_pin(a, double) for a in scene.arrays())
    n = means.shape[0]
    V = len(views)
    views = np.ascontiguousarray(views)
    out = Projected(np.zeros((V, n, 2)), np.zeros((V, n, 3)), np.zeros((V, n)), np.zeros((V, n, 3)),
                    np.zeros((V, n)), np.zeros((V, n)), np.zeros((V, n, 3)),
                    np.zeros((V, n, 4), np.int32), np.zeros((V, n), np.uint32), int(cull))
    L.or_project(_p(means), _p(ls), _p(q), _p(lo), _p(sh), n, _p(views), V, tile, int(cull), _p(out.xy),
                 _p(out.conic), _p(out.opacity), _p(out.rgb), _p(out.depth), _p(out.radius),
                 _p(out.cov2d), _p(out.rect), _p(out.tiles))
    return out


@dataclass
class Bins:
    offsets: np.ndarray   # [V*N+1] uint32 exclusive scan of tiles (view-major)
    keys: np.ndarray      # [K] uint32, sorted within each view segment
    vals: np.ndarray      # [K] uint32, unsorted intersection index, sorted alongside
    gid: np.ndarray       # [K] uint32, Gaussian id by unsorted index
    keys_unsorted: np.ndarray
    seg_begin: np.ndarray  # [V+1]
    ranges: np.ndarray    # [total_tiles, 2] uint32 global positions


def scan(counts: np.ndarray, double=False) -> np.ndarray:
    counts = np.ascontiguousarray(counts, dtype=np.uint32).reshape(-1)
    off = np.zeros(counts.size + 1, np.uint32)
    rc = lib(double).or_scan(_p(counts), counts.size, _p(off))
    if rc != 0:
        raise OverflowError("intersection count exceeds 32 bits")
    return off


def bin_sort(proj: Projected, views, tile: int, double: bool = False) -> Bins:
    L = lib(double)
    V, n = proj.tiles.shape
    views = np.ascontiguousarray(views)
    offsets = scan(proj.tiles.reshape(-1), double)
    K = int(offsets[-1])
    keys = np.zeros(max(K, 1), np.uint32)
    vals = np.zeros(max(K, 1), np.uint32)
    gid = np.zeros(max(K, 1), np.uint32)
    depth = np.ascontiguousarray(proj.depth)
    L.or_emit_keys(_p(np.ascontiguousarray(proj.rect)), _p(np.ascontiguousarray(proj.tiles)),
                   _p(depth), _p(np.ascontiguousarray(proj.xy)), _p(np.ascontiguousarray(proj.conic)),
                   _p(np.ascontiguousarray(proj.opacity)), int(proj.cull), _p(offsets), n, _p(views),
                   V, tile, _p(keys), _p(vals), _p(gid))
    keys_unsorted = keys[:K].copy()
    seg = np.array([offsets[v * n] for v in range(V)] + [K], np.uint32)
    L.or_sort_segments(_p(keys), _p(vals), _p(seg), V)
    ranges = np.zeros((sum(n_tiles(views, tile)), 2), np.uint32)
    L.or_tile_ranges(_p(keys), _p(seg), _p(views), V, tile, _p(ranges))
    return Bins(offsets, keys[:K], vals[:K], gid[:K], keys_unsorted, seg, ranges)


@dataclass
class Image:
    rgb: np.ndarray          # [P, 3] float64, views concatenated
    T: np.ndarray            # [P]
    last: np.ndarray         # [P] uint32
    fragile: np.ndarray      # [P] uint8
    tile_traversed: np.ndarray
    tile_evaluated: np.ndarray


def raster_fwd(proj: Projected, bins: Bins, views, tile: int, double: bool = False,
               margins=DEFAULT_MARGINS, tile_mask=None) -> Image:
    """Compositing forward; tile_mask (total tiles, nonzero = render) limits the
    work to a sample of tiles (other pixels stay zero)."""
    L = lib(double)
    V, n = proj.tiles.shape
    views = np.ascontiguousarray(views)
    P = sum(n_pixels(views))
    nt = sum(n_tiles(views, tile))
    img = Image(np.zeros((P, 3)), np.zeros(P), np.zeros(P, np.uint32), np.zeros(P, np.uint8),
                np.zeros(nt, np.uint32), np.zeros(nt, np.uint64))
    mg = np.asarray(margins, np.float64)
    vals = bins.vals if bins.vals.size else np.zeros(1, np.uint32)
    gid = bins.gid if bins.gid.size else np.zeros(1, np.uint32)
    tm = None if tile_mask is None else np.ascontiguousarray(tile_mask, dtype=np.uint8)
    L.or_raster_fwd(_p(np.ascontiguousarray(proj.xy)), _p(np.ascontiguousarray(proj.conic)),
                    _p(np.ascontiguousarray(proj.opacity)), _p(np.ascontiguousarray(proj.rgb)),
                    _p(bins.ranges), _p(vals), _p(gid), n, _p(views), V, tile, _p(mg),
                    None if tm is None else _p(tm), _p(img.rgb), _p(img.T), _p(img.last), _p(img.fragile),
                    _p(img.tile_traversed), _p(img.tile_evaluated))
    return img


def l1(image_rgb: np.ndarray, target: np.ndarray, double=False, fragile: np.ndarray | None = None,
       last: np.ndarray | None = None):
    """Returns (loss, dL/dC [P,3]); flags near-tie signs in fragile (in/out),
    except at pixels where last says nothing was composited."""
    target = _f32(target).reshape(-1, 3)
    img = np.ascontiguousarray(image_rgb, dtype=np.float64).reshape(-1, 3)
    g = np.zeros_like(img)
    fr = fragile if fragile is not None else np.zeros(img.shape[0], np.uint8)
    lst = None if last is None else np.ascontiguousarray(last, dtype=np.uint32)
    loss = lib(double).or_l1(_p(img), _p(target), img.shape[0], L1_SIGN_MARGIN,
                             None if lst is None else _p(lst), _p(g), _p(fr))
    return loss, g


SUPPORT_MARGIN = 1e-2


def pixel_support(proj: Projected, bins: Bins, views, tile: int, pixmask: np.ndarray,
                  rel_margin: float = SUPPORT_MARGIN, double: bool = False) -> np.ndarray:
    """[V, N] bool: the (view, Gaussian)s whose alpha at some flagged pixel of
    their tile reaches 1/255 (within rel_margin and the quadratic form's float32
    error): the only ones whose gradient a flagged pixel can change."""
    V, n = proj.tiles.shape
    views = np.ascontiguousarray(views)
    out = np.zeros(V * n, np.uint8)
    pm = np.ascontiguousarray(pixmask, dtype=np.uint8).reshape(-1)
    assert pm.size == sum(n_pixels(views))
    if not pm.any() or bins.vals.size == 0:
        return out.reshape(V, n).astype(bool)
    lib(double).or_pixel_support(_p(np.ascontiguousarray(proj.xy)), _p(np.ascontiguousarray(proj.conic)),
                                 _p(np.ascontiguousarray(proj.opacity)), _p(bins.ranges), _p(bins.vals),
                                 _p(bins.gid), n, _p(views), V, tile, _p(pm), float(rel_margin),
                                 float(DEFAULT_MARGINS[4]), _p(out))
    return out.reshape(V, n).astype(bool)


def raster_bwd(proj: Projected, bins: Bins, views, tile: int, dLdC: np.ndarray,
               double: bool = False, tile_mask=None, magnitudes: bool = False):
    """Returns (partials [K,9] by unsorted index, grads2d [V,N,9]); tile_mask
    limits the work to a sample of tiles (others contribute nothing).  With
    magnitudes, also mag2d [V,N,9]: per component the sum over pixels of the
    magnitudes of the terms (the scale of a float summation's rounding)."""
    L = lib(double)
    V, n = proj.tiles.shape
    views = np.ascontiguousarray(views)
    K = int(bins.offsets[-1])
    partials = np.zeros((max(K, 1), 9))
    grads2d = np.zeros((V, n, 9))
    mag2d = np.zeros((V, n, 9)) if magnitudes else None
    vals = bins.vals if bins.vals.size else np.zeros(1, np.uint32)
    gid = bins.gid if bins.gid.size else np.zeros(1, np.uint32)
    L.or_raster_bwd(_p(np.ascontiguousarray(proj.xy)), _p(np.ascontiguousarray(proj.conic)),
                    _p(np.ascontiguousarray(proj.opacity)), _p(np.ascontiguousarray(proj.rgb)),
                    _p(bins.ranges), _p(vals), _p(gid), _p(bins.offsets), n, _p(views), V, tile,
                    None if tile_mask is None else _p(np.ascontiguousarray(tile_mask, dtype=np.uint8)),
                    _p(np.ascontiguousarray(dLdC, dtype=np.float64)), _p(partials), _p(grads2d),
                    _p(mag2d) if magnitudes else None)
    if magnitudes:
        return partials[:K], grads2d, mag2d
    return partials[:K], grads2d


def project_bwd(scene, views, tile: int, grads2d: np.ndarray, double: bool = False,
                cull: int = CULL_RECT) -> np.ndarray:
    """Returns grads [N, 59] in the canonical parameter order."""
    L = lib(double)
    means, ls, q, lo, sh = (_pin(a, double) for a in scene.arrays())
    n = means.shape[0]
    views = np.ascontiguousarray(views)
    grads = np.zeros((n, 59))
    L.or_project_bwd(_p(means), _p(ls), _p(q), _p(lo), _p(sh), n, _p(views), len(views), tile,
                     int(cull), _p(np.ascontiguousarray(grads2d, dtype=np.float64)), _p(grads))
    return grads


def project_bwd_magnitudes(scene, views, tile: int, mag2d: np.ndarray, double: bool = False,
                           cull: int = CULL_RECT) -> np.ndarray:
    """[N, 59]: sum over the 9 screen-space components j of |d param / d g_j| *
    mag2d_j.  The projection backward is linear in the screen-space gradients,
    so one pass per component gives each term; this bounds how far rounding
    errors of the screen-space sums (each within a multiple of mag2d) can move
    a parameter gradient."""
    mag2d = np.ascontiguousarray(mag2d, dtype=np.float64)
    out = np.zeros((mag2d.shape[1], 59))
    for j in range(9):
        one = np.zeros_like(mag2d)
        one[..., j] = mag2d[..., j]
        out += np.abs(project_bwd(scene, views, tile, one, double, cull))
    return out


ADAM_BETAS = (0.9, 0.999)
ADAM_EPS = 1e-15


def adam(flat_params: np.ndarray, m: np.ndarray, v: np.ndarray, grads: np.ndarray, lr, step: int,
         betas=ADAM_BETAS, eps=ADAM_EPS, double=False):
    """In-place Adam on [N,59] float32 arrays; lr is a scalar or 6 group rates."""
    lrs = np.broadcast_to(np.asarray(lr, np.float64), (6,)).copy()
    for a in (flat_params, m, v):
        assert a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]
    lib(double).or_adam(_p(flat_params), _p(m), _p(v), _p(np.ascontiguousarray(grads, np.float64)),
                        flat_params.shape[0], _p(lrs), betas[0], betas[1], eps, step)


def sh_basis(direction, double=False) -> np.ndarray:
    d = np.ascontiguousarray(direction, dtype=np.float64)
    Y = np.zeros(16)
    lib(double).or_sh_basis(_p(d), _p(Y))
    return Y


def cov3d(log_scale, quat, double=False):
    """(R [3,3], Sigma [3,3]) of one Gaussian."""
    R = np.zeros(9)
    Sig = np.zeros(9)
    ok = lib(double).or_cov3d(_p(_pin(log_scale, double)), _p(_pin(quat, double)), _p(R), _p(Sig))
    if not ok:
        raise ValueError("zero quaternion")
    return R.reshape(3, 3), Sig.reshape(3, 3)


def exp_param(x: float, double=False) -> float:
    return float(lib(double).or_exp_param(float(x)))


def sigmoid(x: float, double=False) -> float:
    return float(lib(double).or_sigmoid(float(x)))


def log_spec(x: float, double=False) -> float:
    return float(lib(double).or_log_spec(float(x)))


def ellipse_tiles(u, v, A, B, C, o, tile, gx, gy, double=False) -> np.ndarray:
    """Tile mask [gy, gx] (uint8) of one screen-space Gaussian under exact culling."""
    mask = np.zeros(gx * gy, np.uint8)
    lib(double).or_ellipse_tiles(float(u), float(v), float(A), float(B), float(C), float(o), int(tile),
                                 int(gx), int(gy), _p(mask))
    return mask.reshape(gy, gx)


def threads(double=False) -> int:
    return int(lib(double).or_threads())


# ---------------------------------------------------------------------------
# whole step
# ---------------------------------------------------------------------------

@dataclass
class StepResult:
    proj: Projected
    bins: Bins
    image: Image
    loss: float
    dLdC: np.ndarray
    partials: np.ndarray
    grads2d: np.ndarray
    grads: np.ndarray
    params: np.ndarray | None   # [N,59] after Adam (None when no optimiser step)
    m: np.ndarray | None
    v: np.ndarray | None
    fragile: np.ndarray         # [P] uint8: compositing or L1-sign decisions near a threshold


def train_step(scene, views, tile: int, target: np.ndarray | None, lr=1e-3, step: int = 1, m=None, v=None,
               double: bool = False, adam_step: bool = True, cull: int = CULL_RECT,
               dLdC: np.ndarray | None = None) -> StepResult:
    """One L1 training step over all given views (gradients summed over views).
    With dLdC given ([P,3]), the backward takes that image gradient instead of
    the L1 gradient against target (loss is then None)."""
    proj = project(scene, views, tile, double, cull)
    bins = bin_sort(proj, views, tile, double)
    img = raster_fwd(proj, bins, views, tile, double)
    fragile = img.fragile.copy()
    if dLdC is None:
        loss, dLdC = l1(img.rgb, target, double, fragile, img.last)
    else:
        loss = None
        dLdC = np.ascontiguousarray(dLdC, dtype=np.float64).reshape(-1, 3)
    partials, grads2d = raster_bwd(proj, bins, views, tile, dLdC, double)
    grads = project_bwd(scene, views, tile, grads2d, double, cull)
    params = mm = vv = None
    if adam_step:
        params = scene.flat()
        n = params.shape[0]
        mm = np.zeros((n, 59), np.float32) if m is None else np.ascontiguousarray(m, np.float32).copy()
        vv = np.zeros((n, 59), np.float32) if v is None else np.ascontiguousarray(v, np.float32).copy()
        adam(params, mm, vv, grads, lr, step, double=double)
    return StepResult(proj, bins, img, loss, dLdC, partials, grads2d, grads, params, mm, vv, fragile)


def render(scene, views, tile: int, double: bool = False, cull: int = CULL_RECT) -> np.ndarray:
    """Forward only: the composited image [P,3] float32 (views concatenated)."""
    proj = project(scene, views, tile, double, cull)
    bins = bin_sort(proj, views, tile, double)
    return raster_fwd(proj, bins, views, tile, double).rgb.astype(np.float32)
