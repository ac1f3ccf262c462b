"""Pins of the CPU oracle against facts that do not come from the oracle itself:
library routines (scipy, numpy, torch CPU), closed forms, invariants, brute
force on tiny inputs and central finite differences.

A plausible mistake anywhere in the oracle -- a dropped term, a wrong sign or
index, a transposed operand -- should fail at least one of these.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as S
from helpers import exempt_gaussians, grad_close, masked_image_gradient

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _view(w, h, campos=(0.0, 0.0, -4.0), bg=(0.0, 0.0, 0.0)):
    return S.views_array([S.make_view(w, h, campos, bg=bg)])


def _scene_from(means, log_scales, quats, logits, sh):
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return S.Scene(f(means), f(log_scales), f(quats), f(logits), f(sh))


def _dc_for_colour(c):
    """SH DC coefficient that gives colour c (before clamp): Y0*dc + 0.5 = c."""
    return (np.asarray(c, np.float64) - 0.5) / 0.28209479177387814


# ---------------------------------------------------------------------------
# scalar activations
# ---------------------------------------------------------------------------

def test_exp_param_within_two_ulp_of_exp():
    xs = np.linspace(-20.0, 10.0, 4001).astype(np.float32)
    for x in xs:
        exact = math.exp(float(x))
        got = oracle.exp_param(float(x))
        ulp = float(np.spacing(np.float32(exact)))
        assert abs(got - exact) <= 2.0 * ulp, (x, got, exact)
    # float64 build is libm exp
    assert oracle.exp_param(1.234, double=True) == math.exp(1.234)


def test_sigmoid_matches_scipy_expit():
    from scipy.special import expit
    for x in np.linspace(-12, 12, 2001):
        xf = float(np.float32(x))
        assert abs(oracle.sigmoid(xf) - expit(xf)) <= 4e-7 * max(expit(xf), 1e-30) + 1e-12
        assert abs(oracle.sigmoid(xf, double=True) - expit(xf)) <= 1e-15


# ---------------------------------------------------------------------------
# covariance
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("double", [False, True])
def test_rotation_matches_scipy(double):
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(7)
    for _ in range(200):
        q = rng.normal(size=4)
        R, _ = oracle.cov3d(np.zeros(3), q, double)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scalar-last
        tol = 1e-12 if double else 2e-6
        np.testing.assert_allclose(R, ref, atol=tol)
        assert abs(np.linalg.det(R) - 1) < 10 * tol


@pytest.mark.parametrize("double", [False, True])
def test_covariance_eigenvalues_are_squared_scales(double):
    rng = np.random.default_rng(8)
    for _ in range(200):
        ls = rng.normal(-2, 1, size=3)
        q = rng.normal(size=4)
        R, Sig = oracle.cov3d(ls, q, double)
        np.testing.assert_allclose(Sig, Sig.T, rtol=0, atol=0)
        ev = np.linalg.eigvalsh(Sig)
        s2 = np.sort(np.exp(2 * ls.astype(np.float32 if not double else np.float64)))
        # float32 rounding is absolute relative to the largest eigenvalue
        np.testing.assert_allclose(ev, s2, rtol=1e-10 if double else 2e-6,
                                   atol=(1e-14 if double else 1e-6) * s2.max())


# ---------------------------------------------------------------------------
# projection
# ---------------------------------------------------------------------------

def _pinhole(p, v):
    return np.array([v["fx"] * p[0] / p[2] + v["cx"], v["fy"] * p[1] / p[2] + v["cy"]])


@pytest.mark.parametrize("double", [False, True])
def test_cov2d_matches_finite_difference_jacobian(double):
    from scipy.spatial.transform import Rotation
    scene = S.scene_uniform_cube(300, 11, log_scale_mean=-2.5)
    views = S.views_array([S.make_view(320, 200, c) for c in S.fibonacci_sphere(3, 4.0)])
    pr = oracle.project(scene, views, 16, double)
    checked = 0
    for vi, v in enumerate(views):
        W = v["R"].reshape(3, 3).astype(np.float64)
        t = v["t"].astype(np.float64)
        for g in range(scene.n):
            if pr.tiles[vi, g] == 0:
                continue
            mu = scene.means[g].astype(np.float64)
            p = W @ mu + t
            if abs(p[0] / p[2]) > v["lim_x"] or abs(p[1] / p[2]) > v["lim_y"]:
                continue
            J = np.zeros((2, 3))
            for k in range(3):
                h = 1e-6 * max(1.0, abs(p[k]))
                e = np.zeros(3)
                e[k] = h
                J[:, k] = (_pinhole(p + e, v) - _pinhole(p - e, v)) / (2 * h)
            q = scene.quats[g].astype(np.float64)
            Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
            Sig = Rq @ np.diag(np.exp(2 * scene.log_scales[g].astype(np.float64))) @ Rq.T
            S2 = J @ W @ Sig @ W.T @ J.T + 0.3 * np.eye(2)
            got = pr.cov2d[vi, g]
            ref = np.array([S2[0, 0], S2[0, 1], S2[1, 1]])
            np.testing.assert_allclose(got, ref, rtol=1e-6 if double else 1e-4,
                                       atol=(1e-8 if double else 1e-5) * abs(ref).max())
            # conic is the inverse
            A, B, Cc = pr.conic[vi, g]
            inv = np.linalg.inv(S2)
            np.testing.assert_allclose([A, B, Cc], [inv[0, 0], inv[0, 1], inv[1, 1]],
                                       rtol=1e-5 if double else 2e-4,
                                       atol=(1e-9 if double else 1e-5) * abs(inv).max())
            # projected mean
            np.testing.assert_allclose(pr.xy[vi, g], _pinhole(p, v), rtol=1e-6, atol=1e-3)
            checked += 1
    assert checked > 200


def test_isotropic_gaussian_on_axis_closed_form():
    # Gaussian at the origin, camera at (0,0,-4) looking at it: z0 = 4 and
    # Sigma' = ((f s / z0)^2 + 0.3) I, conic = I / that, radius = ceil(3 sqrt(that)).
    for s in (0.02, 0.1, 0.3):
        for double in (False, True):
            scene = _scene_from([[0, 0, 0]], [[math.log(s)] * 3], [[1, 0, 0, 0]], [0.0],
                                np.zeros((1, 16, 3)))
            views = _view(128, 96)
            pr = oracle.project(scene, views, 16, double)
            f = float(views[0]["fx"])
            var = (f * math.exp(float(np.float32(math.log(s)))) / 4.0) ** 2 + 0.3
            tol = 1e-12 if double else 3e-6
            np.testing.assert_allclose(pr.cov2d[0, 0], [var, 0, var], rtol=tol, atol=tol)
            np.testing.assert_allclose(pr.conic[0, 0], [1 / var, 0, 1 / var], rtol=10 * tol, atol=tol)
            assert pr.radius[0, 0] == math.ceil(3 * math.sqrt(var))
            np.testing.assert_allclose(pr.xy[0, 0], [64.0, 48.0], atol=1e-5)
            assert pr.depth[0, 0] == pytest.approx(4.0)
            assert pr.opacity[0, 0] == pytest.approx(0.5)


@pytest.mark.parametrize("double", [False, True])
def test_sh_basis_orthonormal_by_quadrature(double):
    nodes, weights = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phis = 2 * np.pi * np.arange(nphi) / nphi
    G = np.zeros((16, 16))
    for mu, wt in zip(nodes, weights):
        st = math.sqrt(1 - mu * mu)
        for ph in phis:
            Y = oracle.sh_basis([st * math.cos(ph), st * math.sin(ph), mu], double)
            G += np.outer(Y, Y) * wt * (2 * np.pi / nphi)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12 if double else 2e-6)


def test_sh_dc_only_colour_and_clamp():
    dc = np.array([[0.8, -0.3, -3.0]])
    sh = np.zeros((1, 16, 3))
    sh[0, 0] = dc
    scene = _scene_from([[0.1, 0.2, 0.0]], [[-2.0] * 3], [[1, 0, 0, 0]], [0.0], sh)
    pr = oracle.project(scene, _view(64, 64), 16, double=True)
    ref = np.maximum(0.28209479177387814 * dc[0].astype(np.float32).astype(np.float64) + 0.5, 0)
    np.testing.assert_allclose(pr.rgb[0, 0], ref, rtol=1e-14)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_rect_matches_brute_force_tile_overlap(tile):
    scene = S.scene_uniform_cube(400, 12, log_scale_mean=-2.5, log_scale_std=1.0)
    views = S.views_array([S.make_view(200, 130, (0.3, -0.2, -3.0))])
    pr = oracle.project(scene, views, tile)
    gx, gy = (200 + tile - 1) // tile, (130 + tile - 1) // tile
    nvis = 0
    for g in range(scene.n):
        u, v = pr.xy[0, g]
        r = pr.radius[0, g]
        if pr.depth[0, g] == 0:
            assert pr.tiles[0, g] == 0
            continue
        a, b, c = pr.cov2d[0, g]
        lam = np.linalg.eigvalsh(np.array([[a, b], [b, c]]))[-1]
        if abs(3 * math.sqrt(lam) - round(3 * math.sqrt(lam))) > 1e-4:
            assert r == math.ceil(3 * math.sqrt(lam))
        brute = [(tx, ty) for ty in range(gy) for tx in range(gx)
                 if tx * tile <= u + r and (tx + 1) * tile > u - r
                 and ty * tile <= v + r and (ty + 1) * tile > v - r]
        x0, y0, x1, y1 = pr.rect[0, g]
        if pr.tiles[0, g] == 0:
            # culled only by det/empty-rect rules; an empty brute-force set is required here
            assert len(brute) == 0 or not (pr.opacity[0, g] > 0)
            continue
        nvis += 1
        got = [(tx, ty) for ty in range(y0, y1) for tx in range(x0, x1)]
        assert sorted(got) == sorted(brute)
        assert pr.tiles[0, g] == len(brute)
    assert nvis > 100


# ---------------------------------------------------------------------------
# binning: scan, keys, sort, ranges
# ---------------------------------------------------------------------------

def _two_view_bins(tile=16):
    scene = S.scene_uniform_cube(1500, 21)
    views = S.views_array([S.make_view(256, 192, (0.0, 0.0, -4.0)),
                           S.make_view(160, 100, (2.0, 1.0, -3.0))])
    pr = oracle.project(scene, views, tile)
    return scene, views, pr, oracle.bin_sort(pr, views, tile)


def test_scan_matches_cumsum():
    rng = np.random.default_rng(3)
    c = rng.integers(0, 50, size=10007).astype(np.uint32)
    off = oracle.scan(c)
    np.testing.assert_array_equal(off, np.concatenate([[0], np.cumsum(c, dtype=np.uint64)]).astype(np.uint32))
    with pytest.raises(OverflowError):
        oracle.scan(np.full(3, 2 ** 31, np.uint32))


def test_depth_key_map_is_in_one_two_and_monotone():
    zs = np.sort(np.float32(np.exp(np.linspace(math.log(0.011), math.log(999.0), 5000))))
    prev = -1
    for z in zs:
        num = np.float32(2) * z + np.float32(1)
        f = np.float32(num / (z + np.float32(1)))
        bits = f.view(np.uint32)
        assert (bits >> 23) & 0xFF == 127          # exponent field of [1, 2)
        k = oracle.lib().or_depth_key(float(z), 20)
        assert k == (int(bits) & 0x7FFFFF) >> 3
        assert k >= prev
        prev = k
    assert oracle.lib().or_tile_bits(3600) == 12 and oracle.lib().or_depth_bits(3600) == 20
    assert oracle.lib().or_tile_bits(256) == 8 and oracle.lib().or_depth_bits(256) == 23
    assert oracle.lib().or_tile_bits(8160) == 13 and oracle.lib().or_depth_bits(8160) == 19
    assert oracle.lib().or_tile_bits(1) == 1


def test_emitted_keys_decode_to_rect_tiles():
    scene, views, pr, bins = _two_view_bins()
    n = scene.n
    for vi, v in enumerate(views):
        gx = (int(v["width"]) + 15) // 16
        nt = gx * ((int(v["height"]) + 15) // 16)
        D = oracle.depth_bits(nt)
        for g in range(0, n, 7):
            o = vi * n + g
            b, e = bins.offsets[o], bins.offsets[o + 1]
            assert e - b == pr.tiles[vi, g]
            if e == b:
                continue
            x0, y0, x1, y1 = pr.rect[vi, g]
            exp_tiles = [ty * gx + tx for ty in range(y0, y1) for tx in range(x0, x1)]
            ks = bins.keys_unsorted[b:e]
            np.testing.assert_array_equal(ks >> D, exp_tiles)
            assert np.all(bins.gid[b:e] == g)


def test_sort_is_stable_argsort_per_view_and_ranges_are_searchsorted():
    scene, views, pr, bins = _two_view_bins()
    tb = 0
    for vi, v in enumerate(views):
        b, e = int(bins.seg_begin[vi]), int(bins.seg_begin[vi + 1])
        uk = bins.keys_unsorted[b:e]
        order = np.argsort(uk, kind="stable")
        np.testing.assert_array_equal(bins.keys[b:e], uk[order])
        np.testing.assert_array_equal(bins.vals[b:e], (b + order).astype(np.uint32))
        nt = ((int(v["width"]) + 15) // 16) * ((int(v["height"]) + 15) // 16)
        D = oracle.depth_bits(nt)
        t = np.arange(nt, dtype=np.uint64)
        lo = np.searchsorted(bins.keys[b:e].astype(np.uint64), t << np.uint64(D), side="left")
        hi = np.searchsorted(bins.keys[b:e].astype(np.uint64), (t + np.uint64(1)) << np.uint64(D),
                             side="left")
        np.testing.assert_array_equal(bins.ranges[tb:tb + nt, 0], b + lo)
        np.testing.assert_array_equal(bins.ranges[tb:tb + nt, 1], b + hi)
        # ranges partition the segment
        assert bins.ranges[tb, 0] == b and bins.ranges[tb + nt - 1, 1] == e
        tb += nt


# ---------------------------------------------------------------------------
# compositing forward
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("double", [False, True])
def test_single_gaussian_closed_form(double):
    # o = 0.3 keeps alpha below 1/255 beyond 3 sigma, so the tile rule never
    # hides a visible pixel: C = c alpha + bg (1 - alpha), T = 1 - alpha.
    colour = np.array([0.9, 0.4, 0.2])
    sh = np.zeros((1, 16, 3))
    sh[0, 0] = _dc_for_colour(colour)
    logit = math.log(0.3 / 0.7)
    bg = (0.1, 0.2, 0.3)
    scene = _scene_from([[0, 0, 0]], [[math.log(0.2)] * 3], [[1, 0, 0, 0]], [logit], sh)
    views = _view(64, 48, bg=bg)
    pr = oracle.project(scene, views, 16, double)
    bins = oracle.bin_sort(pr, views, 16, double)
    img = oracle.raster_fwd(pr, bins, views, 16, double)
    var = pr.cov2d[0, 0, 0]
    o = pr.opacity[0, 0]
    c = pr.rgb[0, 0]
    ys, xs = np.mgrid[0:48, 0:64]
    d2 = (xs + 0.5 - 32.0) ** 2 + (ys + 0.5 - 24.0) ** 2
    alpha = np.minimum(0.99, o * np.exp(-0.5 * d2 / var))
    alpha = np.where(alpha < 1 / 255, 0.0, alpha).reshape(-1)
    ref = c[None, :] * alpha[:, None] + np.array(bg)[None, :] * (1 - alpha[:, None])
    tol = 1e-12 if double else 2e-6
    np.testing.assert_allclose(img.rgb, ref, atol=tol)
    np.testing.assert_allclose(img.T, 1 - alpha, atol=tol)
    np.testing.assert_array_equal(img.last, (alpha > 0).astype(np.uint32))
    np.testing.assert_allclose(c, colour, atol=1e-6)


@pytest.mark.parametrize("double", [False, True])
def test_traversal_counts_without_early_stop(double):
    # opacities <= 0.02 and at most a few hundred entries per tile keep T above
    # the 1e-4 stop, so every pixel examines its tile's whole list
    scene = S.workload_plain_small().scene.copy()
    scene.opacity_logits[:] = np.minimum(scene.opacity_logits, np.float32(math.log(0.02 / 0.98)))
    views = _view(200, 150)
    pr = oracle.project(scene, views, 16, double)
    bins = oracle.bin_sort(pr, views, 16, double)
    img = oracle.raster_fwd(pr, bins, views, 16, double)
    length = (bins.ranges[:, 1] - bins.ranges[:, 0]).astype(np.int64)
    assert length.max() < 400 and length.max() > 20
    assert img.T.min() > 1e-3
    gx, gy = (200 + 15) // 16, (150 + 15) // 16
    tx, ty = np.arange(gx * gy) % gx, np.arange(gx * gy) // gx
    npix = (np.minimum(16, 200 - 16 * tx) * np.minimum(16, 150 - 16 * ty)).astype(np.int64)
    np.testing.assert_array_equal(img.tile_traversed.astype(np.int64), length)
    np.testing.assert_array_equal(img.tile_evaluated.astype(np.int64), length * npix)


@pytest.mark.parametrize("double", [False, True])
def test_traversal_stops_at_the_fourth_of_stacked_gaussians(double):
    # ten identical Gaussians centred on the only pixel, alpha = o = 0.95 each:
    # T = 0.05, 0.0025, 1.25e-4 after three; the fourth would leave 6.25e-6 <
    # 1e-4, so it stops the pixel: 4 entries examined, 3 composited
    n = 10
    sh = np.zeros((n, 16, 3))
    sh[:, 0] = _dc_for_colour([0.7, 0.7, 0.7])
    scene = _scene_from([[0, 0, 0]] * n, [[math.log(0.05)] * 3] * n, [[1, 0, 0, 0]] * n,
                        [math.log(0.95 / 0.05)] * n, sh)
    views = _view(1, 1)
    pr = oracle.project(scene, views, 16, double)
    bins = oracle.bin_sort(pr, views, 16, double)
    img = oracle.raster_fwd(pr, bins, views, 16, double)
    np.testing.assert_allclose(pr.xy[0, :, 0], 0.5, atol=1e-6)
    np.testing.assert_allclose(pr.opacity[0], 0.95, rtol=1e-6)
    assert int(bins.ranges[0, 1] - bins.ranges[0, 0]) == n
    assert int(img.tile_traversed[0]) == 4 and int(img.tile_evaluated[0]) == 4
    assert int(img.last[0]) == 3
    np.testing.assert_allclose(img.T[0], 0.05 ** 3, rtol=1e-5)


def test_two_gaussians_closed_form_depth_order():
    sh = np.zeros((2, 16, 3))
    sh[0, 0] = _dc_for_colour([1.0, 0.0, 0.0])
    sh[1, 0] = _dc_for_colour([0.0, 0.0, 1.0])
    # index 0 is behind index 1: the sort must put index 1 first
    scene = _scene_from([[0.05, 0, 0.5], [-0.05, 0.02, -0.5]], [[math.log(0.15)] * 3] * 2,
                        [[1, 0, 0, 0], [0.9, 0.1, 0.3, -0.2]], [0.2, -0.4], sh)
    views = _view(48, 48, bg=(0.05, 0.05, 0.05))
    pr = oracle.project(scene, views, 16, True)
    bins = oracle.bin_sort(pr, views, 16, True)
    img = oracle.raster_fwd(pr, bins, views, 16, True)
    ys, xs = np.mgrid[0:48, 0:48]
    px, py = xs.reshape(-1) + 0.5, ys.reshape(-1) + 0.5

    def alpha(g):
        dx, dy = px - pr.xy[0, g, 0], py - pr.xy[0, g, 1]
        A, B, Cc = pr.conic[0, g]
        a = np.minimum(0.99, pr.opacity[0, g] * np.exp(-0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy))
        # tile membership of the pixel in the Gaussian's rect
        x0, y0, x1, y1 = pr.rect[0, g]
        inside = ((px // 16) >= x0) & ((px // 16) < x1) & ((py // 16) >= y0) & ((py // 16) < y1)
        return np.where((a >= 1 / 255) & inside, a, 0.0)

    a1, a0 = alpha(1), alpha(0)   # front, back
    bg = 0.05
    ref = (pr.rgb[0, 1][None] * a1[:, None] + pr.rgb[0, 0][None] * (a0 * (1 - a1))[:, None]
           + bg * ((1 - a1) * (1 - a0))[:, None])
    np.testing.assert_allclose(img.rgb, ref, atol=1e-12)
    assert (a1 > 0).sum() > 50 and ((a1 > 0) & (a0 > 0)).sum() > 20


@pytest.mark.parametrize("double", [False, True])
def test_weights_plus_final_transmittance_is_one(double):
    scene = S.scene_uniform_cube(300, 31, log_scale_mean=-2.3, logit_mean=1.5)
    scene.sh[:] = 0
    scene.sh[:, 0, :] = np.float32(_dc_for_colour(1.0))
    views = _view(96, 80)
    pr = oracle.project(scene, views, 16, double)
    assert np.all(np.abs(pr.rgb[pr.tiles > 0] - 1) < 1e-6)
    bins = oracle.bin_sort(pr, views, 16, double)
    img = oracle.raster_fwd(pr, bins, views, 16, double)
    # colour 1 and bg 0: C = sum alpha_i T_i
    total = img.rgb[:, 0] + img.T
    np.testing.assert_allclose(total, 1.0, atol=1e-12 if double else 2e-5)
    assert (img.T < 0.5).sum() > 100 and (img.T < 1e-3).sum() > 10  # the early stop is exercised


# ---------------------------------------------------------------------------
# backward: finite differences in float64
# ---------------------------------------------------------------------------

def _tiny_scene(seed, n=6):
    rng = np.random.default_rng(seed)
    means = rng.uniform(-0.5, 0.5, size=(n, 3))
    ls = rng.normal(math.log(0.25), 0.3, size=(n, 3))
    q = rng.normal(size=(n, 4))
    logits = rng.normal(0.0, 1.0, size=n)
    sh = rng.normal(0.0, 0.3, size=(n, 16, 3))
    sh[:, 0] = rng.normal(0.3, 0.5, size=(n, 3))
    return S.Scene(means, ls, q, logits, sh)   # float64 arrays for the float64 build


def _loss_linear(scene, views, w):
    img = oracle.raster_fwd(*(lambda pr: (pr, oracle.bin_sort(pr, views, 16, True)))(
        oracle.project(scene, views, 16, True)), views, 16, True)
    return float(np.sum(img.rgb * w))


def _analytic(scene, views, dLdC):
    pr = oracle.project(scene, views, 16, True)
    bins = oracle.bin_sort(pr, views, 16, True)
    _, g2 = oracle.raster_bwd(pr, bins, views, 16, dLdC, True)
    return oracle.project_bwd(scene, views, 16, g2, True)


def _fd(scene, views, loss, g, k, eps):
    flat = scene.flat().astype(np.float64)
    flat[:] = np.concatenate([scene.means, scene.log_scales, scene.quats,
                              scene.opacity_logits[:, None], scene.sh.reshape(scene.n, 48)], axis=1)

    def with_delta(d):
        f2 = flat.copy()
        f2[g, k] += d
        sc = S.Scene(f2[:, 0:3], f2[:, 3:6], f2[:, 6:10], f2[:, 10], f2[:, 11:].reshape(-1, 16, 3))
        return loss(sc)

    return (with_delta(eps) - with_delta(-eps)) / (2 * eps)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_matches_central_differences_linear_loss(seed):
    scene = _tiny_scene(100 + seed)
    views = S.views_array([S.make_view(32, 32, (0.0, 0.0, -4.0), bg=(0.2, 0.1, 0.3)),
                           S.make_view(40, 24, (1.0, 0.5, -3.5), bg=(0.0, 0.0, 0.0))])
    P = sum(oracle.n_pixels(views))
    w = np.random.default_rng(seed).uniform(-1, 1, size=(P, 3))
    an = _analytic(scene, views, w)
    assert np.all(np.abs(an).max(0) > 0), "every parameter receives a gradient"
    loss = lambda sc: _loss_linear(sc, views, w)
    rms = math.sqrt(np.mean(an ** 2))
    for g in range(scene.n):
        for k in range(59):
            fd = _fd(scene, views, loss, g, k, 1e-6)
            assert abs(fd - an[g, k]) <= 1e-5 * abs(an[g, k]) + 1e-6 * rms, (g, k, fd, an[g, k])


def test_backward_matches_central_differences_l1_loss():
    scene = _tiny_scene(7, n=8)
    views = _view(32, 32, bg=(0.1, 0.1, 0.1))
    target = S.random_image(32, 32, 5)
    pr = oracle.project(scene, views, 16, True)
    bins = oracle.bin_sort(pr, views, 16, True)
    img = oracle.raster_fwd(pr, bins, views, 16, True)
    _, dLdC = oracle.l1(img.rgb, target, True)
    an = _analytic(scene, views, dLdC)

    def loss(sc):
        p2 = oracle.project(sc, views, 16, True)
        b2 = oracle.bin_sort(p2, views, 16, True)
        return oracle.l1(oracle.raster_fwd(p2, b2, views, 16, True).rgb, target, True)[0]

    rms = math.sqrt(np.mean(an ** 2))
    for g in range(scene.n):
        for k in range(59):
            fd = _fd(scene, views, loss, g, k, 1e-6)
            assert abs(fd - an[g, k]) <= 1e-5 * abs(an[g, k]) + 1e-6 * rms, (g, k, fd, an[g, k])


def test_clamped_alpha_passes_no_gradient_to_opacity():
    # a very opaque, wide Gaussian: o*G > 0.99 on the pixels nearest its centre
    sh = np.zeros((1, 16, 3))
    sh[0, 0] = _dc_for_colour([0.7, 0.7, 0.7])
    scene = S.Scene(np.zeros((1, 3)), np.full((1, 3), math.log(1.0)), np.array([[1.0, 0, 0, 0]]),
                    np.array([8.0]), sh)
    views = _view(32, 32)
    pr = oracle.project(scene, views, 16, True)
    bins = oracle.bin_sort(pr, views, 16, True)
    img = oracle.raster_fwd(pr, bins, views, 16, True)
    w = np.ones((32 * 32, 3))
    an = _analytic(scene, views, w)
    fd = _fd(scene, views, lambda sc: _loss_linear(sc, views, w), 0, 10, 1e-6)
    assert abs(fd - an[0, 10]) <= 1e-6 * max(1.0, abs(an[0, 10]))
    assert (img.T <= 0.0100001).sum() > 0   # some pixels saturate at the clamp
    assert (img.T > 0.0100001).sum() > 0    # and the others still pass gradient to o


# ---------------------------------------------------------------------------
# loss and optimiser against torch (CPU)
# ---------------------------------------------------------------------------

def test_l1_gradient_matches_torch_autograd():
    import torch
    rng = np.random.default_rng(4)
    img = rng.uniform(0, 1, size=(500, 3))
    img[::17] = 0.25
    tgt = rng.uniform(0, 1, size=(500, 3)).astype(np.float32)
    tgt[::17] = 0.25
    loss, g = oracle.l1(img, tgt)
    x = torch.tensor(img, dtype=torch.float64, requires_grad=True)
    ref = torch.nn.functional.l1_loss(x, torch.tensor(tgt, dtype=torch.float64))
    ref.backward()
    assert loss == pytest.approx(ref.item(), rel=1e-14)
    np.testing.assert_allclose(g, x.grad.numpy(), rtol=1e-14, atol=0)


def test_adam_matches_torch_optim_adam():
    import torch
    rng = np.random.default_rng(5)
    n = 64
    params = rng.normal(size=(n, 59)).astype(np.float32)
    lrs = [1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1.25e-4]
    groups = [slice(0, 3), slice(3, 6), slice(6, 10), slice(10, 11), slice(11, 14), slice(14, 59)]
    tp = [torch.tensor(params[:, s].astype(np.float64), requires_grad=True) for s in groups]
    opt = torch.optim.Adam([{"params": [t], "lr": lr} for t, lr in zip(tp, lrs)],
                           betas=(0.9, 0.999), eps=1e-15)
    p = params.copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for step in range(1, 4):
        grads = rng.normal(size=(n, 59)) * 10.0 ** rng.integers(-6, 1, size=(n, 59))
        for t, s in zip(tp, groups):
            t.grad = torch.tensor(grads[:, s])
        opt.step()
        oracle.adam(p, m, v, grads, lrs, step)
        ref = np.concatenate([t.detach().numpy() for t in tp], axis=1)
        np.testing.assert_allclose(p, ref, rtol=2e-6, atol=1e-7)


# ---------------------------------------------------------------------------
# the two oracle builds agree on a full step (plain-method workload)
# ---------------------------------------------------------------------------

def test_float32_oracle_agrees_with_float64_oracle_on_full_step():
    w = S.workload_plain_small()
    target = oracle.render(w.target_scene, w.views, 16)
    r32 = oracle.train_step(w.scene, w.views, 16, target)
    r64 = oracle.train_step(w.scene, w.views, 16, target, double=True)
    np.testing.assert_array_equal(r32.proj.tiles, r64.proj.tiles)
    ok = r32.fragile == 0
    assert ok.mean() > 0.999
    assert np.abs(r32.image.rgb - r64.image.rgb)[ok].max() < 1e-4
    ex = exempt_gaussians(r64.proj, r64.bins, w.views, 16, r32.fragile | r64.fragile)[0]
    ok_g = grad_close(r32.grads, r64.grads)
    # every mismatch is a Gaussian a fragile pixel can composite, and mismatches are rare
    assert np.all(ok_g[~ex]), np.argwhere(~ok_g & ~ex[:, None])[:10]
    assert (~ok_g).any(axis=1).mean() < 0.01
    # with the image gradient zeroed at the fragile pixels of either build and
    # given to both, every Gaussian's gradient agrees
    dLdC = masked_image_gradient(r32.dLdC, r32.fragile | r64.fragile)
    g32 = oracle.train_step(w.scene, w.views, 16, None, dLdC=dLdC, adam_step=False).grads
    g64 = oracle.train_step(w.scene, w.views, 16, None, dLdC=dLdC, adam_step=False, double=True).grads
    assert grad_close(g32, g64).all()


def test_pixel_support_covers_every_gaussian_a_pixel_composites():
    """Flagging every pixel marks every (view, Gaussian) with a gradient, and
    only listed ones; one pixel's support holds exactly the Gaussians whose
    partials at that pixel alone are non-zero, within the margin's reach."""
    w = S.workload_plain_small()
    views = w.views
    pr = oracle.project(w.scene, views, 16)
    bins = oracle.bin_sort(pr, views, 16)
    P = 256 * 256
    allpix = np.ones(P, np.uint8)
    sup = oracle.pixel_support(pr, bins, views, 16, allpix)[0]
    img = oracle.raster_fwd(pr, bins, views, 16)
    _, g2 = oracle.raster_bwd(pr, bins, views, 16, np.full((P, 3), 1.0))
    has = np.abs(g2[0]).max(axis=1) > 0
    assert np.all(sup[has])
    listed = np.zeros(w.scene.n, bool)
    listed[bins.gid] = True
    assert not np.any(sup & ~listed)
    # single pixels: the Gaussians whose partials from that pixel are non-zero
    rng = np.random.default_rng(11)
    busy = np.flatnonzero(img.last >= 5)
    for p in rng.choice(busy, size=20, replace=False):
        one = np.zeros(P, np.uint8)
        one[p] = 1
        s1 = oracle.pixel_support(pr, bins, views, 16, one)[0]
        g = np.zeros((P, 3))
        g[p] = 1.0
        _, gp = oracle.raster_bwd(pr, bins, views, 16, g)
        comp = np.abs(gp[0]).max(axis=1) > 0
        assert np.all(s1[comp])
        # the margin adds few beyond the composited ones
        assert s1.sum() <= comp.sum() + 3 + comp.sum() // 4, (s1.sum(), comp.sum())


def test_l1_sign_tie_flag_skips_pixels_that_composited_nothing():
    img = np.array([[0.1, 0.2, 0.05], [0.3, 0.3, 0.3], [0.5, 0.5, 0.5]])
    tgt = np.array([[0.1, 0.2, 0.05], [0.3, 0.3, 0.3], [0.2, 0.6, 0.9]], np.float32)
    tgt64 = tgt.astype(np.float64)
    img[:2] = tgt64[:2]
    fr = np.zeros(3, np.uint8)
    _, g = oracle.l1(img, tgt, fragile=fr, last=np.array([0, 4, 2], np.uint32))
    # pixel 0: background, exact tie, nothing composited -> not flagged;
    # pixel 1: tie where something composited -> flagged; pixel 2: sign certain
    assert fr.tolist() == [0, 1, 0]
    assert np.all(g[0] == 0) and np.all(g[1] == 0)
    fr2 = np.zeros(3, np.uint8)
    oracle.l1(img, tgt, fragile=fr2)
    assert fr2[0] == 1


# ---------------------------------------------------------------------------
# exact tile culling (opacity-threshold ellipse, scan-line spans)
# ---------------------------------------------------------------------------

def test_log_spec_within_few_ulp_of_log():
    xs = np.concatenate([np.geomspace(1.0001, 300.0, 3001), np.geomspace(1e-3, 0.999, 500),
                         [1.0 + 2.0 ** -20, 2.0, 255.0, 0.5, 1.5, 1.41421356]]).astype(np.float32)
    for x in xs:
        exact = math.log(float(x))
        got = oracle.log_spec(float(x))
        tol = 4.0 * float(np.spacing(np.float32(abs(exact)))) + 1e-12
        assert abs(got - exact) <= tol, (x, got, exact)
    assert oracle.log_spec(3.7, double=True) == math.log(3.7)


def _box_min_q(A, B, C, xl, xh, yl, yh):
    """min of A x^2 + 2 B x y + C y^2 over the box [xl, xh] x [yl, yh] (float64);
    convex, so the minimum is 0 inside or on an edge at the clamped 1D minimiser."""
    if xl <= 0.0 <= xh and yl <= 0.0 <= yh:
        return 0.0
    q = lambda x, y: A * x * x + 2.0 * B * x * y + C * y * y
    best = math.inf
    for x in (xl, xh):
        y = min(max(-B * x / C, yl), yh)
        best = min(best, q(x, y))
    for y in (yl, yh):
        x = min(max(-B * y / A, xl), xh)
        best = min(best, q(x, y))
    return best


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_ellipse_tiles_match_brute_force_box_minimum(tile):
    rng = np.random.default_rng(7000 + tile)
    W, H = 333, 197
    gx, gy = (W + tile - 1) // tile, (H + tile - 1) // tile
    checked = fragile = 0
    for _ in range(300):
        # 2D covariance with a random orientation and aspect ratio up to 40
        s1, s2 = np.exp(rng.uniform(np.log(0.8), np.log(60.0), 2))
        th = rng.uniform(0, np.pi)
        R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
        S2 = R @ np.diag([s1 * s1, s2 * s2]) @ R.T
        Q = np.linalg.inv(S2)
        A, B, C = (float(np.float32(Q[0, 0])), float(np.float32(Q[0, 1])), float(np.float32(Q[1, 1])))
        u, v = (float(np.float32(x)) for x in rng.uniform([-60, -60], [W + 60, H + 60]))
        o = float(np.float32(np.exp(rng.uniform(np.log(0.002), 0.0))))
        mask = oracle.ellipse_tiles(u, v, A, B, C, o, tile, gx, gy)
        if 255.0 * o <= 1.0:
            assert mask.sum() == 0
            continue
        tau = 2.0 * math.log(255.0 * o)
        for ty in range(gy):
            for tx in range(gx):
                m = _box_min_q(A, B, C, tx * tile - u, (tx + 1) * tile - u, ty * tile - v,
                               (ty + 1) * tile - v)
                if abs(m - tau) <= 1e-4 * tau + 1e-9:
                    fragile += 1
                    continue
                checked += 1
                assert bool(mask[ty, tx]) == (m <= tau), (u, v, A, B, C, o, tx, ty, m, tau)
    assert checked > 10000 and fragile < 1e-3 * checked


def test_ellipse_emission_follows_the_spans_and_counts():
    scene, views, _, _ = _two_view_bins()
    pr = oracle.project(scene, views, 16, cull=oracle.CULL_ELLIPSE)
    bins = oracle.bin_sort(pr, views, 16)
    prr = oracle.project(scene, views, 16)
    n = scene.n
    assert bins.keys.size < oracle.bin_sort(prr, views, 16).keys.size
    for vi, vw in enumerate(views):
        gx = (int(vw["width"]) + 15) // 16
        gy = (int(vw["height"]) + 15) // 16
        D = oracle.depth_bits(gx * gy)
        for g in range(n):
            o = vi * n + g
            b, e = int(bins.offsets[o]), int(bins.offsets[o + 1])
            assert e - b == pr.tiles[vi, g]
            u, v = pr.xy[vi, g]
            A, B, C = pr.conic[vi, g]
            mask = oracle.ellipse_tiles(u, v, A, B, C, pr.opacity[vi, g], 16, gx, gy) \
                if prr.tiles[vi, g] or e > b else np.zeros((gy, gx), np.uint8)
            want = np.flatnonzero(mask.reshape(-1))       # row-major = emission order
            np.testing.assert_array_equal(bins.keys_unsorted[b:e] >> D, want)
            if e > b:
                x0, y0, x1, y1 = pr.rect[vi, g]
                ty, tx = np.divmod(want, gx)
                assert ty.min() >= y0 and ty.max() < y1 and tx.min() >= x0 and tx.max() < x1


def test_ellipse_culling_changes_no_pixel_below_the_three_sigma_opacity():
    # with o <= 0.35 the opacity ellipse lies inside the 3-sigma box, so exact
    # culling only drops entries that composite nowhere: same pixels, same order
    rng = np.random.default_rng(7100)
    n = 1500
    scene = _scene_from(rng.uniform(-1, 1, (n, 3)), rng.normal(-3.0, 0.5, (n, 3)),
                        rng.normal(size=(n, 4)), np.log(np.full(n, 0.3) / 0.7) + rng.uniform(-4, 0, n),
                        rng.normal(0, 0.3, (n, 48)))
    views = S.views_array([S.make_view(200, 150, (0.0, 0.0, -4.0), bg=(0.1, 0.2, 0.3)),
                           S.make_view(123, 77, (3.0, 1.0, -2.0))])
    for double in (False, True):
        pr = oracle.project(scene, views, 16, double)
        pe = oracle.project(scene, views, 16, double, oracle.CULL_ELLIPSE)
        br, be = oracle.bin_sort(pr, views, 16, double), oracle.bin_sort(pe, views, 16, double)
        assert be.keys.size < 0.8 * br.keys.size
        ir = oracle.raster_fwd(pr, br, views, 16, double)
        ie = oracle.raster_fwd(pe, be, views, 16, double)
        ok = (ir.fragile == 0) & (ie.fragile == 0)
        assert ok.mean() > 0.99
        np.testing.assert_array_equal(ir.rgb[ok], ie.rgb[ok])
        np.testing.assert_array_equal(ir.T[ok], ie.T[ok])


def test_running_error_bound_dominates_the_sums_it_bounds():
    """mag2d (the float32 running error bound of the screen-space sums, in
    rounding units) is at least 8 times the sum of absolute terms, so it bounds
    |grads2d| by the triangle inequality, and is positive wherever a sum is
    non-zero; the projection backward carries it linearly (one component at a
    time), so the parameter bound also dominates the parameter gradients."""
    w = S.workload_plain_small()
    views = w.views
    target = oracle.render(w.target_scene, views, 16)
    r = oracle.train_step(w.scene, views, 16, target, adam_step=False)
    pr = oracle.project(w.scene, views, 16)
    bins = oracle.bin_sort(pr, views, 16)
    _, g2, m2 = oracle.raster_bwd(pr, bins, views, 16, r.dLdC, magnitudes=True)
    np.testing.assert_array_equal(g2, r.grads2d)
    assert np.all(np.abs(g2) * 8.0 <= m2 * (1 + 1e-12))
    assert np.all(m2[np.abs(g2) > 0] > 0)
    M = oracle.project_bwd_magnitudes(w.scene, views, 16, m2)
    assert np.all(np.abs(r.grads) * 8.0 <= M * (1 + 1e-9) + 1e-300)
