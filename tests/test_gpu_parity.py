"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: bit-exact for tile rectangles, counts, offsets, keys, values and ranges;
pixels within 1e-4 (max abs) outside pixels whose compositing decisions lie at
a threshold ("fragile", counted); gradients within 1e-3 relative (floored at
1e-2 of the column maximum); updated parameters within 1e-3 relative, except
where the oracle's gradient is too small for its sign to be certain (Adam's
first step moves such parameters by +-lr, so those are held to 2 lr).
"""
import math

import numpy as np
import pytest

import oracle
import synthetic as S
from gpu_common import note, per_gaussian_2d, rect_from_packed, run_gpu_step
from helpers import checked_fraction, exempt_gaussians, grad_close, masked_image_gradient

pytestmark = pytest.mark.gpu

PIX_TOL = 1e-4
GRAD_RTOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_00219_amd import _lib  # noqa: F401  (fails loudly if not built)
    yield


def _workloads():
    w1 = S.workload_plain_small()
    # two views of different (ragged) sizes, tile edge not dividing the image
    scene = S.scene_uniform_cube(3000, 77, log_scale_mean=-3.2)
    target_scene = S.scene_uniform_cube(3000, 78, log_scale_mean=-3.2)
    views = S.views_array([S.make_view(200, 150, (0.5, -0.3, -4.0), bg=(0.1, 0.2, 0.05)),
                           S.make_view(333, 97, (-2.0, 1.0, -3.0))])
    # the sparse-footprint distribution (log-scales N(-6, 0.3)): sub-pixel
    # Gaussians, about 1.5 tiles each, many never reaching alpha 1/255 at a
    # pixel centre
    cams = S.fibonacci_sphere(50, 5.0)
    sub = (S.scene_normal(20000, 9200, log_scale_mean=-6.0, log_scale_std=0.3),
           S.scene_normal(20000, 9201, log_scale_mean=-6.0, log_scale_std=0.3),
           S.views_array([S.make_view(640, 360, cams[3]), S.make_view(320, 240, cams[17])]), 16)
    return {"plain-2k-256": (w1.scene, w1.target_scene, w1.views, 16),
            "ragged-2view": (scene, target_scene, views, 16),
            "subpixel-20k-2view": sub}


WL = _workloads()


def _oracle_step(scene, target_scene, views, tile, lr=1e-3):
    target = oracle.render(target_scene, views, tile)
    return target, oracle.train_step(scene, views, tile, target, lr=lr)


@pytest.mark.parametrize("name", list(WL))
@pytest.mark.parametrize("order", ["direct", "depth_first"])
def test_projection_and_binning_bit_exact(name, order):
    """Both sort orders: all 32 key bits directly (few intersections per
    Gaussian, the fitted capacity) and depth bits of the Gaussians first, then
    tile bits (chosen when the capacity is at least 12 x views x n)."""
    scene, target_scene, views, tile = WL[name]
    note(f"projection/binning parity {name} ({order})")
    ref = oracle.train_step(scene, views, tile, oracle.render(target_scene, views, tile), adam_step=False)
    cap = None if order == "direct" else 16 * len(views) * scene.n
    if order == "direct":
        assert int(ref.bins.offsets[-1]) * 1.25 + 1024 < 12 * len(views) * scene.n
    g = run_gpu_step(scene, views, tile, capacity=cap)
    assert g["status"] == 0
    np.testing.assert_array_equal(g["tiles"], ref.proj.tiles)
    vis = ref.proj.tiles > 0
    assert vis.sum() > 100
    np.testing.assert_array_equal(rect_from_packed(g["rect"])[vis], ref.proj.rect[vis])
    # float outputs: same operation order without contraction -> same bits
    f32 = lambda a: a.astype(np.float32)
    rec = g["rec"]
    fields = {0: ref.proj.xy[..., 0], 1: ref.proj.xy[..., 1], 2: ref.proj.conic[..., 0],
              3: ref.proj.conic[..., 1], 4: ref.proj.conic[..., 2], 5: ref.proj.opacity,
              6: ref.proj.rgb[..., 0], 7: ref.proj.rgb[..., 1], 8: ref.proj.rgb[..., 2],
              9: ref.proj.depth, 10: ref.proj.radius}
    for k, want in fields.items():
        np.testing.assert_array_equal(rec[..., k][vis], f32(want)[vis], err_msg=f"record field {k}")
    # depth code: mantissa of the float32 (2z + 1) / (z + 1)
    z = f32(ref.proj.depth)
    fz = (np.float32(2) * z + np.float32(1)) / (z + np.float32(1))
    np.testing.assert_array_equal(rec[..., 14].view(np.uint32)[vis], (fz.view(np.uint32) & 0x7FFFFF)[vis])
    # binning: keys, the Gaussian id carried by the sort, ranges
    np.testing.assert_array_equal(g["offsets"], ref.bins.offsets)
    np.testing.assert_array_equal(g["keys"], ref.bins.keys)
    np.testing.assert_array_equal(g["vals"], ref.bins.gid[ref.bins.vals])
    np.testing.assert_array_equal(g["ranges"], ref.bins.ranges)


def test_depth_first_sort_with_more_tiles_than_one_scatter_pass_takes():
    """Depth-first order with a view of 20,480 tiles (1280x1024 at 8-pixel
    tiles, more than the 4,096 a single tile partition handles): the depth
    order takes the low 16 key bits and radix passes sort the rest; keys,
    values and ranges bit for bit; the same with 3,600 tiles (the single
    partition) on the same scene."""
    scene = S.scene_normal(20_000, 6100, log_scale_mean=-3.5)
    for W, H, tile in ((1280, 1024, 8), (1280, 720, 16)):
        views = S.views_array([S.make_view(W, H, (0.5, 0.2, -5.0))])
        note(f"depth-first binning, {W}x{H} at tile {tile}")
        pr = oracle.project(scene, views, tile)
        bins = oracle.bin_sort(pr, views, tile)
        K = int(bins.offsets[-1])
        cap = max(16 * scene.n, int(1.25 * K) + 1024)     # at least 12 x n: depth first
        g = run_gpu_step(scene, views, tile, capacity=cap)
        assert g["status"] == 0
        np.testing.assert_array_equal(g["offsets"], bins.offsets)
        np.testing.assert_array_equal(g["keys"], bins.keys)
        np.testing.assert_array_equal(g["vals"], bins.gid[bins.vals])
        np.testing.assert_array_equal(g["ranges"], bins.ranges)


def _tile_of_pixel(views, tile):
    """Global tile index of every pixel (views concatenated)."""
    out, tb = [], 0
    for v in views:
        W, H = int(v["width"]), int(v["height"])
        gx, gy = (W + tile - 1) // tile, (H + tile - 1) // tile
        iy, ix = np.divmod(np.arange(W * H), W)
        out.append(tb + (iy // tile) * gx + ix // tile)
        tb += gx * gy
    return np.concatenate(out)


@pytest.mark.parametrize("name,tile,ppl", [("plain-2k-256", 16, 1), ("plain-2k-256", 16, 2),
                                           ("plain-2k-256", 16, 4), ("plain-2k-256", 8, 1),
                                           ("plain-2k-256", 32, 2), ("ragged-2view", 16, 2),
                                           ("ragged-2view", 32, 4)])
def test_tile_statistics(name, tile, ppl):
    """Per tile: the most list entries any pixel examined and the pixel-Gaussian
    pairs examined, equal to the oracle's on tiles without a fragile pixel."""
    scene, _, views, _ = WL[name]
    note(f"tile statistics {name} tile={tile} pixels/lane={ppl}")
    pr = oracle.project(scene, views, tile)
    bins = oracle.bin_sort(pr, views, tile)
    ref = oracle.raster_fwd(pr, bins, views, tile)
    g = run_gpu_step(scene, views, tile, pixels_per_lane=ppl, tile_stats=True)
    st = g["tile_stats"].reshape(-1, 4).astype(np.int64)
    nt = st.shape[0]
    frag = np.zeros(nt, bool)
    frag[_tile_of_pixel(views, tile)[ref.fragile != 0]] = True
    ok = ~frag
    assert ok.mean() > 0.8      # large tiles: few tiles, more of them hold a fragile pixel
    np.testing.assert_array_equal(st[ok, 0], ref.tile_traversed[ok].astype(np.int64))
    np.testing.assert_array_equal(st[ok, 1], ref.tile_evaluated[ok].astype(np.int64))
    assert np.all(st[:, 2] <= st[:, 1])
    assert st[:, 2].sum() > 0


@pytest.mark.parametrize("name", list(WL))
@pytest.mark.parametrize("lds_batch,ppl", [(32, 4), (64, 1), (64, 2), (256, 4)])
def test_forward_pixels(name, lds_batch, ppl):
    scene, target_scene, views, tile = WL[name]
    note(f"forward parity {name} S={lds_batch} pixels/lane={ppl}")
    ref = oracle.train_step(scene, views, tile, oracle.render(target_scene, views, tile), adam_step=False)
    g = run_gpu_step(scene, views, tile, lds_batch=lds_batch, pixels_per_lane=ppl)
    ok = ref.image.fragile == 0
    assert ok.mean() > 0.995, f"fragile fraction {1 - ok.mean():.4f}"
    err = np.abs(g["image"] - ref.image.rgb).max(axis=1)
    assert err[ok].max() <= PIX_TOL, err[ok].max()
    assert np.abs(g["T"] - ref.image.T)[ok].max() <= PIX_TOL
    np.testing.assert_array_equal(g["last"][ok], ref.image.last[ok])
    note(f"  max pixel err {err[ok].max():.2e}, fragile {int((~ok).sum())} px, "
         f"last mismatches at fragile {int((g['last'] != ref.image.last).sum())}")


def _check_step(g, ref, views, tile, n, ex, floor, label=""):
    """Records, per-(view, Gaussian) sums, parameter gradients and the Adam
    update of a GPU step against the oracle's, every (view, Gaussian) outside
    ex held to the bar; returns the checked fraction."""
    V = len(views)
    ex_any = ex.any(axis=0)
    touched = np.abs(ref.grads).max(axis=1) > 0
    frac = checked_fraction(ex_any, touched, floor, label)
    # per-Gaussian 2D gradients (sums of the intersection records)
    tb = np.cumsum([0] + oracle.n_tiles(views, tile))
    g2 = per_gaussian_2d(g["grec"], ref.bins.vals, g["vals"], g["ranges"], g["tile_stop"], tb, n)
    # traversal stops are within the ranges
    stop = g["tile_stop"]
    assert np.all(stop >= g["ranges"][:, 0]) and np.all(stop <= g["ranges"][:, 1])
    assert (stop < g["ranges"][:, 1]).any()
    # records: written (flagged) exactly for the traversed entries some pixel
    # composited; they match the oracle's partials at the same unsorted index,
    # and the traversed entries without a record have no oracle gradient
    bit = lambda m, i: (m[i >> 5] >> (i & 31)) & 1
    pos = [np.arange(int(g["ranges"][t, 0]), int(stop[t])) for t in range(len(stop))]
    pview = np.concatenate([np.full(len(p_), np.searchsorted(tb, t, side="right") - 1) for t, p_ in
                            enumerate(pos)]).astype(np.int64)
    pos = np.concatenate(pos).astype(np.int64)
    trav = ref.bins.vals[pos].astype(np.int64)
    comp = bit(g["comp_mask"], pos).astype(bool)
    flag = bit(g["rec_mask"], trav).astype(bool)
    np.testing.assert_array_equal(comp, flag)
    assert flag.any() and not flag.all()
    exr = ex[pview, g["vals"][pos]]
    okr = grad_close(g["grec"][trav, :9], ref.partials[trav], GRAD_RTOL).all(axis=1)
    badr = flag & ~okr & ~exr
    assert not badr.any(), (pos[badr][:5], trav[badr][:5])
    # each written record names its (view, Gaussian)
    owner = np.ascontiguousarray(g["grec"][trav[flag], 9]).view(np.uint32)
    np.testing.assert_array_equal(owner, (pview * n + g["vals"][pos])[flag])
    assert not (~flag & (np.abs(ref.partials[trav]).max(axis=1) > 0) & ~exr).any()
    untrav = np.setdiff1d(np.arange(g["K"]), trav)
    assert not bit(g["rec_mask"], untrav).any()
    ok2 = grad_close(g2.reshape(-1, 9), ref.grads2d.reshape(-1, 9), GRAD_RTOL).reshape(V, n, 9)
    bad = ~ok2.all(axis=2) & ~ex
    assert not bad.any(), np.argwhere(bad)[:5]
    # the gather's per-(view, Gaussian) sums equal the sums of the records
    oks = grad_close(g["sums"].reshape(-1, 9), g2.reshape(-1, 9), 1e-5)
    assert oks.all(), np.argwhere(~oks)[:5]
    # parameter gradients
    okg = grad_close(g["grads"], ref.grads, GRAD_RTOL)
    badg = ~okg.all(axis=1) & ~ex_any
    assert not badg.any(), (np.argwhere(~okg & ~ex_any[:, None])[:5])
    assert (~okg.all(axis=1)).mean() < 0.02
    # updated parameters after one Adam step
    p0 = g["p0"]
    lr = 1e-3
    gmax = np.abs(ref.grads).max(axis=0, keepdims=True)
    certain = np.abs(ref.grads) >= 1e-3 * gmax
    diff = np.abs(g["params"] - ref.params)
    tol = np.where(certain, 1e-3 * np.abs(ref.params) + 1e-6, 2 * lr + 1e-6)
    badp = (diff > tol) & ~ex_any[:, None]
    assert not badp.any(), np.argwhere(badp)[:5]
    # every parameter moved by about lr (Adam step 1 with eps = 1e-15)
    moved = np.abs(g["params"] - p0)
    assert np.median(moved[np.abs(ref.grads) > 0]) == pytest.approx(lr, rel=1e-3)
    note(f"  sign-uncertain {int((~certain).sum())} elems")
    return frac


# share of the Gaussians with a gradient that must stay checked when the fused
# L1 gradient is used (the fragile pixels of these dense scenes each reach 30-40
# Gaussians); with a given image gradient zeroed at fragile pixels it is all
L1_CHECKED_FLOOR = {"plain-2k-256": 0.8, "ragged-2view": 0.7, "subpixel-20k-2view": 0.95}


@pytest.mark.parametrize("name", list(WL))
@pytest.mark.parametrize("ppl", [1, 2, 4])
def test_training_step(name, ppl):
    """The whole step with the fused L1 gradient: the loss, then records, sums,
    gradients and updates of every Gaussian no fragile pixel can reach."""
    scene, target_scene, views, tile = WL[name]
    note(f"training-step parity {name} pixels/lane={ppl}")
    target, ref = _oracle_step(scene, target_scene, views, tile)
    g = run_gpu_step(scene, views, tile, target=target, pixels_per_lane=ppl)
    g["p0"] = scene.flat()
    loss_gpu = g["loss_tiles"].astype(np.float64).sum() / (3 * sum(oracle.n_pixels(views)))
    assert abs(loss_gpu - ref.loss) <= 1e-4 * ref.loss
    ex = exempt_gaussians(ref.proj, ref.bins, views, tile, ref.fragile)
    _check_step(g, ref, views, tile, scene.n, ex, L1_CHECKED_FLOOR[name])


@pytest.mark.parametrize("name,tile,ppl,variant", [("plain-2k-256", 16, 2, None),
                                                   ("subpixel-20k-2view", 16, 1, None),
                                                   ("plain-2k-256", 16, 1, ("twophase", 32)),
                                                   ("ragged-2view", 8, 1, None),
                                                   ("ragged-2view", 16, 2, None),
                                                   ("ragged-2view", 16, 4, ("twophase", 16)),
                                                   ("ragged-2view", 32, 4, None)])
def test_training_step_every_gaussian(name, tile, ppl, variant):
    """The oracle's L1 image gradient with its fragile pixels zeroed, given to
    both sides: no pixel whose decisions may differ adds to any gradient, so
    the records, sums, all 59 gradients and all updates of every Gaussian are
    held to the bar (no exemption)."""
    scene, target_scene, views, _ = WL[name]
    note(f"training-step parity, every Gaussian: {name} tile={tile} pixels/lane={ppl} {variant}")
    target = oracle.render(target_scene, views, tile)
    fwd = oracle.train_step(scene, views, tile, target, adam_step=False)
    dLdC = masked_image_gradient(fwd.dLdC, fwd.fragile)
    ref = oracle.train_step(scene, views, tile, None, dLdC=dLdC)
    assert not (ref.fragile & ~fwd.fragile).any()      # compositing flags are a subset
    g = run_gpu_step(scene, views, tile, dLdC=dLdC, lds_batch=128, pixels_per_lane=ppl, bwd_batch=variant)
    g["p0"] = scene.flat()
    ex = np.zeros((len(views), scene.n), bool)
    frac = _check_step(g, ref, views, tile, scene.n, ex, 1.0)
    assert frac == 1.0
    # the fused L1 prologue gives the records of the same backward fed the L1
    # gradient of the GPU's own render (sign(C - target) / 3P in float32)
    fused = run_gpu_step(scene, views, tile, target=target, lds_batch=128, pixels_per_lane=ppl,
                         bwd_batch=variant)
    P = sum(oracle.n_pixels(views))
    d = fused["image"].astype(np.float32) - np.asarray(target, np.float32).reshape(-1, 3)
    inv = np.float32(1.0) / (np.float32(3.0) * np.float32(P))
    own = (np.sign(d).astype(np.float32) * inv).astype(np.float32)
    given = run_gpu_step(scene, views, tile, dLdC=own, lds_batch=128, pixels_per_lane=ppl, bwd_batch=variant)
    for k in ("grec", "rec_mask", "tile_stop", "sums", "grads", "params"):
        np.testing.assert_array_equal(fused[k], given[k], err_msg=k)


def test_deterministic_bitwise():
    scene, target_scene, views, tile = WL["plain-2k-256"]
    note("determinism")
    target = oracle.render(target_scene, views, tile)
    a = run_gpu_step(scene, views, tile, target=target)
    b = run_gpu_step(scene, views, tile, target=target)
    for k in ("image", "grec", "rec_mask", "comp_mask", "tile_stop", "sums", "grads", "params", "keys",
              "vals"):
        np.testing.assert_array_equal(a[k], b[k])


def test_persistent_and_permuted_schedules_change_no_bit():
    scene, target_scene, views, tile = WL["ragged-2view"]
    note("schedule invariance")
    target = oracle.render(target_scene, views, tile)
    base = run_gpu_step(scene, views, tile, target=target)
    nt = sum(oracle.n_tiles(views, tile))
    perm = np.random.default_rng(3).permutation(nt).astype(np.int32)
    for kw in (dict(persistent=True), dict(sched_order=perm), dict(sched_order=perm, persistent=True)):
        other = run_gpu_step(scene, views, tile, target=target, **kw)
        for k in ("image", "T", "last", "grec", "rec_mask", "comp_mask", "tile_stop", "sums", "grads",
                  "params"):
            np.testing.assert_array_equal(base[k], other[k], err_msg=str(kw))


@pytest.mark.parametrize("name", ["plain-2k-256", "ragged-2view"])
def test_backward_batch_changes_no_bit(name):
    """The backward's LDS batch -- fixed 64 / 256, or per tile sqrt(N P) to a
    multiple of 64 capped at 64, 128, 256 -- changes the schedule, not a bit."""
    scene, target_scene, views, tile = WL[name]
    note(f"backward batch invariance {name}")
    target = oracle.render(target_scene, views, tile)
    base = run_gpu_step(scene, views, tile, target=target, lds_batch=128)
    for bb in (64, 256, -64, -128, -256):
        other = run_gpu_step(scene, views, tile, target=target, lds_batch=128, bwd_batch=bb)
        for k in ("grec", "rec_mask", "tile_stop", "sums", "grads", "params"):
            np.testing.assert_array_equal(base[k], other[k], err_msg=f"bwd_batch={bb} {k}")


@pytest.mark.parametrize("name,ppl,S", [("plain-2k-256", 1, 32), ("plain-2k-256", 2, 16), ("plain-2k-256", 4, 32),
                                        ("plain-2k-256", 1, 64), ("ragged-2view", 1, 16), ("ragged-2view", 2, 32),
                                        ("ragged-2view", 1, 64)])
def test_twophase_backward_against_oracle(name, ppl, S):
    """The two-phase backward: gradients and the Adam update against the oracle
    (same bar as the first backward), its records against the first backward's
    (equal up to float summation order), the same flagged records and stops."""
    scene, target_scene, views, tile = WL[name]
    note(f"two-phase backward {name} pixels/lane={ppl} S={S}")
    target, ref = _oracle_step(scene, target_scene, views, tile)
    g = run_gpu_step(scene, views, tile, target=target, lds_batch=128, pixels_per_lane=ppl,
                     bwd_batch=("twophase", S))
    base = run_gpu_step(scene, views, tile, target=target, lds_batch=128, pixels_per_lane=ppl)
    for k in ("rec_mask", "tile_stop"):
        np.testing.assert_array_equal(g[k], base[k])
    flagged = np.unpackbits(g["rec_mask"].view(np.uint8), bitorder="little")[:g["K"]].astype(bool)
    ra, rb = g["grec"][flagged][:, :9], base["grec"][flagged][:, :9]
    np.testing.assert_array_equal(g["grec"][flagged][:, 9].view(np.uint32),
                                  base["grec"][flagged][:, 9].view(np.uint32))          # owners
    scale = np.abs(rb).max(axis=0, keepdims=True) + 1e-30
    assert (np.abs(ra - rb) <= 1e-4 * scale + 1e-5 * np.abs(rb)).all()
    ex_any = exempt_gaussians(ref.proj, ref.bins, views, tile, ref.fragile).any(axis=0)
    checked_fraction(ex_any, np.abs(ref.grads).max(axis=1) > 0, L1_CHECKED_FLOOR[name])
    okg = grad_close(g["grads"], ref.grads, GRAD_RTOL)
    assert not (~okg.all(axis=1) & ~ex_any).any(), np.argwhere(~okg & ~ex_any[:, None])[:5]


def test_twophase_backward_tile8_and_determinism():
    scene, target_scene, views, _ = WL["ragged-2view"]
    note("two-phase backward, 8x8 tiles, twice")
    target, ref = _oracle_step(scene, target_scene, views, 8)
    a = run_gpu_step(scene, views, 8, target=target, lds_batch=64, bwd_batch=("twophase", 32))
    b = run_gpu_step(scene, views, 8, target=target, lds_batch=64, bwd_batch=("twophase", 32))
    c = run_gpu_step(scene, views, 8, target=target, lds_batch=64, bwd_batch=("twophase", 64))
    okc = grad_close(c["grads"], a["grads"], 1e-4)
    assert okc.all(), np.argwhere(~okc)[:5]
    for k in ("grec", "rec_mask", "sums", "grads", "params"):
        np.testing.assert_array_equal(a[k], b[k])
    ex_any = exempt_gaussians(ref.proj, ref.bins, views, 8, ref.fragile).any(axis=0)
    checked_fraction(ex_any, np.abs(ref.grads).max(axis=1) > 0, L1_CHECKED_FLOOR["ragged-2view"])
    okg = grad_close(a["grads"], ref.grads, GRAD_RTOL)
    assert not (~okg.all(axis=1) & ~ex_any).any()


def test_twophase_backward_argument_errors():
    from paper_2605_00219_amd import _lib as G
    from paper_2605_00219_amd import pipeline as P
    scene, _, views, _ = WL["plain-2k-256"]
    vd = P.views_to_device(views)
    frame = P.Frame(scene.n, [256], [256], 16)
    with pytest.raises(G.GsError, match="lds_batch"):
        P.rasterize_bwd_twophase(frame, vd, dLdC=frame.image, lds_batch=128)
    frame32 = P.Frame(scene.n, [256], [256], 32)
    with pytest.raises(G.GsError, match="tile"):
        P.rasterize_bwd_twophase(frame32, vd, dLdC=frame32.image, lds_batch=32)


def test_thompson_scheduled_backward_trains_the_same_bits():
    """Six training steps whose backward batch is chosen by Thompson sampling
    end with the parameters of six fixed-batch steps, bit for bit."""
    import torch
    from paper_2605_00219_amd import pipeline as P
    scene, target_scene, views, tile = WL["ragged-2view"]
    note("Thompson-scheduled backward, 6 steps")
    target = torch.as_tensor(np.ascontiguousarray(oracle.render(target_scene, views, tile), np.float32),
                             device="cuda").reshape(-1, 3)
    vd = P.views_to_device(views)
    outs = []
    for scheduled in (False, True):
        model = P.Model(scene.flat())
        frame = P.Frame(scene.n, [int(v["width"]) for v in views], [int(v["height"]) for v in views], tile)
        P.fit_capacity(model.params, frame, vd)
        sbwd = P.ScheduledBackward((64, 128, 256, -128), seed=2, prior_ms=0.05, time_every=1) if scheduled else None
        for _ in range(6):
            P.project(model.params, frame, vd)
            P.bin_sort(frame)
            P.rasterize_fwd(frame, vd, 128)
            if sbwd is None:
                P.rasterize_bwd(frame, vd, target=target, lds_batch=128)
            else:
                sbwd(frame, vd, target=target)
            P.project_bwd_adam(model, frame, vd)
        torch.cuda.synchronize()
        assert frame.status_bits() == 0
        outs.append(model.params.cpu().numpy())
        if sbwd is not None:
            sbwd.harvest(block=True)
            # every step's latency was folded in; which arms were tried depends on
            # timing (each arm's bits are checked directly in the batch test above)
            assert sum(sbwd.ts.counts()) == 6 and len(sbwd.history) == 6
    np.testing.assert_array_equal(outs[0], outs[1])


@pytest.mark.parametrize("tile,ppl", [(8, 1), (32, 1), (32, 2), (32, 4)])
def test_other_tile_sizes(tile, ppl):
    scene, target_scene, views, _ = WL["ragged-2view"]
    note(f"tile {tile} pixels/lane {ppl}")
    target, ref = _oracle_step(scene, target_scene, views, tile)
    g = run_gpu_step(scene, views, tile, target=target, lds_batch=128, pixels_per_lane=ppl)
    np.testing.assert_array_equal(g["keys"], ref.bins.keys)
    np.testing.assert_array_equal(g["ranges"], ref.bins.ranges)
    ok = ref.image.fragile == 0
    assert np.abs(g["image"] - ref.image.rgb).max(axis=1)[ok].max() <= PIX_TOL
    ex_any = exempt_gaussians(ref.proj, ref.bins, views, tile, ref.fragile).any(axis=0)
    checked_fraction(ex_any, np.abs(ref.grads).max(axis=1) > 0, L1_CHECKED_FLOOR["ragged-2view"])
    okg = grad_close(g["grads"], ref.grads, GRAD_RTOL)
    assert not (~okg.all(axis=1) & ~ex_any).any()


def test_empty_scene_and_culled_gaussians():
    note("edge: nothing visible")
    scene = S.scene_uniform_cube(500, 5)
    scene.means[:] = scene.means + np.float32([0, 0, -10])   # all behind the camera at z=-4
    scene.means[:7, 2] = np.float32(0)                        # a few visible
    scene.quats[3] = 0                                         # zero quaternion: culled
    scene.sh[5, 2, 1] = np.float32("nan")                      # non-finite: culled
    views = S.views_array([S.make_view(64, 48, (0, 0, -4.0))])
    target = S.random_image(48, 64, 1)
    ref = oracle.train_step(scene, views, 16, target)
    g = run_gpu_step(scene, views, 16, target=target)
    np.testing.assert_array_equal(g["tiles"], ref.proj.tiles)
    assert g["tiles"][0, 3] == 0 and g["tiles"][0, 5] == 0
    assert np.abs(g["image"] - ref.image.rgb).max() <= PIX_TOL
    okg = grad_close(g["grads"], ref.grads, GRAD_RTOL)
    assert okg.all()
    # a scene with no visible Gaussian at all
    scene.means[:, 2] = np.float32(-10)
    ref = oracle.train_step(scene, views, 16, target)
    g = run_gpu_step(scene, views, 16, target=target)
    assert g["K"] == 0 and ref.bins.offsets[-1] == 0
    np.testing.assert_array_equal(g["ranges"], ref.bins.ranges)
    assert np.all(g["image"] == 0) and np.all(g["T"] == 1)
    assert np.all(g["grads"] == 0)


@pytest.mark.parametrize("order", ["direct", "depth_first"])
def test_binning_with_a_view_that_sees_nothing(order):
    """Three views, the middle one looking away from the scene (no
    intersection): keys, values and every tile range bit-exact, through the
    direct 32-bit sort and k_ranges (capacity under 12 intersections per
    (view, Gaussian)) and through the depth order and the tile partition."""
    scene = WL["plain-2k-256"][0]
    views = S.views_array([S.make_view(256, 256, (0.0, 0.0, -5.0)),
                           S.make_view(128, 96, (0.0, 0.0, -4.0), target=(0.0, 0.0, -10.0)),
                           S.make_view(192, 160, (3.0, 1.0, -4.0))])
    note(f"binning, 3 views with an empty one, {order} order")
    pr = oracle.project(scene, views, 16)
    bins = oracle.bin_sort(pr, views, 16)
    assert pr.tiles[1].sum() == 0 and pr.tiles[0].sum() > 0 and pr.tiles[2].sum() > 0
    K, m = int(bins.offsets[-1]), 3 * scene.n
    capacity = K + 1024 if order == "direct" else 12 * m + 1024
    assert (capacity < 12 * m) == (order == "direct")
    g = run_gpu_step(scene, views, 16, capacity=capacity)
    assert g["status"] == 0 and g["K"] == K
    np.testing.assert_array_equal(g["keys"], bins.keys[:K])
    np.testing.assert_array_equal(g["vals"], bins.gid[bins.vals[:K]])
    np.testing.assert_array_equal(g["ranges"], bins.ranges)


def test_depth_first_order_with_long_tile_lists():
    """The depth order and the tile partition with a few long lists: 6000
    Gaussians clustered on the centre of a 128x128 view give four tiles of
    about 5000-6000 entries; keys, values and ranges bit-exact."""
    scene = S.scene_normal(6000, 9300, log_scale_mean=-3.5, log_scale_std=0.3)
    scene.means[:] = (scene.means * np.float32(0.05)).astype(np.float32)
    views = S.views_array([S.make_view(128, 128, (0.0, 0.0, -4.0))])
    note("depth order, tile lists past 4096 entries")
    pr = oracle.project(scene, views, 16)
    bins = oracle.bin_sort(pr, views, 16)
    K = int(bins.offsets[-1])
    lens = np.diff(bins.ranges.reshape(-1, 2), axis=1)
    assert lens.max() > 4096
    g = run_gpu_step(scene, views, 16, capacity=12 * scene.n + 1024)
    assert g["status"] == 0 and g["K"] == K
    np.testing.assert_array_equal(g["keys"], bins.keys[:K])
    np.testing.assert_array_equal(g["vals"], bins.gid[bins.vals[:K]])
    np.testing.assert_array_equal(g["ranges"], bins.ranges)


def test_capacity_overflow_is_reported_and_recovered():
    import torch
    from paper_2605_00219_amd import pipeline as P
    scene, target_scene, views, tile = WL["plain-2k-256"]
    note("edge: capacity overflow")
    model = P.Model(scene.flat())
    frame = P.Frame(scene.n, [256], [256], 16, capacity=1000)
    vd = P.views_to_device(views)
    P.project(model.params, frame, vd)
    P.bin_sort(frame)
    torch.cuda.synchronize()
    assert frame.status_bits() & 1
    ref = oracle.train_step(scene, views, tile, oracle.render(target_scene, views, tile), adam_step=False)
    assert frame.intersections() == int(ref.bins.offsets[-1]) > 1000
    # the step grows the buffers and succeeds
    target = torch.as_tensor(oracle.render(target_scene, views, tile), device="cuda")
    P.train_step(model, frame, vd, target)
    torch.cuda.synchronize()
    assert frame.status_bits() == 0 and frame.capacity >= frame.intersections()


def test_invalid_arguments_raise():
    from paper_2605_00219_amd import _lib as G
    from paper_2605_00219_amd import pipeline as P
    scene, _, views, _ = WL["plain-2k-256"]
    frame = P.Frame(scene.n, [256], [256], 16)
    vd = P.views_to_device(views)
    with pytest.raises(G.GsError, match="lds_batch"):
        P.rasterize_fwd(frame, vd, lds_batch=48)
    with pytest.raises(G.GsError, match="lds_batch"):
        P.rasterize_fwd(frame, vd, lds_batch=-128)     # the per-tile batch is the backward's
    with pytest.raises(G.GsError, match="lds_batch"):
        P.rasterize_bwd(frame, vd, dLdC=frame.image, lds_batch=-32)
    with pytest.raises(G.GsError, match="exactly one"):
        P.rasterize_bwd(frame, vd, target=None, dLdC=None)


# ---------------------------------------------------------------------------
# exact tile culling (opacity-threshold ellipse)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(WL))
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_ellipse_culling_tiles_rows_and_keys_bit_exact(name, tile):
    scene, target_scene, views, _ = WL[name]
    note(f"exact culling binning parity {name} tile {tile}")
    pr = oracle.project(scene, views, tile, cull=oracle.CULL_ELLIPSE)
    bins = oracle.bin_sort(pr, views, tile)
    g = run_gpu_step(scene, views, tile, cull=1)
    assert g["status"] == 0
    np.testing.assert_array_equal(g["tiles"], pr.tiles)
    vis = pr.tiles > 0
    np.testing.assert_array_equal(rect_from_packed(g["rect"])[vis], pr.rect[vis])
    np.testing.assert_array_equal(g["offsets"], bins.offsets)
    np.testing.assert_array_equal(g["keys"], bins.keys)
    np.testing.assert_array_equal(g["vals"], bins.gid[bins.vals])
    np.testing.assert_array_equal(g["ranges"], bins.ranges)
    # row slots: one per bounding-box row, first index of each row, spans that
    # reproduce the unsorted keys
    V, n = pr.tiles.shape
    h = np.where(vis, pr.rect[..., 3] - pr.rect[..., 1], 0).reshape(-1)
    np.testing.assert_array_equal(g["row_offsets"], np.concatenate([[0], np.cumsum(h)]).astype(np.uint32))
    rows = g["rows"].astype(np.int64)
    o = rows[:, 1]
    xa, ty = rows[:, 2] & 0xFFFF, rows[:, 2] >> 16
    ends = np.append(rows[1:, 0], int(bins.offsets[-1]))
    count = ends - rows[:, 0]
    assert np.all(count >= 0)
    np.testing.assert_array_equal(rows[:, 0][np.searchsorted(o, np.flatnonzero(vis.reshape(-1)))],
                                  bins.offsets[:-1][vis.reshape(-1)])
    gx = np.array([(int(v["width"]) + tile - 1) // tile for v in views])
    vw = o // n
    for r in range(0, len(rows), max(1, len(rows) // 2000)):
        t = ty[r] * gx[vw[r]] + np.arange(xa[r], xa[r] + count[r])
        D = oracle.depth_bits(int(gx[vw[r]]) * ((int(views[vw[r]]["height"]) + tile - 1) // tile))
        k = bins.keys_unsorted[rows[r, 0]:rows[r, 0] + len(t)].astype(np.int64)
        np.testing.assert_array_equal(k >> D, t)
        assert np.all(k & ((1 << D) - 1) == rows[r, 3])      # the row carries the depth bits


@pytest.mark.parametrize("name", list(WL))
def test_ellipse_culling_training_step(name):
    scene, target_scene, views, tile = WL[name]
    note(f"exact culling training-step parity {name}")
    target = oracle.render(target_scene, views, tile, cull=oracle.CULL_ELLIPSE)
    ref = oracle.train_step(scene, views, tile, target, cull=oracle.CULL_ELLIPSE)
    g = run_gpu_step(scene, views, tile, target=target, cull=1)
    V, n = len(views), scene.n
    ok = ref.image.fragile == 0
    assert ok.mean() > 0.995
    assert np.abs(g["image"] - ref.image.rgb).max(axis=1)[ok].max() <= PIX_TOL
    np.testing.assert_array_equal(g["last"][ok], ref.image.last[ok])
    ex = exempt_gaussians(ref.proj, ref.bins, views, tile, ref.fragile)
    ex_any = ex.any(axis=0)
    checked_fraction(ex_any, np.abs(ref.grads).max(axis=1) > 0, L1_CHECKED_FLOOR[name])
    # the gather's per-(view, Gaussian) sums against the oracle's
    oks = grad_close(g["sums"].reshape(-1, 9), ref.grads2d.reshape(-1, 9), GRAD_RTOL).reshape(V, n, 9)
    assert not (~oks.all(axis=2) & ~ex).any()
    okg = grad_close(g["grads"], ref.grads, GRAD_RTOL)
    assert not (~okg.all(axis=1) & ~ex_any).any()
    # fewer intersections than the 3-sigma rectangle on the same scene
    assert g["K"] < oracle.bin_sort(oracle.project(scene, views, tile), views, tile).keys.size
    # every Gaussian, with the oracle's image gradient zeroed at fragile pixels
    dLdC = masked_image_gradient(ref.dLdC, ref.fragile)
    ref2 = oracle.train_step(scene, views, tile, None, cull=oracle.CULL_ELLIPSE, dLdC=dLdC)
    g2 = run_gpu_step(scene, views, tile, dLdC=dLdC, cull=1)
    g2["p0"] = scene.flat()
    assert _check_step(g2, ref2, views, tile, n, np.zeros((V, n), bool), 1.0) == 1.0


def test_plain_step_graph_replays_match_eager_steps():
    """A training step captured in a HIP graph, replayed three times with eager
    work between the replays, gives the eager steps' parameters bit for bit
    after every replay."""
    import torch
    from paper_2605_00219_amd import pipeline as P
    scene, target_scene, views, tile = WL["plain-2k-256"]
    note("graph-replayed plain steps")
    target = torch.as_tensor(np.ascontiguousarray(oracle.render(target_scene, views, tile), np.float32),
                             device="cuda").reshape(-1, 3)
    vd = P.views_to_device(views)

    def setup():
        model = P.Model(scene.flat())
        frame = P.Frame(scene.n, [int(v["width"]) for v in views], [int(v["height"]) for v in views], tile)
        P.fit_capacity(model.params, frame, vd)
        frame.resize(frame.capacity * 2)
        return model, frame

    def step(model, frame):
        P.project(model.params, frame, vd)
        P.bin_sort(frame)
        P.rasterize_fwd(frame, vd, 128)
        P.rasterize_bwd(frame, vd, target=target, lds_batch=128)
        P.project_bwd_adam(model, frame, vd)

    me, fe = setup()
    eager = []
    for _ in range(3):
        step(me, fe)
        torch.cuda.synchronize()
        eager.append(me.params.cpu().numpy())
    mg, fg = setup()
    saved = [t.clone() for t in (mg.params, mg.m, mg.v, mg.step)]
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        step(mg, fg)
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(mg, fg)
    torch.cuda.synchronize()
    for t, s0 in zip((mg.params, mg.m, mg.v, mg.step), saved):
        t.copy_(s0)
    for i in range(3):
        g.replay()
        torch.cuda.synchronize()
        junk = torch.ones(1 << 20, device="cuda").sum()      # eager work between replays
        assert float(junk.item()) == float(1 << 20)
        assert fg.status_bits() == 0
        np.testing.assert_array_equal(mg.params.cpu().numpy(), eager[i], err_msg=f"replay {i}")
