"""The plain workload at its full size, in the configuration bench.py times:
300k Gaussians (means N(0,1), log-scales N(-4, 0.7)), one 1280x720 view,
16x16 tiles, 2 pixels per lane, S = 128, the fitted capacity (so the binning
takes its depth-first order and every sort pass runs in two rounds of
workgroups).  Projection, keys, values and ranges are compared bit for bit in
full; pixels and gradient records on a seeded sample of tiles, with the
oracle restricted to those tiles."""
import numpy as np
import pytest

import oracle
import synthetic as S
from gpu_common import note, run_gpu_step
from helpers import exempt_gaussians, grad_close

pytestmark = pytest.mark.gpu


def test_plain_300k_1280x720_full_size():
    w = S.workload_plain_300k()
    views = w.views[:1]
    scene = w.scene
    W, H = 1280, 720
    note("full size: 300k Gaussians, 1280x720, tile 16")
    target = S.random_image(H, W, 4242).reshape(-1, 3)
    g = run_gpu_step(scene, views, 16, target=target, lds_batch=128)
    assert g["status"] == 0
    pr = oracle.project(scene, views, 16)
    bins = oracle.bin_sort(pr, views, 16)
    K = int(bins.offsets[-1])
    assert K > 4_000_000
    assert g["frame"].capacity >= 12 * scene.n          # depth-first order
    np.testing.assert_array_equal(g["tiles"], pr.tiles)
    np.testing.assert_array_equal(g["offsets"], bins.offsets)
    np.testing.assert_array_equal(g["keys"], bins.keys)
    np.testing.assert_array_equal(g["vals"], bins.gid[bins.vals])
    np.testing.assert_array_equal(g["ranges"], bins.ranges)
    # a sample of tiles: pixels, last, T, then the backward's records
    gx, gy = (W + 15) // 16, (H + 15) // 16
    rng = np.random.default_rng(7)
    sample = rng.choice(gx * gy, size=48, replace=False)
    tmask = np.zeros(gx * gy, np.uint8)
    tmask[sample] = 1
    fwd = oracle.raster_fwd(pr, bins, views, 16, tile_mask=tmask)
    pix_tile = (np.arange(W * H) // W // 16) * gx + (np.arange(W * H) % W) // 16
    inside = tmask[pix_tile].astype(bool)
    _, dLdC = oracle.l1(fwd.rgb, target, fragile=fwd.fragile, last=fwd.last)
    ok = inside & (fwd.fragile == 0)
    assert ok.sum() > 0.9 * inside.sum()
    err = np.abs(g["image"] - fwd.rgb).max(axis=1)
    assert err[ok].max() <= 1e-4, err[ok].max()
    np.testing.assert_array_equal(g["last"][ok], fwd.last[ok])
    assert np.abs(g["T"] - fwd.T)[ok].max() <= 1e-4
    partials, _ = oracle.raster_bwd(pr, bins, views, 16, dLdC, tile_mask=tmask)
    ex = exempt_gaussians(pr, bins, views, 16, fwd.fragile & inside)[0]
    bit = lambda m, i: (m[i >> 5] >> (i & 31)) & 1
    kept, quiet = [], []
    for t in sample:
        s, stop = int(g["ranges"][t, 0]), int(g["tile_stop"][t])
        pos = np.arange(s, stop)
        idx = bins.vals[pos].astype(np.int64)
        flag = bit(g["rec_mask"], idx).astype(bool)
        np.testing.assert_array_equal(flag, bit(g["comp_mask"], pos).astype(bool))
        free = ~ex[bins.gid[idx]]
        kept.append(idx[flag & free])
        quiet.append(idx[~flag & free])
    kept, quiet = np.concatenate(kept), np.concatenate(quiet)
    checked = kept.size
    okr = grad_close(g["grec"][kept, :9], partials[kept], 1e-3).all(axis=1)
    assert okr.all(), kept[~okr][:5]
    # entries traversed without a record carry no oracle gradient
    assert not (np.abs(partials[quiet]).max(axis=1) > 0).any()
    note(f"  K = {K}, {checked} records checked on {len(sample)} tiles")
    assert checked > 1000


def test_batched_3m_8_views_binning_full_size():
    """The batched workload's first step at full size: 3M Gaussians, 8 views
    of uneven resolution in one frame, 32x32 tiles (the autotuner's choice),
    fitted capacity (few intersections per (view, Gaussian): the direct
    32-bit sort over 8 view segments).  Projection, keys, values and ranges
    bit for bit."""
    import torch
    from paper_2605_00219_amd import pipeline as P
    w = S.workload_batched()
    cams, res = w.extra["cameras"], w.extra["resolutions"]
    views = S.batched_views(cams, res, 0)
    tile = 32
    note("full size: 3M Gaussians, 8 views, tile 32, binning")
    frame = P.Frame(w.scene.n, [wd for wd, _ in res], [ht for _, ht in res], tile)
    vd = P.views_to_device(views)
    params = P.pack_flat(w.scene.flat())
    P.fit_capacity(params, frame, vd)
    P.project(params, frame, vd)
    P.bin_sort(frame)
    torch.cuda.synchronize()
    assert frame.status_bits() == 0
    m = len(views) * w.scene.n
    assert frame.capacity < 12 * m                      # direct order
    u32 = lambda t: t.cpu().numpy().view(np.uint32)
    pr = oracle.project(w.scene, views, tile)
    bins = oracle.bin_sort(pr, views, tile)
    K = int(bins.offsets[-1])
    np.testing.assert_array_equal(u32(frame.tiles).reshape(len(views), -1), pr.tiles)
    np.testing.assert_array_equal(u32(frame.offsets), bins.offsets)
    np.testing.assert_array_equal(u32(frame.keys)[:K], bins.keys)
    np.testing.assert_array_equal(u32(frame.vals)[:K], bins.gid[bins.vals])
    np.testing.assert_array_equal(u32(frame.ranges), bins.ranges)
    note(f"  K = {K} over {len(views)} views")


def test_twophase_backward_full_size_against_first_backward():
    """The second (two-phase) backward at the full plain size, on the frame the
    bench times: the same flagged records, tile stops and owners as the first
    backward (itself checked against the oracle above), and every record equal
    to the first's up to float summation order."""
    import torch
    from paper_2605_00219_amd import pipeline as P
    w = S.workload_plain_300k()
    views = w.views[:1]
    W, H = 1280, 720
    note("full size: two-phase backward against the first, 300k, 1280x720")
    target = torch.as_tensor(S.random_image(H, W, 4243).reshape(-1, 3), device="cuda").contiguous()
    model = P.Model(w.scene.flat())
    frame = P.Frame(w.scene.n, [W], [H], 16)
    vd = P.views_to_device(views)
    P.fit_capacity(model.params, frame, vd)
    P.project(model.params, frame, vd)
    P.bin_sort(frame)
    P.rasterize_fwd(frame, vd, 128)
    out = []
    for variant in (128, ("twophase", 32)):
        P.backward(frame, vd, variant, target=target)
        torch.cuda.synchronize()
        K = frame.intersections()
        out.append(dict(rec_mask=frame.rec_mask.cpu().numpy().view(np.uint32).copy(),
                        stop=frame.tile_stop.cpu().numpy().copy(),
                        grec=frame.grec[:K].cpu().numpy().copy(), K=K))
    assert frame.status_bits() == 0
    a, b = out
    np.testing.assert_array_equal(a["rec_mask"], b["rec_mask"])
    np.testing.assert_array_equal(a["stop"], b["stop"])
    flagged = np.unpackbits(a["rec_mask"].view(np.uint8), bitorder="little")[:a["K"]].astype(bool)
    assert flagged.sum() > 100_000
    ra, rb = a["grec"][flagged], b["grec"][flagged]
    np.testing.assert_array_equal(ra[:, 9].view(np.uint32), rb[:, 9].view(np.uint32))
    scale = np.abs(ra[:, :9]).max(axis=0, keepdims=True) + 1e-30
    diff = np.abs(ra[:, :9] - rb[:, :9])
    assert (diff <= 1e-4 * scale + 1e-5 * np.abs(ra[:, :9])).all(), diff.max(axis=0) / scale
