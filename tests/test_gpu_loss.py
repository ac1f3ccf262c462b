"""Fused L1 + D-SSIM loss gradient (gs_loss_l1_ssim) against the oracle
(oracle/ssim.py): two ragged views whole, and the 1280x720 bench resolution
on padded crops.  Bar: gradients within 1e-3 relative (floored at 1e-2 of the
maximum), pixels whose L1 sign is a near-tie (fragile) excluded; loss sums
within 1e-5 relative."""
import numpy as np
import pytest

import synthetic as S
from gpu_common import note
from helpers import grad_close
from oracle import ssim as O

pytestmark = pytest.mark.gpu


def _frame(sizes):
    from paper_2605_00219_amd import pipeline as P
    return P.Frame(16, [w for w, _ in sizes], [h for _, h in sizes], 16, capacity=1024)


def _inputs(sizes, seed):
    rng = np.random.default_rng(seed)
    P = sum(w * h for w, h in sizes)
    x = rng.uniform(0.0, 1.0, size=(P, 3)).astype(np.float32)
    t = rng.integers(0, 256, size=(P, 4)).astype(np.uint8)
    # smooth structure as well as noise, and some fully masked pixels
    base = 0
    for w, h in sizes:
        yy, xx = np.mgrid[0:h, 0:w]
        wave = (0.5 + 0.4 * np.sin(xx / 7.0) * np.cos(yy / 5.0)).reshape(-1)
        x[base:base + w * h, 1] = wave.astype(np.float32)
        t[base:base + w * h, 1] = np.clip(wave * 255 + rng.normal(0, 10, w * h), 0, 255).astype(np.uint8)
        base += w * h
    t[rng.random(P) < 0.05, 3] = 0
    return x, t


def _run(frame, x, t, lam, mask):
    import torch
    from paper_2605_00219_amd import pipeline as P
    frame.image.copy_(torch.as_tensor(x, device="cuda"))
    loss = P.LossL1SSIM(frame, lam=lam, use_mask=mask)
    g = loss(torch.as_tensor(t, device="cuda").contiguous())
    torch.cuda.synchronize()
    return g.cpu().numpy(), loss.blocks.cpu().numpy().reshape(-1, 2), loss.loss()


@pytest.mark.parametrize("lam,mask", [(0.2, True), (0.2, False), (0.0, True), (1.0, True)])
def test_loss_gradient_two_ragged_views(lam, mask):
    sizes = [(200, 150), (333, 97)]
    note(f"L1 + D-SSIM loss gradient, lam={lam}, mask={mask}")
    x, t = _inputs(sizes, 11)
    g, blocks, loss = _run(_frame(sizes), x, t, lam, mask)
    ref_loss, ref, parts, fragile = O.loss_and_grad(x, t, sizes, lam=lam, mask=mask)
    ok = fragile == 0
    assert ok.mean() > 0.99
    close = grad_close(g[ok], ref[ok], 1e-3)
    assert close.all(), np.argwhere(~close)[:5]
    assert loss == pytest.approx(ref_loss, rel=1e-5)
    # per-view sums of the (64 x 16 block, channel) units
    nu = [3 * ((w + 63) // 64) * ((h + 15) // 16) for w, h in sizes]
    assert blocks.shape[0] == nu[0] + nu[1]
    b0 = blocks[:nu[0]].astype(np.float64).sum(0)
    b1 = blocks[nu[0]:nu[0] + nu[1]].astype(np.float64).sum(0)
    np.testing.assert_allclose(b0, parts[0], rtol=1e-5)
    np.testing.assert_allclose(b1, parts[1], rtol=1e-5)


def test_loss_gradient_small_views():
    """Views smaller than one 64 x 16 block, and one block wider than a view."""
    sizes = [(40, 9), (7, 30), (130, 17)]
    note("L1 + D-SSIM loss gradient on views smaller than a block")
    x, t = _inputs(sizes, 12)
    g, blocks, loss = _run(_frame(sizes), x, t, 0.2, True)
    ref_loss, ref, parts, fragile = O.loss_and_grad(x, t, sizes, lam=0.2, mask=True)
    ok = fragile == 0
    close = grad_close(g[ok], ref[ok], 1e-3)
    assert close.all(), np.argwhere(~close)[:5]
    assert loss == pytest.approx(ref_loss, rel=1e-5)
    assert blocks.shape[0] == 3 * (1 + 2 + 3 * 2)


def test_loss_gradient_1280x720_on_padded_crops():
    W, H = 1280, 720
    note("L1 + D-SSIM loss gradient at 1280x720, 12 crops")
    x = np.clip(np.random.default_rng(21).normal(0.5, 0.25, size=(W * H, 3)), 0, 1).astype(np.float32)
    t = (S.random_image(H, W, 22).reshape(-1, 3) * 255).astype(np.uint8)
    t = np.concatenate([t, np.full((W * H, 1), 255, np.uint8)], axis=1)
    t[np.random.default_rng(23).random(W * H) < 0.1, 3] = 128
    g, blocks, _ = _run(_frame([(W, H)]), x, t, 0.2, True)
    rng = np.random.default_rng(24)
    xi, ti, gi = x.reshape(H, W, 3), t.reshape(H, W, 4), g.reshape(H, W, 3)
    bw = (W + 63) // 64
    for c in range(12):
        # a 64 x 64 region on the 64 x 16 block grid (corners included), margin 10
        if c < 4:
            bx, by = [(0, 0), (W // 64 - 1, 0), (0, H // 16 - 4), (W // 64 - 1, H // 16 - 4)][c]
        else:
            bx, by = int(rng.integers(0, W // 64)), int(rng.integers(0, H // 16 - 3))
        x0, y0 = 64 * bx, 16 * by
        cx0, cy0 = max(0, x0 - 10), max(0, y0 - 10)
        cx1, cy1 = min(W, x0 + 64 + 10), min(H, y0 + 64 + 10)
        cw, ch = cx1 - cx0, cy1 - cy0
        xc = xi[cy0:cy1, cx0:cx1].reshape(-1, 3)
        tc = ti[cy0:cy1, cx0:cx1].reshape(-1, 4)
        _, rc, _, fr = O.loss_and_grad(xc, tc, [(cw, ch)], lam=0.2, mask=True)
        rc = rc.reshape(ch, cw, 3) * (cw * ch) / (W * H)     # the crop's own 1/(3P)
        fr = fr.reshape(ch, cw)
        sl = (slice(y0 - cy0, y0 - cy0 + 64), slice(x0 - cx0, x0 - cx0 + 64))
        got, want, ok = gi[y0:y0 + 64, x0:x0 + 64], rc[sl], fr[sl] == 0
        close = grad_close(got[ok], want[ok], 1e-3)
        assert close.all(), (c, np.argwhere(~close)[:5])
        # sums of the region's 4 blocks (3 channel units each)
        s, _, _, _ = O.ssim_terms(xc.reshape(ch, cw, 3)[..., 0].astype(np.float64),
                                   tc.reshape(ch, cw, 4)[..., 0].astype(np.float64) / 255.0)
        for k in range(1, 3):
            s = s + O.ssim_terms(xc.reshape(ch, cw, 3)[..., k].astype(np.float64),
                                 tc.reshape(ch, cw, 4)[..., k].astype(np.float64) / 255.0)[0]
        m = tc.reshape(ch, cw, 4)[..., 3].astype(np.float64) / 255.0
        one_minus = (3.0 - s) * m
        for j in range(4):
            blk = (by + j) * bw + bx
            yy, xx = y0 - cy0 + 16 * j, x0 - cx0
            want_s = one_minus[yy:yy + 16, xx:xx + 64].sum()
            got_s = blocks[3 * blk:3 * blk + 3, 1].astype(np.float64).sum()
            assert got_s == pytest.approx(want_s, rel=1e-5, abs=1e-4)


def test_loss_gradient_multiview_full_resolutions_on_crops():
    """Three views of uneven full resolutions in one call (block bases, padded
    workspace views and pixel bases at scale): padded crops of each view
    against the oracle, and the per-view sums against the oracle's L1 sums."""
    sizes = [(800, 600), (1920, 1080), (640, 480)]
    note("L1 + D-SSIM loss gradient, 3 views up to 1920x1080, crops")
    P_tot = sum(w * h for w, h in sizes)
    rng = np.random.default_rng(31)
    x = np.clip(rng.normal(0.5, 0.25, size=(P_tot, 3)), 0, 1).astype(np.float32)
    t = rng.integers(0, 256, size=(P_tot, 4)).astype(np.uint8)
    t[rng.random(P_tot) < 0.5, 3] = 255
    g, blocks, loss = _run(_frame(sizes), x, t, 0.2, True)
    base = np.cumsum([0] + [w * h for w, h in sizes])
    nu = [3 * ((w + 63) // 64) * ((h + 15) // 16) for w, h in sizes]
    ub = np.cumsum([0] + nu)
    for v, (W, H) in enumerate(sizes):
        xi = x[base[v]:base[v + 1]].reshape(H, W, 3)
        ti = t[base[v]:base[v + 1]].reshape(H, W, 4)
        gi = g[base[v]:base[v + 1]].reshape(H, W, 3)
        # per-view L1 sum: m |x - y| over the view, against float64
        m = ti[..., 3].astype(np.float64) / 255.0
        l1 = (m[..., None] * np.abs(xi.astype(np.float64) - ti[..., :3].astype(np.float64) / 255.0)).sum()
        assert blocks[ub[v]:ub[v + 1], 0].astype(np.float64).sum() == pytest.approx(l1, rel=1e-5)
        for c in range(3):
            x0 = int(rng.integers(0, W - 48)) if c else W - 48      # one crop at the right edge
            y0 = int(rng.integers(0, H - 40)) if c else H - 40      # and the bottom edge
            cx0, cy0 = max(0, x0 - 10), max(0, y0 - 10)
            cx1, cy1 = min(W, x0 + 48 + 10), min(H, y0 + 40 + 10)
            cw, ch = cx1 - cx0, cy1 - cy0
            xc = xi[cy0:cy1, cx0:cx1].reshape(-1, 3)
            tc = ti[cy0:cy1, cx0:cx1].reshape(-1, 4)
            _, rc, _, fr = O.loss_and_grad(xc, tc, [(cw, ch)], lam=0.2, mask=True)
            rc = rc.reshape(ch, cw, 3) * (cw * ch) / P_tot
            fr = fr.reshape(ch, cw)
            sl = (slice(y0 - cy0, y0 - cy0 + 40), slice(x0 - cx0, x0 - cx0 + 48))
            got, want, ok = gi[y0:y0 + 40, x0:x0 + 48], rc[sl], fr[sl] == 0
            close = grad_close(got[ok], want[ok], 1e-3)
            assert close.all(), (v, c, np.argwhere(~close)[:5])
