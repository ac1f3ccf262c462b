"""Pins of the L1 + D-SSIM loss oracle (oracle/ssim.py) against facts that do
not come from its own formulas: SSIM of an image with itself, the interior
closed form for constant images, brute-force window sums on a tiny image,
central differences of the loss, the L1 part against torch's l1_loss autograd,
and the mask's limits."""
import math

import numpy as np
import pytest

from oracle import ssim as O


def _rand(seed, W, H):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.05, 0.95, size=(W * H, 3))
    t = rng.integers(0, 256, size=(W * H, 4)).astype(np.uint8)
    return x, t


def test_window_is_normalised_gaussian():
    g = O.gaussian_window()
    assert g.shape == (11, 11)
    assert abs(g.sum() - 1.0) < 1e-14
    i = np.arange(11) - 5
    ref = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2 * 1.5 ** 2))
    np.testing.assert_allclose(g, ref / ref.sum(), rtol=1e-14)


def test_ssim_of_an_image_with_itself_is_one_and_stationary():
    rng = np.random.default_rng(1)
    W, H = 23, 17
    rgba = rng.integers(0, 256, size=(W * H, 4)).astype(np.uint8)
    rgba[:, 3] = 255
    x = rgba[:, :3].astype(np.float64) / 255.0
    loss, g, parts, _ = O.loss_and_grad(x, rgba, [(W, H)], lam=1.0)
    assert abs(parts[0][1]) < 1e-9          # sum of (1 - S)
    assert abs(loss) < 1e-12
    assert np.abs(g).max() < 1e-9           # S is at its maximum


def test_constant_images_interior_closed_form():
    W, H, a, b = 31, 29, 0.7, 0.3
    s, _, _, _ = O.ssim_terms(np.full((H, W), a), np.full((H, W), b))
    want = (2 * a * b + O.C1) / (a * a + b * b + O.C1)
    np.testing.assert_allclose(s[5:-5, 5:-5], want, rtol=1e-12)
    assert np.abs(s[0, 0] - want) > 1e-6   # zero padding shows at the border


def test_window_sums_brute_force_on_a_tiny_image():
    rng = np.random.default_rng(2)
    H, W = 7, 9
    x, y = rng.uniform(size=(H, W)), rng.uniform(size=(H, W))
    g = O.gaussian_window()

    def wsum(img, i, j):
        tot = 0.0
        for di in range(-5, 6):
            for dj in range(-5, 6):
                ii, jj = i + di, j + dj
                if 0 <= ii < H and 0 <= jj < W:
                    tot += g[di + 5, dj + 5] * img[ii, jj]
        return tot

    s, _, _, _ = O.ssim_terms(x, y)
    for i in range(H):
        for j in range(W):
            mx, my = wsum(x, i, j), wsum(y, i, j)
            vx = wsum(x * x, i, j) - mx * mx
            vy = wsum(y * y, i, j) - my * my
            cxy = wsum(x * y, i, j) - mx * my
            ref = ((2 * mx * my + O.C1) * (2 * cxy + O.C2)) / ((mx * mx + my * my + O.C1) * (vx + vy + O.C2))
            assert abs(s[i, j] - ref) < 1e-12


@pytest.mark.parametrize("mask", [False, True])
def test_gradient_central_differences(mask):
    W, H = 16, 13
    x, t = _rand(3, W, H)
    # keep render and reference apart so no L1 kink lies within the step
    y = t[:, :3].astype(np.float64) / 255.0
    x = np.where(np.abs(x - y) < 0.02, y + 0.05, x)
    loss, g, _, _ = O.loss_and_grad(x, t, [(W, H)], lam=0.2, mask=mask)
    rng = np.random.default_rng(4)
    h = 1e-6
    for _ in range(40):
        p, k = int(rng.integers(W * H)), int(rng.integers(3))
        xp, xm = x.copy(), x.copy()
        xp[p, k] += h
        xm[p, k] -= h
        fd = (O.loss_and_grad(xp, t, [(W, H)], mask=mask)[0] - O.loss_and_grad(xm, t, [(W, H)], mask=mask)[0]) / (2 * h)
        assert abs(fd - g[p, k]) <= 1e-6 * abs(g).max() + 1e-4 * abs(fd), (p, k, fd, g[p, k])


def test_l1_part_matches_torch_l1_loss():
    import torch
    W, H = 12, 10
    x, t = _rand(5, W, H)
    t[:, 3] = 255
    loss, g, _, _ = O.loss_and_grad(x, t, [(W, H)], lam=0.0, mask=True)
    xt = torch.tensor(x, requires_grad=True)
    ref = torch.nn.functional.l1_loss(xt, torch.tensor(t[:, :3] / 255.0))
    ref.backward()
    assert abs(loss - float(ref.detach())) < 1e-12
    np.testing.assert_allclose(g, xt.grad.numpy(), atol=1e-15)


def test_mask_zero_gives_nothing_and_views_are_separate():
    W, H = 10, 8
    x, t = _rand(6, W, H)
    t0 = t.copy()
    t0[:, 3] = 0
    loss, g, _, _ = O.loss_and_grad(x, t0, [(W, H)])
    assert loss == 0.0 and np.all(g == 0.0)
    # two views: each one's SSIM windows stay inside it
    x2, t2 = _rand(7, 6, 5)
    both = O.loss_and_grad(np.concatenate([x, x2]), np.concatenate([t, t2]), [(W, H), (6, 5)])
    a = O.loss_and_grad(x, t, [(W, H)])
    b = O.loss_and_grad(x2, t2, [(6, 5)])
    assert both[2][0] == pytest.approx(a[2][0]) and both[2][1] == pytest.approx(b[2][0])
    P = W * H + 30
    np.testing.assert_allclose(both[1][:W * H], a[1] * (W * H) / P, rtol=1e-12)
