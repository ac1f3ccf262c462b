"""Oracle (test infrastructure only: imported by tests/ and the bench's CPU
baseline, never by the product path): the fused L1 + D-SSIM loss of a
rendered image against an RGBA8 reference with an alpha mask, and its
gradient with respect to the render (Sec. 4.5: the weighted sum of the L1 and
SSIM losses, the reference kept as 4 x UINT8 RGBA, alpha masking fused).

The paper names neither the window nor the weight; the readings are those of
the 3DGS training loss it replaces:

  L = (1 - lam) / (3P) sum_p m_p sum_k |x_pk - y_pk|
    + lam / (3P) sum_p m_p sum_k (1 - S_pk),            lam = 0.2,

over the P pixels of all views, x the render, y = rgb / 255 and m = a / 255
the reference's colour and alpha (m = 1 without masking).  S is the SSIM map
of each colour channel of each view: an 11 x 11 Gaussian window with
sigma = 1.5 (normalised), zero outside the image ("same" correlation with
zero fill), mu = G * x, sigma_x^2 = G * x^2 - mu_x^2, sigma_xy = G * (xy) -
mu_x mu_y, C1 = 0.01^2, C2 = 0.03^2,
  S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2)).

The gradient follows from mu_x, E[x^2], E[xy] being window sums of x: with
a = m dS/dmu_x, b = m dS/dE[x^2], c = m dS/dE[xy] (per pixel),
  d(sum_p m_p S_p)/dx_q = (G * a)_q + 2 x_q (G * b)_q + y_q (G * c)_q.
Everything is float64 numpy; the window sums are scipy's 2-D correlation.
"""
import numpy as np
from scipy.signal import correlate2d

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA = 0.2
SIGN_MARGIN = 1e-5


def gaussian_window() -> np.ndarray:
    i = np.arange(WINDOW, dtype=np.float64) - WINDOW // 2
    g = np.exp(-(i * i) / (2.0 * SIGMA * SIGMA))
    g /= g.sum()
    return np.outer(g, g)


def blur(img: np.ndarray) -> np.ndarray:
    """Window sum at every pixel, zero outside the image."""
    return correlate2d(img, gaussian_window(), mode="same", boundary="fill", fillvalue=0.0)


def ssim_terms(x: np.ndarray, y: np.ndarray):
    """SSIM map of one channel and its partial derivatives with respect to
    mu_x, E[x^2] and E[xy] (at fixed y statistics)."""
    mx, my = blur(x), blur(y)
    exx, eyy, exy = blur(x * x), blur(y * y), blur(x * y)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    a1, a2 = 2.0 * mx * my + C1, 2.0 * sxy + C2
    b1, b2 = mx * mx + my * my + C1, sxx + syy + C2
    s = a1 * a2 / (b1 * b2)
    # sigma_x^2 and sigma_xy also depend on mu_x
    ds_dmx = 2.0 * my * (a2 - a1) / (b1 * b2) - 2.0 * mx * s / b1 + 2.0 * mx * s / b2
    ds_dexx = -s / b2
    ds_dexy = 2.0 * a1 / (b1 * b2)
    return s, ds_dmx, ds_dexx, ds_dexy


def decode(rgba: np.ndarray, mask: bool):
    """Colour and mask weight of an RGBA8 reference [..., 4]."""
    rgba = np.asarray(rgba, np.uint8)
    y = rgba[..., :3].astype(np.float64) / 255.0
    m = rgba[..., 3].astype(np.float64) / 255.0 if mask else np.ones(rgba.shape[:-1])
    return y, m


def loss_and_grad(render: np.ndarray, target_rgba: np.ndarray, sizes, lam: float = LAMBDA,
                  mask: bool = True):
    """render [P, 3] (views concatenated, row-major per view), target_rgba
    [P, 4] uint8, sizes [(W, H), ...].  Returns (loss, dL/drender [P, 3],
    per-view (L1 sum, SSIM-loss sum), fragile [P] uint8 marking pixels whose
    L1 sign is a near-tie)."""
    x_all = np.asarray(render, np.float64).reshape(-1, 3)
    y_all, m_all = decode(np.asarray(target_rgba).reshape(-1, 4), mask)
    P = x_all.shape[0]
    inv = 1.0 / (3.0 * P)
    grad = np.zeros_like(x_all)
    fragile = np.zeros(P, np.uint8)
    parts = []
    base = 0
    for (W, H) in sizes:
        sl = slice(base, base + W * H)
        x = x_all[sl].reshape(H, W, 3)
        y = y_all[sl].reshape(H, W, 3)
        m = m_all[sl].reshape(H, W)
        l1_sum = 0.0
        ls_sum = 0.0
        g = np.zeros((H, W, 3))
        for k in range(3):
            s, a, b, c = ssim_terms(x[..., k], y[..., k])
            d = x[..., k] - y[..., k]
            l1_sum += float((m * np.abs(d)).sum())
            ls_sum += float((m * (1.0 - s)).sum())
            g_l1 = (1.0 - lam) * inv * m * np.sign(d)
            g_s = -lam * inv * (blur(m * a) + 2.0 * x[..., k] * blur(m * b) + y[..., k] * blur(m * c))
            g[..., k] = g_l1 + g_s
            mag = np.maximum(np.abs(x[..., k]), np.abs(y[..., k]))
            near = (mag > 0) & (np.abs(d) <= SIGN_MARGIN * mag) & (m > 0)
            fragile[sl] |= near.reshape(-1).astype(np.uint8)
        grad[sl] = g.reshape(-1, 3)
        parts.append((l1_sum, ls_sum))
        base += W * H
    loss = (1.0 - lam) * inv * sum(p[0] for p in parts) + lam * inv * sum(p[1] for p in parts)
    return loss, grad, parts, fragile
