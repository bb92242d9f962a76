"""FP64 reference of one training step around the renderer (test
infrastructure only: tests, the smoke check and the benchmark's CPU baseline
use it; the library never does).

Photometric loss of Sec. 3.3, Eq. 9:  L = (1 - lam) L2 + lam D-SSIM,
lam = 0.2.  The paper states the loss "as in 3DGS" and leaves the terms'
definitions to it; the readings taken:
  - L2 is the mean squared error over every pixel and colour channel of every
    view (views packed, so a view weighs by its pixel count);
  - D-SSIM = 1 - SSIM, with SSIM the mean over the same pixel-channels of the
    structural-similarity map of Wang et al. (2004) with an 11x11 Gaussian
    window of standard deviation 1.5 (normalised to sum 1), C1 = 0.01^2,
    C2 = 0.03^2, evaluated per channel and per view with the window
    zero-padded at the view's borders.

The optimiser is not given either; the reading is Adam (Kingma and Ba 2015,
Algorithm 1) with bias correction, beta1 = 0.9, beta2 = 0.999, eps = 1e-15,
one learning rate per parameter tensor.
"""
from __future__ import annotations

import numpy as np

C1 = 0.01 ** 2
C2 = 0.03 ** 2
WINDOW = 11
WINDOW_SIGMA = 1.5
LAMBDA = 0.2


def gaussian_window(size=WINDOW, sigma=WINDOW_SIGMA):
    """1-D taps g[k] ~ exp(-(k - r)^2 / (2 sigma^2)), summing to 1; the 2-D
    window is their outer product."""
    r = size // 2
    x = np.arange(size, dtype=np.float64) - r
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    return g / g.sum()


def window_mean(img, g=None):
    """sum_{p'} w(p' - p) img(p') with the 2-D window w = g g^T, zero outside
    the image (same size as img [H, W]).  The window is separable, so the sum
    is taken as a horizontal then a vertical pass."""
    g = gaussian_window() if g is None else g
    H, W = img.shape
    r = len(g) // 2
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    h = sum(g[k] * pad[:, k:k + W] for k in range(len(g)))
    return sum(g[k] * h[k:k + H, :] for k in range(len(g)))


def ssim_terms(x, y):
    """Per-pixel SSIM map and its partial derivatives with respect to the
    window moments mu_x, E[x^2] and E[xy] (y fixed), for one channel [H, W]."""
    mx, my = window_mean(x), window_mean(y)
    exx, eyy, exy = window_mean(x * x), window_mean(y * y), window_mean(x * y)
    sxx, syy, sxy = exx - mx * mx, eyy - my * my, exy - mx * my
    A1, A2 = 2 * mx * my + C1, 2 * sxy + C2
    B1, B2 = mx * mx + my * my + C1, sxx + syy + C2
    S = A1 * A2 / (B1 * B2)
    # S = A1 A2 / (B1 B2) with sigma_xy = E[xy] - mu_x mu_y, sigma_x^2 = E[x^2] - mu_x^2
    d_mx = S * (2 * my / A1 - 2 * my / A2 - 2 * mx / B1 + 2 * mx / B2)
    d_exx = -S / B2
    d_exy = 2 * S / A2
    return S, d_mx, d_exx, d_exy


def _views(images, wh):
    off = 0
    for W, H in wh:
        n = int(W) * int(H)
        yield off, int(W), int(H), images[off:off + n].reshape(int(H), int(W), 3)
        off += n


def loss(images, targets, wh, lam=LAMBDA):
    """Eq. 9 over packed HWC images [sum W H][3]; returns (L, L2, SSIM)."""
    images = np.asarray(images, np.float64)
    targets = np.asarray(targets, np.float64)
    n = images.size
    l2 = float(((images - targets) ** 2).sum() / n)
    ssum = 0.0
    for (off, W, H, x), (_, _, _, y) in zip(_views(images, wh), _views(targets, wh)):
        for c in range(3):
            ssum += ssim_terms(x[:, :, c], y[:, :, c])[0].sum()
    ssim = ssum / n
    return (1.0 - lam) * l2 + lam * (1.0 - ssim), l2, ssim


def loss_grad(images, targets, wh, lam=LAMBDA):
    """dL/dC for Eq. 9 (same layout as images).  The SSIM part chains the
    per-pixel derivatives through the window: dS(p)/dx(q) sums over the
    pixels p whose window holds q, which for the symmetric, zero-padded window
    is one more window pass over d_mx + 2 x(q) d_exx + y(q) d_exy."""
    images = np.asarray(images, np.float64)
    targets = np.asarray(targets, np.float64)
    n = images.size
    g = (1.0 - lam) * 2.0 * (images - targets) / n
    for (off, W, H, x), (_, _, _, y) in zip(_views(images, wh), _views(targets, wh)):
        gv = g[off:off + W * H].reshape(H, W, 3)
        for c in range(3):
            _, a, b, cc = ssim_terms(x[:, :, c], y[:, :, c])
            ds = window_mean(a) + 2 * x[:, :, c] * window_mean(b) + y[:, :, c] * window_mean(cc)
            gv[:, :, c] -= lam * ds / n
    return g


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam update (Kingma and Ba 2015, Algorithm 1) at 1-based step
    `step`; returns new (param, m, v)."""
    param, grad = np.asarray(param, np.float64), np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return param - lr * mhat / (np.sqrt(vhat) + eps), m, v
