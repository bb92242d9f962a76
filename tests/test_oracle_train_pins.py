"""Pins of the training-step oracle (loss of Sec. 3.3 Eq. 9, Adam) against
facts that do not come from the oracle itself: brute-force sums, the closed
forms of SSIM and Adam, and finite differences."""
import math

import numpy as np
import pytest

from oracle import train as T


def test_window_taps():
    """Gaussian window of 11 taps, sigma 1.5, summing to 1: symmetric, peaked
    at the centre, neighbouring taps in the ratio exp(-(2k+1) / (2 sigma^2))."""
    g = T.gaussian_window()
    assert g.shape == (11,) and abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1], rtol=0, atol=0)
    for k in range(5):
        assert math.isclose(g[5 + k + 1] / g[5 + k], math.exp(-(2 * k + 1) / (2 * 1.5 ** 2)), rel_tol=1e-13)


def test_window_mean_brute_force():
    """The separable pass equals the 2-D window sum over in-image pixels."""
    rng = np.random.default_rng(0)
    img = rng.random((9, 13))
    g = T.gaussian_window()
    w = np.outer(g, g)
    got = T.window_mean(img)
    for y in range(9):
        for x in range(13):
            s = 0.0
            for dy in range(-5, 6):
                for dx in range(-5, 6):
                    if 0 <= y + dy < 9 and 0 <= x + dx < 13:
                        s += w[dy + 5, dx + 5] * img[y + dy, x + dx]
            assert abs(got[y, x] - s) < 1e-14


def test_ssim_against_wang_definition():
    """SSIM map against Wang et al.'s form with centred second moments
    sigma_xy = sum w (x - mu_x)(y - mu_y), taken by explicit loops at
    interior and border pixels."""
    rng = np.random.default_rng(1)
    x, y = rng.random((14, 12)), rng.random((14, 12))
    S = T.ssim_terms(x, y)[0]
    g = T.gaussian_window()
    w = np.outer(g, g)
    for (py, px) in [(7, 6), (0, 0), (13, 5), (3, 11)]:
        ws, xs, ys = [], [], []
        for dy in range(-5, 6):
            for dx in range(-5, 6):
                yy, xx = py + dy, px + dx
                ws.append(w[dy + 5, dx + 5])
                inside = 0 <= yy < 14 and 0 <= xx < 12
                xs.append(x[yy, xx] if inside else 0.0)   # zero padding
                ys.append(y[yy, xx] if inside else 0.0)
        ws, xs, ys = map(np.array, (ws, xs, ys))
        mx, my = (ws * xs).sum(), (ws * ys).sum()
        vx, vy = (ws * (xs - mx) ** 2).sum(), (ws * (ys - my) ** 2).sum()
        cxy = (ws * (xs - mx) * (ys - my)).sum()
        # the window weights sum to 1, so the centred and raw forms agree
        ref = (2 * mx * my + T.C1) * (2 * cxy + T.C2) / ((mx * mx + my * my + T.C1) * (vx + vy + T.C2))
        assert abs(S[py, px] - ref) < 1e-12


def test_ssim_identity_symmetry_and_constants():
    """SSIM(x, x) = 1; SSIM(x, y) = SSIM(y, x); for constant images a, b the
    interior map is (2ab + C1) / (a^2 + b^2 + C1)."""
    rng = np.random.default_rng(2)
    x, y = rng.random((16, 16)), rng.random((16, 16))
    assert np.allclose(T.ssim_terms(x, x)[0], 1.0, rtol=0, atol=1e-12)
    assert np.allclose(T.ssim_terms(x, y)[0], T.ssim_terms(y, x)[0], rtol=0, atol=1e-14)
    a, b = 0.3, 0.8
    S = T.ssim_terms(np.full((16, 16), a), np.full((16, 16), b))[0]
    assert abs(S[8, 8] - (2 * a * b + T.C1) / (a * a + b * b + T.C1)) < 1e-12
    assert abs(S[5:11, 5:11] - S[8, 8]).max() < 1e-12


def test_loss_closed_forms():
    """lam = 0: the mean squared error and its gradient 2 (x - y) / n; lam = 1
    and x = y: loss 0; the SSIM map is largest at x = y, so there the whole
    gradient vanishes."""
    rng = np.random.default_rng(3)
    wh = [(11, 9), (7, 13)]
    n = sum(w * h for w, h in wh)
    x, y = rng.random((n, 3)), rng.random((n, 3))
    L, l2, _ = T.loss(x, y, wh, lam=0.0)
    assert abs(L - ((x - y) ** 2).mean()) < 1e-15 and L == l2
    assert np.allclose(T.loss_grad(x, y, wh, lam=0.0), 2 * (x - y) / x.size, rtol=0, atol=1e-17)
    assert abs(T.loss(x, x, wh, lam=1.0)[0]) < 1e-12
    assert np.abs(T.loss_grad(x, x, wh)).max() < 1e-13


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_loss_gradient_matches_finite_differences(lam):
    """dL/dC against FP64 central differences, two views of different sizes
    (the window stops at each view's border)."""
    rng = np.random.default_rng(4)
    wh = [(11, 9), (7, 13)]
    n = sum(w * h for w, h in wh)
    x, y = rng.random((n, 3)), rng.random((n, 3))
    g = T.loss_grad(x, y, wh, lam)
    scale = np.abs(g).max()
    idx = list(rng.choice(x.size, 40, replace=False)) + [0, 98 * 3 + 2, x.size - 1]   # include view corners
    for fi in idx:
        i = np.unravel_index(fi, x.shape)
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        fd = (T.loss(xp, y, wh, lam)[0] - T.loss(xm, y, wh, lam)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * scale, (i, fd, g[i])


def test_adam_closed_forms():
    """Step 1: theta - lr g / (|g| + eps).  A constant gradient keeps the
    bias-corrected moments at g and g^2, so every step moves by the same
    lr g / (|g| + eps).  A zero gradient from zero moments moves nothing."""
    rng = np.random.default_rng(5)
    p, g = rng.normal(size=50), rng.normal(size=50)
    m, v = np.zeros(50), np.zeros(50)
    lr = 1e-3
    p1, m1, v1 = T.adam_step(p, g, m, v, 1, lr)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + 1e-15), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g, rtol=1e-15) and np.allclose(v1, 0.001 * g * g, rtol=1e-12)
    q, mq, vq = p.copy(), m.copy(), v.copy()
    for t in range(1, 8):
        q_new, mq, vq = T.adam_step(q, g, mq, vq, t, lr)
        assert np.allclose(q - q_new, lr * g / (np.abs(g) + 1e-15), rtol=1e-9, atol=0)
        q = q_new
    z, _, _ = T.adam_step(p, np.zeros(50), m, v, 1, lr)
    assert np.array_equal(z, p)
