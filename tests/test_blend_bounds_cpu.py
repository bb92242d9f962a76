"""The blend forward's row masks skip a 4x4 sub-block for a Gaussian whose
exponent at the sub-block's centre lies below kE (kappa + sqrt(lambda_max(Q))
rho)^2, widened by 1e-3 (relative and absolute); rho = 1.5 sqrt 2 is the
distance from the centre to the farthest pixel centre.  Skipping must never
drop a pixel whose own support test passes (Sec. 3.2: the Gaussian's support
is the ellipse d^T Q d <= kappa^2 of the projected covariance).  This checks
the bound in FP32, as the kernel evaluates both sides, on random projected
covariances (including very elongated ones) and means around the block."""
import numpy as np

KE = np.float32(-0.5 * 1.44269504088896341)
KAPPA2 = 2.0 * np.log(2.0 ** 15)


def _bound(qa, qb, qc, kappa):
    f = np.float32
    h = f(0.5) * (qa - qc)
    lmax = f(0.5) * (qa + qc) + np.sqrt(h * h + qb * qb)
    rad = (kappa + np.sqrt(np.maximum(lmax, f(0))) * f(2.1214)) * f(1.001) + f(1e-3)
    return KE * rad * rad


def _expo(ex, ey, ez, dx, dy):
    return dx * (ex * dx + ey * dy) + ez * dy * dy


def test_sub_block_bound_never_drops_a_live_pixel():
    rng = np.random.default_rng(7)
    n = 200_000
    f = np.float32
    # projected covariance R diag(s^2) R^T + 0.3 I, scales from 0.05 to 60 px
    s1 = np.exp(rng.uniform(np.log(0.05), np.log(60.0), n))
    s2 = s1 * np.exp(rng.uniform(np.log(1e-3), 0.0, n))
    th = rng.uniform(0, np.pi, n)
    c, s = np.cos(th), np.sin(th)
    sxx = c * c * s1 ** 2 + s * s * s2 ** 2 + 0.3
    syy = s * s * s1 ** 2 + c * c * s2 ** 2 + 0.3
    sxy = c * s * (s1 ** 2 - s2 ** 2)
    det = sxx * syy - sxy * sxy
    qa, qb, qc = (syy / det).astype(f), (-sxy / det).astype(f), (sxx / det).astype(f)
    # means around the 4x4 block whose pixel centres are 0..3 (block centre 1.5)
    reach = 1.5 + np.sqrt(KAPPA2 * np.maximum(sxx, syy))
    mx = (1.5 + rng.uniform(-1, 1, n) * reach).astype(f)
    my = (1.5 + rng.uniform(-1, 1, n) * reach).astype(f)
    ex, ey, ez = KE * qa, f(2) * KE * qb, KE * qc
    e_min = KE * f(KAPPA2)
    thr = _bound(qa, qb, qc, f(np.sqrt(KAPPA2)))
    e_c = _expo(ex, ey, ez, f(1.5) - mx, f(1.5) - my)
    skipped = e_c < thr
    live = np.zeros(n, bool)
    for py in range(4):
        for px in range(4):
            live |= _expo(ex, ey, ez, f(px) - mx, f(py) - my) >= e_min
    assert not (skipped & live).any()
    # the bound is useful: it skips a good share of the boxes it is tested on
    assert skipped.mean() > 0.2 and live.mean() > 0.2
