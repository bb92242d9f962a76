"""Pins of the oracle's attribute maps (Eq. 5's Theta at resolution 3) and
view-dependent SH colour, against facts that do not come from the oracle:
exactness on linear functions, the orthonormality and addition theorem of
real spherical harmonics, a closed-form colour, the reduction to
resolution 1, and finite differences of the whole chain."""
import math

import numpy as np
import pytest

from paper_2503_13961_amd import scenes as S
from tests import helpers as H


def test_theta_reproduces_linear_functions_and_nodes(orc):
    """Resolution 3: texels on the level-2 lattice, linear inside each lattice
    triangle: a linear f(u, v) sampled at the nodes is reproduced exactly
    everywhere, a texel is returned at its own node, the weights are a
    partition of unity; resolution 1 is the constant texel."""
    rng = np.random.default_rng(0)
    nodes = [(a / 2, b / 2) for a in range(3) for b in range(3 - a)]   # lattice order, a outer
    for _ in range(5):
        al, be, ga = rng.normal(size=3)
        tex = np.array([al + be * u + ga * v for u, v in nodes])
        for _ in range(50):
            u, v = rng.random(2)
            if u + v > 1:
                u, v = 1 - u, 1 - v
            ti, tw = orc.theta(3, u, v)
            assert len(ti) == 3 and abs(tw.sum() - 1) < 1e-15 and (tw >= -1e-15).all()
            assert abs((tw * tex[ti]).sum() - (al + be * u + ga * v)) < 1e-13
    for t, (u, v) in enumerate(nodes):
        ti, tw = orc.theta(3, u, v)
        assert abs(tw[list(ti).index(t)] - 1.0) < 1e-15
    ti, tw = orc.theta(1, 0.3, 0.4)
    assert list(ti) == [0] and tw[0] == 1.0


def test_theta_is_continuous_across_cell_edges(orc):
    """Arbitrary texel values: the interpolant agrees from both sides of the
    lattice lines u = 1/2, v = 1/2 and u + v = 1/2."""
    rng = np.random.default_rng(1)
    tex = rng.normal(size=6)
    eps = 1e-9

    def f(u, v):
        ti, tw = orc.theta(3, u, v)
        return (tw * tex[ti]).sum()
    for _ in range(30):
        t = rng.random() * 0.5
        for (u, v), (du, dv) in (((0.5, t), (1, 0)), ((t, 0.5), (0, 1)), ((t, 0.5 - t), (1, 1))):
            assert abs(f(u - eps * du, v - eps * dv) - f(u + eps * du, v + eps * dv)) < 1e-7


def _sphere_quadrature(n=8, m=16):
    x, w = np.polynomial.legendre.leggauss(n)
    phi = 2 * np.pi * np.arange(m) / m
    pts, wts = [], []
    for xi, wi in zip(x, w):
        r = math.sqrt(1 - xi * xi)
        for ph in phi:
            pts.append((r * math.cos(ph), r * math.sin(ph), xi))
            wts.append(wi * 2 * np.pi / m)
    return np.array(pts), np.array(wts)


def test_sh_orthonormal_and_addition_theorem(orc):
    """int Y_i Y_j = delta_ij over the sphere (Gauss-Legendre x uniform
    azimuth, exact for these degrees); sum_m Y_lm(a) Y_lm(b) =
    (2l + 1) / (4 pi) P_l(a . b); the gradients are those of the polynomials."""
    pts, wts = _sphere_quadrature()
    Y = np.array([orc.sh_basis(3, p)[0] for p in pts])      # [N][15]
    G = (Y * wts[:, None]).T @ Y
    assert np.allclose(G, np.eye(15), atol=1e-12)
    rng = np.random.default_rng(2)
    for _ in range(10):
        a, b = rng.normal(size=(2, 3))
        a, b = a / np.linalg.norm(a), b / np.linalg.norm(b)
        Ya, Yb = orc.sh_basis(3, a)[0], orc.sh_basis(3, b)[0]
        c = float(a @ b)
        for l, P in ((1, c), (2, 0.5 * (3 * c * c - 1)), (3, 0.5 * (5 * c ** 3 - 3 * c))):
            lo, hi = l * l - 1, (l + 1) ** 2 - 1
            assert abs((Ya[lo:hi] * Yb[lo:hi]).sum() - (2 * l + 1) / (4 * np.pi) * P) < 1e-13
        Yv, dY = orc.sh_basis(3, a)
        for c3 in range(3):
            e = np.zeros(3)
            e[c3] = 1e-6
            fd = (orc.sh_basis(3, a + e)[0] - orc.sh_basis(3, a - e)[0]) / 2e-6
            assert np.allclose(fd, dY[:, c3], atol=1e-8)


def test_sh_colour_closed_form(orc):
    """A flat patch across the optical axis of a camera at the origin looking
    down +z: the principal pixel's view direction is (0, 0, 1), where only
    Y_10 = sqrt(3 / (4 pi)) z of band 1 is non-zero, so the colour is the
    diffuse colour plus sqrt(3 / (4 pi)) times that coefficient."""
    W, Ht, f, z0 = 41, 41, 60.0, 4.0
    cam = H.axis_camera(W, Ht, f)
    c3 = [H.pixel_ray_point(cam, 5.0, 5.0, z0), H.pixel_ray_point(cam, 36.0, 8.0, z0),
          H.pixel_ray_point(cam, 20.0, 36.0, z0)]
    sc = H.flat_patch_scene(c3, degree=1, color=(0.2, 0.5, 0.9), log_scale=-4.0, opacity=0.7, sharpness=2.0)
    sc.sh_degree = 1
    sc.sh = np.zeros((3, 3, 1), np.float32)
    sc.sh[:, 1, 0] = (0.3, -0.2, 0.1)            # Y_10 coefficients
    fr = orc.Frame(sc, cam, W, Ht)
    rec = fr.records()
    G = orc.GR
    pix = 20 * W + 20
    Sx, Sy, Sz = rec[pix, G["SX"]], rec[pix, G["SY"]], rec[pix, G["SZ"]]
    # the pixel centre (20.5, 20.5) is the principal point of this camera
    C = -cam[:9].reshape(3, 3).astype(np.float64).T @ cam[9:12].astype(np.float64)
    d = np.array([Sx, Sy, Sz]) - C
    d /= np.linalg.norm(d)
    assert np.allclose(d, (0, 0, 1), atol=1e-9)
    c10 = math.sqrt(3 / (4 * math.pi))
    want = np.array([0.2, 0.5, 0.9], np.float32).astype(np.float64) + c10 * d[2] * sc.sh[:, 1, 0].astype(np.float64)
    assert np.allclose(rec[pix, [G["CR"], G["CG"], G["CB"]]], want, atol=1e-12)


def test_equal_texels_render_as_resolution_one(orc):
    """Resolution 3 with its six texels equal to the patch's single texel
    renders the resolution-1 image (Theta's weights sum to 1)."""
    sc, cams, _ = S.workload("tiny")
    W, Ht = (int(v) for v in cams.wh[0])
    r3 = S.with_attributes(sc, attr_res=3, sh_degree=0, scale_jitter=0.0, quat_jitter=0.0)
    a = orc.Frame(sc, cams.cams[0], W, Ht).render()[0]
    b = orc.Frame(r3, cams.cams[0], W, Ht).render()[0]
    assert np.abs(a - b).max() < 1e-12
