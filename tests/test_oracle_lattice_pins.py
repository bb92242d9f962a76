"""Pins of the oracle's Gaussian-lattice variant: instead of one Gaussian per
foreground pixel (Sec. 3.2, Sub-Primitive Generation), each patch carries a
lattice of m Gaussians per flat sub-triangle edge, shared along the edges
of neighbouring sub-triangles, i.e. the nodes (a, b), a + b <= L (m - 1), of
the patch's (u, v) domain.  Boundary points and blending coefficients are
those of the pixel variant.
"""
import math

import numpy as np
import pytest

from paper_2503_13961_amd import scenes as S
from tests import helpers as H


def _proj(cam, X):
    R = cam[:9].astype(np.float64).reshape(3, 3)
    t = R @ np.asarray(X, np.float64) + cam[9:12]
    return np.array([cam[12] * t[0] / t[2] + cam[14], cam[13] * t[1] / t[2] + cam[15]]), t[2]


def _nodes(level):
    return [(a, b) for a in range(level + 1) for b in range(level + 1 - a)]


@pytest.mark.parametrize("m,L", [(4, 4), (2, 1), (3, 2)])
def test_lattice_records_sit_on_the_surface(orc, m, L):
    """Record npx + p NL + k is the Gaussian of patch p at node k = (a, b) of
    the level-L(m-1) lattice, (u, v) = (a, b) / (L (m-1)): its mean is the
    projection of S(u, v) (triangular de Casteljau, Eq. 1-3), its colour
    the colour net at (u, v) (Eq. 4), its depth the camera z; the lattice
    holds every tessellation vertex."""
    sc, cams, _ = S.workload("tiny")
    W, Ht = (int(v) for v in cams.wh[0])
    cam = cams.cams[0]
    fr = orc.Frame(sc, cam, W, Ht, orc.Config(L=L, lattice=m))
    lev = L * (m - 1)
    nodes = _nodes(lev)
    NL = len(nodes)
    assert NL == (lev + 1) * (lev + 2) // 2 and fr.nlat == sc.num_prims * NL
    rec, ren = fr.records(rendered=True)
    G = orc.GR
    npx = W * Ht
    assert not ren[:npx].any()            # pixel records are boundary points only
    checked = 0
    for p in range(sc.num_prims):
        cp, cc = H.scene_ctrl(sc, p), sc.color_ctrl[:, :, p].T.astype(np.float64)
        for k, (a, b) in enumerate(nodes):
            u, v = a / lev, b / lev
            X = H.decasteljau(cp, sc.degree, u, v, 1.0 - u - v)
            mu, z = _proj(cam, X)
            r = rec[npx + p * NL + k]
            if z <= 0.2:
                assert not ren[npx + p * NL + k]
                continue
            assert ren[npx + p * NL + k] and int(r[G["PRIM"]]) == p
            assert np.allclose(r[[G["MUX"], G["MUY"]]], mu, rtol=0, atol=1e-9)
            assert abs(r[G["DEPTH"]] - z) < 1e-12
            col = H.decasteljau(cc, sc.degree, u, v, 1.0 - u - v)
            assert np.allclose(r[[G["CR"], G["CG"], G["CB"]]], col, rtol=0, atol=1e-12)
            checked += 1
    assert checked > 0.9 * fr.nlat
    # the tessellation vertices (a', b') / L are the nodes (a' (m-1), b' (m-1))
    tess = orc.tessellate(sc, L)
    for k, (a, b) in enumerate(_nodes(L)):
        kk = nodes.index((a * (m - 1), b * (m - 1)))
        for p in range(sc.num_prims):
            mu, _ = _proj(cam, tess[:, k, p])
            assert np.allclose(rec[npx + p * NL + kk, [G["MUX"], G["MUY"]]], mu, rtol=0, atol=1e-9)


def test_lattice_lists_hold_lattice_gaussians_and_pixel_boundary_points(orc):
    """The tile lists of the rendered Gaussians hold lattice records only,
    sorted by (depth key, record index); the boundary lists hold the boundary
    pixels of the pixel variant, unchanged."""
    sc, cams, _ = S.workload("tiny")
    W, Ht = (int(v) for v in cams.wh[0])
    pix = orc.Frame(sc, cams.cams[0], W, Ht, orc.Config(tile=8))
    lat = orc.Frame(sc, cams.cams[0], W, Ht, orc.Config(tile=8, lattice=4))
    npx = W * Ht
    gs, gl = lat.lists(0)
    assert len(gl) and (gl >= npx).all()
    rec = lat.records()
    for t in range(lat.tiles_x * lat.tiles_y):
        e = gl[gs[t]:gs[t + 1]]
        key = [(int(np.float64(z).view(np.uint64)) >> 24, int(i)) for z, i in zip(rec[e, orc.GR["DEPTH"]], e)]
        assert key == sorted(key)
    np.testing.assert_array_equal(pix.lists(1)[0], lat.lists(1)[0])
    np.testing.assert_array_equal(pix.lists(1)[1], lat.lists(1)[1])
    np.testing.assert_array_equal(pix.raster()[2], lat.raster()[2])
    rp = pix.records()
    bp = np.nonzero(pix.raster()[2])[0]
    np.testing.assert_array_equal(rp[bp], rec[bp])     # boundary points: same records


@pytest.mark.parametrize("no_boundary", [True, False])
def test_lattice_composite_bruteforce(orc, no_boundary):
    """Every pixel composites, front to back, the lattice Gaussians whose
    support reaches it: alpha = min(alpha_max, o w G) with w = gamma* for the
    patch that owns the pixel in I_id and 1 - gamma* for the others (Eq. 6-8),
    gamma* the smallest gamma over all boundary points of the Gaussian's patch
    (no tiles), and w = 1 without blending coefficients."""
    sc, cams, _ = S.workload("tiny")
    sc.log_scale[:] -= 0.5
    W, Ht = (int(v) for v in cams.wh[0])
    cfg = orc.Config(tile=8, lattice=4, no_boundary=no_boundary)
    fr = orc.Frame(sc, cams.cams[0], W, Ht, cfg)
    it, _, isb, has = fr.raster()
    rec, ren = fr.records(rendered=True)
    G = orc.GR
    gid = np.nonzero(ren)[0]
    key = np.array([int(np.float64(z).view(np.uint64)) >> 24 for z in rec[gid, G["DEPTH"]]])
    order = gid[np.lexsort((gid, key))]
    r = rec[order]
    bp = np.nonzero(isb & has)[0]
    img, T, _, nc = fr.render()
    L2 = cfg.L * cfg.L
    checked = 0
    for pix in range(0, W * Ht, 5):
        qx, qy = pix % W + 0.5, pix // W + 0.5
        dx, dy = qx - r[:, G["MUX"]], qy - r[:, G["MUY"]]
        pw = r[:, G["QA"]] * dx * dx + 2 * r[:, G["QB"]] * dx * dy + r[:, G["QC"]] * dy * dy
        cov = np.nonzero(pw <= cfg.kappa2)[0]
        h = it[pix] // L2 if it[pix] >= 0 else -1
        want, wa, wal = [], [], []
        Tacc = 1.0
        for c in cov:
            g = int(r[c, G["PRIM"]])
            w = 1.0
            if not no_boundary:
                b = bp[rec[bp, G["PRIM"]].astype(int) == g]
                d = np.hypot(qx - rec[b, G["MUX"]], qy - rec[b, G["MUY"]])
                gam = min(1.0, float(np.min(np.exp2(d / rec[b, G["SIGMA"]] - 1.0), initial=1.0)))
                w = gam if g == h else 1.0 - gam
            if w <= 0.0:
                continue
            a = min(cfg.alpha_max, float(sc.opacity[g]) * w * math.exp(-0.5 * pw[c]))
            want.append(order[c]); wa.append(w); wal.append(a)
            Tacc *= 1.0 - a
            if Tacc < cfg.t_min:
                break
        g, al, Tt, w = fr.trace(pix)
        np.testing.assert_array_equal(g, want)
        assert np.allclose(w, wa, rtol=0, atol=1e-12) and np.allclose(al, wal, rtol=0, atol=1e-12)
        col = r[[list(order).index(x) for x in want]][:, [G["CR"], G["CG"], G["CB"]]] if want else np.zeros((0, 3))
        Tb = np.concatenate([[1.0], np.cumprod(1.0 - np.array(wal))])
        assert np.allclose(img[pix], (Tb[:-1, None] * np.array(wal)[:, None] * col).sum(0),
                           rtol=0, atol=1e-12)
        checked += len(want) > 0
    assert checked > 100


def test_lattice_of_a_flat_patch_fills_it(orc):
    """A flat patch facing the camera, with Gaussians as wide as the lattice
    spacing: the interior pixels receive a nearly constant opacity (the
    lattice covers the patch evenly), which is what the variant is for."""
    W, Ht, f, z0 = 64, 64, 64.0, 2.0
    cam = H.axis_camera(W, Ht, f)
    c3 = [H.pixel_ray_point(cam, 4, 4, z0), H.pixel_ray_point(cam, 60, 4, z0), H.pixel_ray_point(cam, 4, 60, z0)]
    spacing = np.linalg.norm(c3[1] - c3[0]) / 12
    sc = H.flat_patch_scene(c3, degree=1, color=(1, 1, 1), log_scale=math.log(0.6 * spacing), opacity=0.9)
    fr = orc.Frame(sc, cam, W, Ht, orc.Config(lattice=4, no_boundary=True))
    img = fr.render()[0][:, 0].reshape(Ht, W)
    inner = img[14:36, 14:36][np.add.outer(np.arange(14, 36), np.arange(14, 36)) < 52]
    assert inner.min() > 0.9 and inner.max() - inner.min() < 0.05


def test_lattice_config_validation(orc):
    sc, cams, _ = S.workload("tiny")
    with pytest.raises(ValueError):
        orc.Frame(sc, cams.cams[0], 70, 53, orc.Config(lattice=1))
