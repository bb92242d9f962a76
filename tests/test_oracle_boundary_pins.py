"""Pins of the oracle's boundary radius, alpha clamp, boundary arg-min and
depth-key truncation, and a brute-force composite of the per-pixel mode with
blending coefficients (CPU only).

Each test checks the oracle against something it does not compute itself:
an eigen-decomposition by numpy, a closed form of Eq. 8 with the alpha
clamp, finite differences of its own forward, an exhaustive search over all
boundary points of a patch, or an exhaustive composite over all Gaussians
of the view without tiles.
"""
import math

import numpy as np
import pytest

from paper_2503_13961_amd import scenes as S
from tests import helpers as H


# ------------------------------------------------ sigma_i off the optical axis

def _uv_surface_points(sc, it, iu, pix, L=4):
    """S(I_uv(q)) of each pixel by de Casteljau (not the oracle's Bernstein sum)."""
    out = []
    for q in pix:
        p = int(it[q]) // (L * L)
        u, v = iu[q]
        out.append(H.decasteljau(H.scene_ctrl(sc, p), sc.degree, u, v, 1.0 - u - v))
    return np.array(out)


def test_boundary_radius_off_axis(orc):
    """sigma_i = 3 sqrt(lambda_max(r_b^2 J J^T + 0.3 I)) (Sec. 3.2, boundary
    radius; reading of the 3DGS radius convention): checked against numpy's
    symmetric eigen-solver at off-axis boundary pixels of a rotated camera,
    with wide boundary Gaussians (r_b = 0.1) so that J J^T is far from
    isotropic and has a large off-diagonal term.  Taking lambda_min, or
    dropping the off-diagonal term, moves sigma by more than 1e-3 px at
    these pixels."""
    sc = S.random_triangles(P=24, degree=2, seed=11)
    sc.sharpness[:] = np.float32(0.1)                  # r_b = r_ref / s = 0.1
    W, Ht = 96, 80
    cams = S.make_cameras([(1.4, -1.7, 2.9)], [(W, Ht)])
    cam = cams.cams[0]
    fr = orc.Frame(sc, cam, W, Ht)
    it, iu, isb, valid = fr.raster()
    rec = fr.records()
    G = orc.GR
    bpix = np.nonzero(isb & valid)[0]
    assert len(bpix) > 100
    Sq = _uv_surface_points(sc, it, iu, bpix)
    R = cam[:9].astype(np.float64).reshape(3, 3)
    t = Sq @ R.T + cam[9:12].astype(np.float64)
    f = float(cam[12])
    rb = orc.Config().r_ref / float(np.float32(0.1))
    far = 0
    for k, q in enumerate(bpix):
        tx, ty, tz = t[k]
        J = np.array([[f / tz, 0.0, -f * tx / tz ** 2], [0.0, f / tz, -f * ty / tz ** 2]])
        M = rb * rb * (J @ J.T) + 0.3 * np.eye(2)
        lam = np.linalg.eigvalsh(M)
        want = 3.0 * math.sqrt(lam[-1])
        got = rec[q, G["SIGMA"]]
        assert abs(got - want) <= 1e-9 * want, (q, got, want)
        # the pin discriminates: lambda_min, or M without its off-diagonal term
        wrong_min = 3.0 * math.sqrt(lam[0])
        wrong_diag = 3.0 * math.sqrt(max(M[0, 0], M[1, 1]))
        far += abs(wrong_min - want) > 1e-3 and abs(wrong_diag - want) > 1e-3
    assert far > len(bpix) // 2


# ------------------------------------------------ the alpha clamp of Eq. 8

def _clamp_scene(W, Ht, f, z0, log_scale=-14.0, opacity=1.0, color=(0.2, 0.5, 0.9)):
    cam = H.axis_camera(W, Ht, f)
    c3 = [H.pixel_ray_point(cam, -30.0, -20.0, z0), H.pixel_ray_point(cam, W + 40.0, -10.0, z0),
          H.pixel_ray_point(cam, 5.0, Ht + 50.0, z0)]
    sc = H.flat_patch_scene(c3, degree=1, color=color, log_scale=log_scale, opacity=opacity)
    return sc, cam


def test_alpha_clamp_closed_form(orc):
    """alpha = min(alpha_max, o w G) (Eq. 8, alpha_max = 0.99 from 3DGS).  A
    flat patch facing the camera with opacity 1: deep inside it w = 1 (no
    boundary point within sigma), every Gaussian sits on its pixel centre
    with Sigma2D = ((f s / z)^2 + 0.3) I, and a pixel composites the Gaussians
    of the 21 pixels within the support radius.  Its own has o w G = 1, so
    alpha = 0.99 and, the colour being uniform and the background black,
      C = c (1 - (1 - 0.99) prod_{d != 0} (1 - exp(-|d|^2 / (2 Sigma))))
    whatever the order.  Without the clamp C would be c exactly."""
    W, Ht, f, z0 = 24, 20, 30.0, 2.0
    sc, cam = _clamp_scene(W, Ht, f, z0)
    fr = orc.Frame(sc, cam, W, Ht)
    it, _, isb, valid = fr.raster()
    assert valid.all() and not isb.any()         # the patch covers the frame
    img, T, _, nc = fr.render()
    col = np.array([0.2, 0.5, 0.9], np.float32).astype(np.float64)
    Sig = (f * math.exp(float(np.float32(-14.0))) / z0) ** 2 + float(np.float32(0.3))
    k2 = orc.Config().kappa2
    prod = 1.0
    n_in = 0
    for dy in range(-3, 4):
        for dx in range(-3, 4):
            d2 = dx * dx + dy * dy
            if d2 / Sig > k2:
                continue
            n_in += 1
            if d2:
                prod *= 1.0 - min(0.99, math.exp(-0.5 * d2 / Sig))
    assert n_in == 21
    want = col * (1.0 - 0.01 * prod)
    checked = 0
    for y in range(4, Ht - 4):
        for x in range(4, W - 4):
            q = y * W + x
            assert nc[q] == 21
            assert np.allclose(img[q], want, rtol=0, atol=1e-9), (x, y, img[q], want)
            assert abs(T[q] - 0.01 * prod) < 1e-9
            g, al, Tt, w = fr.trace(q)
            assert (al == 0.99).sum() == 1 and np.allclose(w, 1.0)
            checked += 1
    assert checked > 100


def test_alpha_clamp_has_zero_derivative(orc):
    """A clamped alpha does not depend on o, w or G (Eq. 8): the analytic
    gradients of a scene where every interior pixel has a clamped
    contributor (opacity 1) match FP64 central differences, which stay on
    the clamped side (o w G ~ 1 > 0.99 at both ends of each step).  Routing
    the clamped term's dl/dalpha into o, the mean or the conic fails."""
    W, Ht, f, z0 = 18, 16, 30.0, 2.0
    sc, cam = _clamp_scene(W, Ht, f, z0, log_scale=-2.6)
    # no support cut-off or early stop, so the loss is smooth in the parameters
    cfg = orc.Config(tile=8, g_min=1e-300, t_min=0.0)
    fr0 = orc.Frame(sc, cam, W, Ht, cfg)
    it, iu, _, _ = fr0.raster()
    rng = np.random.default_rng(3)
    gimg = rng.normal(size=(W * Ht, 3))
    an = fr0.grad(gimg)
    clamped = sum(int((fr0.trace(q)[1] == 0.99).sum()) for q in range(W * Ht))
    assert clamped > 100

    def loss(s):
        img = orc.Frame(s, cam, W, Ht, cfg, I_tri=it, I_uv=iu).render()[0]
        return float((img * gimg).sum())

    checked = 0
    for name, idxs in (("opacity", [(0,)]), ("log_scale", [(0, 0, 0), (1, 0, 0), (2, 0, 0)]),
                       ("ctrl", [(0, 0, 0), (1, 1, 0), (2, 2, 0)]), ("quat", [(1, 0, 0), (2, 0, 0)])):
        arr = getattr(sc, name)
        for idx in idxs:
            th = float(arr[idx])
            h = max(abs(th) * 1e-4, 1e-4)
            sp, sm = sc.copy(), sc.copy()
            getattr(sp, name)[idx] = np.float32(th + h)
            getattr(sm, name)[idx] = np.float32(th - h)
            den = float(getattr(sp, name)[idx]) - float(getattr(sm, name)[idx])
            fd = (loss(sp) - loss(sm)) / den
            a = float(an[name][idx])
            assert abs(fd - a) <= 1e-6 * max(abs(fd), 1.0), (name, idx, fd, a)
            checked += 1
    assert checked == 9


# ------------------------------------------------ the boundary arg-min (Suppl. Sec. C, dl/db)

def _routing_scenes():
    cam_w, cam_h = 64, 48
    cams = S.make_cameras([(0.4, 0.3, 3.0)], [(cam_w, cam_h)])
    cam = cams.cams[0]
    # planar patches tilted against the image plane: their boundary points sit
    # on pixel centres, so pixels see many of them at (nearly) equal distances
    tilted = S.concat([
        H.flat_patch_scene([H.pixel_ray_point(cam, 5, 4, 2.6), H.pixel_ray_point(cam, 40, 6, 3.1),
                            H.pixel_ray_point(cam, 12, 40, 2.9)], sharpness=10.0),
        H.flat_patch_scene([H.pixel_ray_point(cam, 30, 20, 2.4), H.pixel_ray_point(cam, 60, 10, 2.5),
                            H.pixel_ray_point(cam, 55, 45, 2.7)], sharpness=5.0),
    ])
    curved = S.random_triangles(P=12, degree=2, seed=4)
    curved.sharpness[:] = np.float32(1.0)
    # a right-angled planar patch facing the camera, with dyadic corners,
    # focal length and depth: every boundary point lands exactly on its pixel
    # centre, and r_b is so small that every radius rounds to 3 sqrt(0.3), so
    # pixels at the inner corner and along the staircase of the long edge see
    # two points at exactly equal d/sigma
    W, Ht, f = 48, 40, 32.0
    axis = H.axis_camera(W, Ht, f)
    exact = H.flat_patch_scene([H.pixel_ray_point(axis, 8, 6, 2.0), H.pixel_ray_point(axis, 40, 6, 2.0),
                                H.pixel_ray_point(axis, 8, 38, 2.0)], sharpness=4e7)
    return [(tilted, cam, cam_w, cam_h), (curved, cam, cam_w, cam_h), (exact, axis, W, Ht)]


def test_boundary_argmin_is_exact(orc):
    """The gradient of gamma* = min_b gamma(|q - b| / sigma_b) (Eq. 7) goes to
    the boundary point that attains the minimum: the smallest d/sigma among
    the patch's points with d/sigma < 1, the lowest raster index only at an
    exactly equal ratio.  Checked at every (pixel, patch) pair of two
    scenes against an exhaustive search over all boundary points of the
    patch (not only the tile's list).  Many pixels of the tilted planar
    patches have two points within 1e-5 of each other in d/sigma with the
    higher raster index the nearer: a tie band would route those wrongly;
    and the third scene has exact ties, where the lower index must win."""
    G = orc.GR
    band_would_differ = exact_ties = 0
    for sc, cam, W, Ht in _routing_scenes():
        fr = orc.Frame(sc, cam, W, Ht, orc.Config(tile=8))
        it, _, isb, valid = fr.raster()
        rec = fr.records()
        bp = np.nonzero(isb & valid)[0]
        bprim = rec[bp, G["PRIM"]].astype(int)
        for q in range(W * Ht):
            qx, qy = q % W + 0.5, q // W + 0.5
            for g in range(sc.num_prims):
                b = bp[bprim == g]
                if not len(b):
                    continue
                dx, dy = qx - rec[b, G["MUX"]], qy - rec[b, G["MUY"]]
                ratio = np.sqrt(dx * dx + dy * dy) / rec[b, G["SIGMA"]]
                gam, arg = fr.gamma_star(q, g)
                inr = np.nonzero(ratio < 1.0)[0]
                if not len(inr):
                    assert arg == -1 and gam == 1.0
                    continue
                best = inr[np.argmin(ratio[inr])]          # first index among equal minima
                exact_ties += (ratio[inr] == ratio[best]).sum() > 1
                assert arg == b[best], (q, g, arg, b[best])
                assert abs(gam - min(1.0, 2.0 ** (ratio[best] - 1.0))) <= 1e-15
                # what a 1e-5 tie band (first point within 1e-5 of the running best) would pick
                cur = inr[0]
                for e in inr[1:]:
                    if ratio[e] < ratio[cur] - 1e-5:
                        cur = e
                band_would_differ += cur != best
    assert band_would_differ > 20 and exact_ties > 20


# ------------------------------------------------ the per-pixel mode by brute force

def test_composite_with_coefficients_bruteforce(orc):
    """The 64-patch quadratic workload at 128 x 128, every pixel: composite,
    front to back, every Gaussian of the view whose support reaches the
    pixel centre (d^T Q d <= 2 ln(1/g_min)), ordered by (depth key, pixel),
    with w = gamma* for the patch that owns the pixel in I_id and 1 - gamma*
    for the others (Eq. 6), gamma* the smallest gamma over all boundary
    points of the Gaussian's patch (Eq. 7; no tiles), alpha = min(0.99, o w
    G) (Eq. 8) and the stop after T < T_min -- against the oracle's tiled
    render, every pixel."""
    sc, cams, _ = S.workload("random64")
    W, Ht = (int(v) for v in cams.wh[0])
    cfg = orc.Config()
    fr = orc.Frame(sc, cams.cams[0], W, Ht, cfg)
    it, _, isb, valid = fr.raster()
    rec = fr.records()
    G = orc.GR
    L2 = cfg.L * cfg.L
    gid = np.nonzero(valid)[0]
    key = np.array([int(np.float64(z).view(np.uint64)) >> 24 for z in rec[gid, G["DEPTH"]]])
    order = gid[np.lexsort((gid, key))]
    r = rec[order]
    bp = np.nonzero(isb & valid)[0]
    bprim = rec[bp, G["PRIM"]].astype(int)
    # every (Gaussian, pixel) pair in the support, by the Gaussian's bbox of pixel centres
    cover = [[] for _ in range(W * Ht)]
    for rank in range(len(order)):
        mx, my = r[rank, G["MUX"]], r[rank, G["MUY"]]
        rx, ry = r[rank, G["RX"]], r[rank, G["RY"]]
        xs = np.arange(max(0, int(math.floor(mx - rx)) - 1), min(W, int(math.ceil(mx + rx)) + 2))
        ys = np.arange(max(0, int(math.floor(my - ry)) - 1), min(Ht, int(math.ceil(my + ry)) + 2))
        X, Y = np.meshgrid(xs, ys)
        dx, dy = X + 0.5 - mx, Y + 0.5 - my
        pw = r[rank, G["QA"]] * dx * dx + 2 * r[rank, G["QB"]] * dx * dy + r[rank, G["QC"]] * dy * dy
        for q, p in zip((Y * W + X)[pw <= cfg.kappa2], pw[pw <= cfg.kappa2]):
            cover[q].append((rank, p))
    img, T, _, nc = fr.render()
    checked = 0
    for q in range(W * Ht):
        qx, qy = q % W + 0.5, q // W + 0.5
        h = it[q] // L2 if it[q] >= 0 else -1
        gstar = {}
        C, Tacc, n = np.zeros(3), 1.0, 0
        for rank, pw in sorted(cover[q]):
            g = int(r[rank, G["PRIM"]])
            if g not in gstar:
                b = bp[bprim == g]
                d = np.hypot(qx - rec[b, G["MUX"]], qy - rec[b, G["MUY"]])
                gstar[g] = min(1.0, float(np.min(np.exp2(d / rec[b, G["SIGMA"]] - 1.0), initial=1.0)))
            w = gstar[g] if g == h else 1.0 - gstar[g]
            if w <= 0.0:
                continue
            a = min(cfg.alpha_max, float(sc.opacity[g]) * w * math.exp(-0.5 * pw))
            C += Tacc * a * r[rank, [G["CR"], G["CG"], G["CB"]]]
            Tacc *= 1.0 - a
            n += 1
            if Tacc < cfg.t_min:
                break
        assert n == nc[q], q
        assert np.allclose(img[q], C, rtol=0, atol=1e-12), (q, img[q], C)
        assert abs(T[q] - Tacc) <= 1e-12
        checked += n > 0
    assert checked > 0.15 * W * Ht


# ------------------------------------------------ 40-bit depth keys

@pytest.mark.parametrize("name", ["random64", "sphere_small", "flat"])
def test_truncated_depth_keys_only_break_ties(orc, name):
    """The depth test and the Gaussian order compare the FP64 depth truncated
    to its 40 high bits, ties going to the lower id (reading of the paper's
    silent tie rule).  Truncation is monotone, so against the untruncated
    FP64 depths it can only reorder items whose truncated keys are equal:
    every pixel whose winner changes, and every tile whose Gaussian order
    changes, is checked to be such a tie, and the count of flips is kept
    small.  The flat patch faces the camera, so all its depths agree to
    rounding: there the truncation turns rounding noise into raster order."""
    if name == "flat":
        W, Ht, f = 40, 32, 40.0
        cam = H.axis_camera(W, Ht, f)
        sc = H.flat_patch_scene([H.pixel_ray_point(cam, -5, -5, 2.0), H.pixel_ray_point(cam, 50, -3, 2.0),
                                 H.pixel_ray_point(cam, 8, 45, 2.0)], log_scale=-3.0)
        views = [(cam, W, Ht)]
    else:
        sc, cams, _ = S.workload(name)
        views = [(cams.cams[v], int(cams.wh[v, 0]), int(cams.wh[v, 1])) for v in range(cams.n_views)]
    G = orc.GR
    flips = pixels = reordered = 0
    for cam, W, Ht in views:
        a = orc.Frame(sc, cam, W, Ht, orc.Config(tile=8))
        b = orc.Frame(sc, cam, W, Ht, orc.Config(tile=8, exact_keys=True))
        ia, ib = a.raster()[0], b.raster()[0]
        ka, kb = a.zkeys(), b.zkeys()
        diff = np.nonzero(ia != ib)[0]
        pixels += W * Ht
        flips += len(diff)
        # the exact winner's key truncated equals the truncated winner's key,
        # and the truncated rule gave the pixel to the lower sub-triangle id
        assert ((kb[diff] >> np.uint64(24)) == (ka[diff] >> np.uint64(24))).all()
        assert (ia[diff] < ib[diff]).all()
        if len(diff):
            continue   # lists of frames with different index maps are not comparable
        rec = a.records()
        sa, la = a.lists(0)
        sb, lb = b.lists(0)
        np.testing.assert_array_equal(sa, sb)
        for t in range(len(sa) - 1):
            x, y = la[sa[t]:sa[t + 1]], lb[sb[t]:sb[t + 1]]
            if np.array_equal(x, y):
                continue
            reordered += 1
            assert sorted(x.tolist()) == sorted(y.tolist())
            kx = [int(np.float64(z).view(np.uint64)) >> 24 for z in rec[x, G["DEPTH"]]]
            ky = [int(np.float64(z).view(np.uint64)) >> 24 for z in rec[y, G["DEPTH"]]]
            assert kx == ky            # same sequence of truncated keys: only ties moved
    assert flips <= 1e-3 * pixels
    if name == "flat":
        assert reordered > 0
