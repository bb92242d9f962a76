"""Rare paths of the HIP path against the oracle: tile lists longer than the
LDS sort holds (the global-memory sort), patches with NaN or infinite
control points, and thin sub-triangles reaching far outside the view."""
import numpy as np
import pytest

import oracle
from paper_2503_13961_amd import scenes as S
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


def _lists_equal(g, fr, to, po, v):
    """Both tile lists of view v in the same order as the oracle's."""
    for which, (cnt, start, lst) in enumerate(((g["g_count"], g["g_start"], g["g_list"]),
                                               (g["b_count"], g["b_start"], g["b_list"]))):
        os_, ol = fr.lists(which)
        c = cnt[to[v]:to[v + 1]]
        np.testing.assert_array_equal(c, np.diff(os_))
        for t in range(len(c)):
            s0 = start[to[v] + t]
            np.testing.assert_array_equal(lst[s0:s0 + c[t]] - po[v], ol[os_[t]:os_[t + 1]])


def _long_lists(which):
    sc, _, _ = S.workload("random64")
    if which == "gauss":     # Gaussians about 7 times wider: up to 2675 per 16 x 16 tile
        sc.log_scale[:] += np.float32(2.0)
        cams = S.make_cameras([(0.0, 0.0, 4.0)], [(128, 128)])
    else:                    # boundary radii of tens of pixels: every boundary point in every tile's list
        sc.sharpness[:] = np.float32(0.01)
        cams = S.make_cameras([(0.0, 0.0, 4.0)], [(256, 256)])
    return sc, cams


@pytest.mark.parametrize("which", ["gauss", "boundary"])
def test_tile_lists_beyond_the_lds_sort(which):
    """Tile lists of more than 2048 entries are sorted by the global-memory
    network instead of in LDS: the library counts them, the lists are
    bit-exact against the oracle's, and image and gradients match."""
    G.log(f"[rare] lists over the LDS sort: {which}")
    sc, cams = _long_lists(which)
    cfg = G.oracle_config(tile=16)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    gi = G.l1_cotangent(img_ref, S.l1_target(cams.num_pixels))
    g = G.run_gpu(sc, cams, tile=16, grad_images=gi)
    assert g["status"] == 0, g["counters"]
    G.log(f"    {g['counters'][6]} tiles sorted in global memory")
    assert g["counters"][6] > 0
    longest = max(np.diff(frames[0].lists(w)[0]).max() for w in (0, 1))
    assert longest > 2048
    _lists_equal(g, frames[0], G.tile_offsets(cams, 16), G.view_offsets(cams), 0)
    err = np.abs(g["images"] - img_ref).max()
    G.log(f"    image max abs err {err:.3e}")
    assert err <= IMG_TOL
    G.check_grads(g["grads"], oracle.grad_views(frames, gi))


def test_nonfinite_control_points():
    """Patches with a NaN control point, or with +inf and -inf in one
    coordinate, evaluate to NaN at every tessellation node: every vertex
    fails the near-plane test (NaN compares false), so their sub-triangles
    are culled and they win no pixel.  The other patches render as the
    oracle renders the same input (which culls them the same way), no
    overflow is flagged, and every gradient is finite (those of the culled
    patches zero)."""
    G.log("[rare] non-finite control points")
    sc, cams, _ = S.workload("random64")
    bad_nan, bad_inf = [3, 17, 40], [8, 51]
    for p in bad_nan:
        sc.ctrl[1, 2, p] = np.nan
    for p in bad_inf:
        sc.ctrl[0, 0, p] = np.inf
        sc.ctrl[0, 4, p] = -np.inf
    cfg = G.oracle_config(tile=16)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    gi = G.l1_cotangent(img_ref, S.l1_target(cams.num_pixels))
    g = G.run_gpu(sc, cams, tile=16, grad_images=gi)
    assert g["status"] == 0 and g["counters"][0] == 0, g["counters"]
    it = frames[0].raster()[0]
    np.testing.assert_array_equal(g["I_tri"], it)
    won = set((it[it >= 0] // 16).tolist())
    assert won and not won & set(bad_nan + bad_inf)
    err = np.abs(g["images"] - img_ref).max()
    G.log(f"    {len(won)} patches win pixels; image max abs err {err:.3e}")
    assert np.isfinite(g["images"]).all() and err <= IMG_TOL
    ref = oracle.grad_views(frames, gi)
    for k, v in g["grads"].items():
        assert np.isfinite(v).all(), k
        assert not v.reshape(ref[k].shape)[..., bad_nan + bad_inf].any(), k
    G.check_grads(g["grads"], ref)


def test_far_reaching_slivers():
    """Sub-triangles with a small box in the image whose corners lie more
    than 2^17 px apart (thin bands across the view from corners 600000 px
    outside it) are rasterized by the int64 path, not the per-wave FP64 one,
    whose edge functions are exact only for narrower triangles: the library
    counts them as big triangles (27 of the three bands' sub-triangles have a
    box in the view, each under 256 px), and the index map is bit-exact
    against the oracle's."""
    from tests import helpers as H
    G.log("[rare] far-reaching slivers")
    W, Hh = 64, 48
    cam = H.axis_camera(W, Hh, 40.0)
    pts = lambda cs, z: [H.pixel_ray_point(cam, x, y, z) for x, y in cs]
    sc = S.concat([H.flat_patch_scene(pts(c, z), color=col) for c, z, col in (
        ([(-600000.0, 10.0), (600000.0, 10.0), (30.3, 13.5)], 2.0, (1, 0, 0)),
        ([(20.2, -600000.0), (20.2, 600000.0), (23.9, 24.6)], 2.5, (0, 1, 0)),
        ([(-600000.0, 30.1), (600000.0, 33.2), (41.7, 36.6)], 1.5, (0, 0, 1)),
        ([(-5.0, -5.0), (70.0, -3.0), (20.0, 60.0)], 4.0, (1, 1, 1)),  # an ordinary patch behind them
    )])
    cams = S.Cameras(cam[None, :].copy(), np.array([[W, Hh]], np.int32), [(0.0, 0.0, 0.0)])
    cfg = G.oracle_config(tile=16)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    g = G.run_gpu(sc, cams, tile=16)
    assert g["status"] == 0 and g["counters"][0] == 0, g["counters"]
    G.log(f"    {g['counters'][5]} big triangles")
    assert g["counters"][5] >= 27
    it = frames[0].raster()[0]
    assert set(range(4)) <= set((it[it >= 0] // 16).tolist())  # every band wins pixels
    np.testing.assert_array_equal(g["I_tri"], it)
    err = np.abs(g["images"] - img_ref).max()
    G.log(f"    image max abs err {err:.3e}")
    assert err <= IMG_TOL
