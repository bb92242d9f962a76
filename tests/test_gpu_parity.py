"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Integer outputs (index map, boundary set, per-tile sorted lists) must be
bit-exact; images within 1e-4 max abs per channel; gradients within 1e-3 of
each tensor's largest reference entry and, per element, within 1e-3 of the
entry itself (entries below 1/20 of the largest: of that floor).
"""
import numpy as np
import pytest

import oracle
from paper_2503_13961_amd import scenes as S
from tests import gpu_common as G
from tests import helpers as H

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4
GRAD_TOL = 1e-3


def _workload(name):
    if "_r" in name and "_sh" in name:  # resolution-R attribute maps and SH colour of degree D
        base, rest = name.split("_r")
        R, D = (int(x) for x in rest.split("_sh"))
        sc, cams = _workload(base)
        return S.with_attributes(sc, attr_res=R, sh_degree=D, seed=R + D, sh_std=0.2), cams
    if name.startswith("degree"):  # small random scenes of every Bezier degree
        n = int(name[len("degree"):])
        sc = S.random_triangles(P=24, degree=n, seed=10 + n)
        cams = S.make_cameras([(0.2, -0.1, 4.0), (2.5, 1.5, 2.8)], [(72, 56), (45, 61)])
        return sc, cams
    if name == "ragged":
        sc = S.random_triangles(P=24, degree=3, seed=4)
        cams = S.make_cameras([(0.1, 0.2, 4.0), (3.0, 1.0, 2.5)], [(37, 29), (1, 17)])
        return sc, cams
    sc, cams, _ = S.workload(name)
    return sc, cams


@pytest.mark.parametrize("tile", [8, 16, 32])
@pytest.mark.parametrize("name", ["tiny", "random64", "sphere_small", "ragged", "degree1", "degree5",
                                  "random64_r3_sh3", "sphere_small_r3_sh3"])
def test_stage_parity(name, tile):
    """Index map, boundary set, Gaussians, tile lists and images per view."""
    G.log(f"[stage_parity] workload={name} tile={tile}")
    sc, cams = _workload(name)
    g = G.run_gpu(sc, cams, tile=tile)
    assert g["status"] == 0, g["counters"]
    cfg = G.oracle_config(tile=tile)
    po, to = G.view_offsets(cams), G.tile_offsets(cams, tile)
    for v, fr in enumerate(G.oracle_frames(sc, cams, cfg)):
        sl = slice(po[v], po[v + 1])
        it, iu, isb, val = fr.raster()
        np.testing.assert_array_equal(g["I_tri"][sl], it)
        np.testing.assert_array_equal((g["pflags"][sl] & 1) != 0, val)
        np.testing.assert_array_equal((g["pflags"][sl] & 2) != 0, isb)
        assert np.abs(g["I_uv"][sl][it >= 0] - iu[it >= 0]).max(initial=0) < 1e-6
        rec, gr = fr.records(), g["rec"][sl]
        W = fr.W
        xs = (np.arange(fr.npx) % W + 0.5)[val]
        ys = (np.arange(fr.npx) // W + 0.5)[val]
        R = oracle.GR
        assert np.abs(xs + gr[val, 0] - rec[val, R["MUX"]]).max(initial=0) < 1e-5
        assert np.abs(ys + gr[val, 1] - rec[val, R["MUY"]]).max(initial=0) < 1e-5
        for j, key in ((2, "QA"), (3, "QB"), (4, "QC")):
            ref = rec[val, R[key]]
            assert np.abs(gr[val, j] - ref).max(initial=0) <= 1e-6 * np.abs(rec[val, R["QA"]]).max(initial=1)
        for j, key in ((5, "CR"), (6, "CG"), (7, "CB")):
            assert np.abs(gr[val, j] - rec[val, R[key]]).max(initial=0) < 1e-6
        # the record's pixel (x | y << 16); the depth sort key (top 40 bits of
        # the FP64 depth) equal or, where the depth sits on a key boundary, one off
        anchor = np.ascontiguousarray(gr[val, 11]).view(np.int32)
        np.testing.assert_array_equal(anchor, (np.arange(fr.npx) % W + (np.arange(fr.npx) // W << 16))[val])
        kd = g["gkey"][sl][val].astype(np.int64) - (rec[val, R["DEPTH"]].view(np.uint64) >> np.uint64(24)).astype(np.int64)
        assert np.abs(kd).max(initial=0) <= 1
        sig = rec[isb, R["SIGMA"]]
        assert np.abs(gr[isb, 10] - sig).max(initial=0) <= 1e-6 * max(sig.max(initial=1), 1)
        # per-tile lists: same entries in the same order
        for which, (cnt, start, lst) in enumerate(((g["g_count"], g["g_start"], g["g_list"]),
                                                   (g["b_count"], g["b_start"], g["b_list"]))):
            os_, ol = fr.lists(which)
            c = cnt[to[v]:to[v + 1]]
            np.testing.assert_array_equal(c, np.diff(os_))
            for t in range(len(c)):
                s0 = start[to[v] + t]
                mine = lst[s0:s0 + c[t]] - po[v]
                np.testing.assert_array_equal(mine, ol[os_[t]:os_[t + 1]])
        img, T, vis, nc = fr.render()
        err = np.abs(g["images"][sl] - img).max()
        G.log(f"    view {v}: image max abs err {err:.3e}")
        assert err <= IMG_TOL


def test_tessellate_matches_oracle():
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log("[tessellate] degrees 1..5")
    r = Renderer(0)
    for n in range(1, 6):
        sc = S.random_triangles(P=37, degree=n, seed=n)
        out = r.tessellate(n, scene_tensors(sc, torch.device("cuda", 0))).cpu().numpy()
        ref = oracle.tessellate(sc, 4)
        assert np.abs(out - ref).max() <= 2e-7 * (1 + np.abs(ref).max())


def test_full_size_sphere_image():
    """One 800x800 view of the 2000-patch sphere: bit-exact index map, image 1e-4."""
    G.log("[full_size] sphere2k_1v 800x800")
    sc, cams, _ = S.workload("sphere2k_1v")
    g = G.run_gpu(sc, cams, tile=16)
    fr = G.oracle_frames(sc, cams, G.oracle_config(tile=16))[0]
    it = fr.raster()[0]
    np.testing.assert_array_equal(g["I_tri"], it)
    img = fr.render()[0]
    err = np.abs(g["images"] - img).max()
    G.log(f"    image max abs err {err:.3e}")
    assert err <= IMG_TOL


@pytest.mark.parametrize("name", ["random64", "sphere_small", "ragged", "degree1", "degree4", "degree5",
                                  "random64_r3_sh3", "sphere_small_r3_sh3", "random64_r3_sh0", "random64_r1_sh2",
                                  "degree5_r3_sh3", "degree1_r3_sh1"])
def test_gradient_parity(name):
    """Backward against the oracle's analytic FP64 gradient (itself pinned by
    finite differences) for an L1 loss to a random target."""
    G.log(f"[grad_parity] workload={name}")
    sc, cams = _workload(name)
    cfg = G.oracle_config(tile=16)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    gi = G.l1_cotangent(img_ref, S.l1_target(cams.num_pixels))
    g = G.run_gpu(sc, cams, tile=16, grad_images=gi)
    ref = oracle.grad_views(frames, gi)
    G.check_grads(g["grads"], ref, GRAD_TOL)


@pytest.mark.parametrize("W,tile", [(300, 16), (200, 32)])
def test_boundary_lists_over_the_lds_stage(W, tile):
    """Tiles whose boundary list is longer than the LDS stage holds (the dense
    20,000-patch box at a small size): runs staged in full are read from LDS,
    the others from global memory; image and gradients still match."""
    G.log(f"[edge] boundary lists over the LDS stage: box20k {W}x{W} tile {tile}")
    sc, _, _ = S.workload("box20k_cubic")
    cams = S.make_cameras([(0.0, 0.0, 8.0)], [(W, W)])
    cfg = G.oracle_config(tile=tile)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    gi = G.l1_cotangent(img_ref, S.l1_target(cams.num_pixels))
    g = G.run_gpu(sc, cams, tile=tile, grad_images=gi, lean=True)
    assert g["counters"][7] > 0, "no tile overflowed the boundary stage"
    err = np.abs(g["images"] - img_ref).max()
    G.log(f"    {g['counters'][7]} tiles over the stage; image max abs err {err:.3e}")
    assert err <= IMG_TOL
    ref = oracle.grad_views(frames, gi)
    G.check_grads(g["grads"], ref, GRAD_TOL)


@pytest.mark.parametrize("name", ["random64", "sphere_small", "degree3", "random64_r3_sh3"])
def test_without_coefficients_parity(name):
    """The ablation variant without blending coefficients (w = 1 for every
    Gaussian): no boundary points, index map bit-exact, image 1e-4 and
    gradients 1e-3 against the oracle run in the same mode."""
    from paper_2503_13961_amd import native as N
    G.log(f"[no_boundary] workload={name}")
    sc, cams = _workload(name)
    cfg = G.oracle_config(tile=16, no_boundary=True)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    gi = G.l1_cotangent(img_ref, S.l1_target(cams.num_pixels))
    g = G.run_gpu(sc, cams, tile=16, grad_images=gi, flags=N.BGT_FLAG_NO_BOUNDARY)
    assert g["status"] == 0, g["counters"]
    assert not (g["pflags"] & 2).any() and not g["b_count"].any()
    po = G.view_offsets(cams)
    for v, fr in enumerate(frames):
        np.testing.assert_array_equal(g["I_tri"][po[v]:po[v + 1]], fr.raster()[0])
    err = np.abs(g["images"] - img_ref).max()
    G.log(f"    image max abs err {err:.3e}")
    assert err <= IMG_TOL
    ref = oracle.grad_views(frames, gi)
    assert not g["grads"]["sharpness"].any()
    G.check_grads(g["grads"], ref, GRAD_TOL, skip=("sharpness",))


def test_batched_equals_per_view():
    """All views in one call give bit-identical images to one call per view."""
    G.log("[batched_vs_per_view] sphere_small")
    sc, cams = _workload("sphere_small")
    g = G.run_gpu(sc, cams, tile=16)
    po = G.view_offsets(cams)
    for v in range(cams.n_views):
        gv = G.run_gpu(sc, cams.view(v), tile=16)
        np.testing.assert_array_equal(gv["images"], g["images"][po[v]:po[v + 1]])
        np.testing.assert_array_equal(gv["I_tri"], g["I_tri"][po[v]:po[v + 1]])


def test_tile_size_and_determinism():
    """Images are bit-identical across tile sizes 8/16/32 and across runs."""
    G.log("[tile_invariance] sphere_small")
    sc, cams = _workload("sphere_small")
    base = G.run_gpu(sc, cams, tile=16)
    again = G.run_gpu(sc, cams, tile=16)
    np.testing.assert_array_equal(base["images"], again["images"])
    for tile in (8, 32):
        np.testing.assert_array_equal(G.run_gpu(sc, cams, tile=tile)["images"], base["images"])


@pytest.mark.parametrize("name", ["sphere2k_16v_mixed", "box20k_300"])
def test_gradients_repeat_across_runs(name):
    """Forward and backward of the same inputs, six times on one state: the
    gradients agree to 1e-5 of each tensor's largest entry and, per element,
    to 1e-5 of max(|g|, floor) (the float atomics of the sums may add in any
    order, which moves the last bits, but no contribution may be lost or
    counted twice).  The 20,000-patch box at 300 x 300 puts more boundary
    runs in a tile than the gamma* maps hold and more boundary points than the
    LDS stage holds, so the per-pixel searches and their global atomics run
    too.  Images are bit-identical."""
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log(f"[repeat] {name}: gradients of six runs")
    if name == "box20k_300":
        sc, _, _ = S.workload("box20k_cubic")
        cams = S.make_cameras([(0.0, 0.0, 8.0)], [(300, 300)])
    else:
        sc, cams, _ = S.workload(name)
    dev = torch.device("cuda", 0)
    r = Renderer(0)
    params = scene_tensors(sc, dev)
    camt = torch.from_numpy(cams.cams).to(dev)
    wh = np.ascontiguousarray(cams.wh, np.int32)
    gi = torch.from_numpy((np.sign(np.random.default_rng(0).random((cams.num_pixels, 3)) - 0.5)
                           / (3 * cams.num_pixels)).astype(np.float32)).to(dev)
    runs, imgs, state, images = [], [], None, None
    for _ in range(6):
        images, state = r.forward(sc.degree, params, camt, wh, state=state, images=images)
        g = r.backward(sc.degree, params, camt, wh, images, gi, state)
        torch.cuda.synchronize()
        runs.append({k: v.cpu().numpy().copy() for k, v in g.items()})
        imgs.append(images.cpu().numpy().copy())
    if name == "box20k_300":
        cnt = r.query(state)[1]
        assert cnt[7] > 0 and cnt[8] > 0, cnt
    for img in imgs[1:]:
        np.testing.assert_array_equal(img, imgs[0])
    for run in runs[1:]:
        for k, ref in runs[0].items():
            e = G.grad_error(run[k], ref)
            el = G.grad_rel_error(run[k], ref)
            assert e <= 1e-5 and el <= 1e-5, (k, e, el)


def test_everything_behind_the_camera():
    """All geometry behind z_near: background image and zero gradients."""
    G.log("[edge] behind camera")
    sc = S.random_triangles(P=8, degree=2, seed=2)
    cams = S.make_cameras([(0.0, 0.0, 4.0)], [(40, 30)])
    cams.cams[0, 9:12] = (0.0, 0.0, -10.0)  # move the world 10 units behind the camera
    bg = (0.25, 0.5, 0.75)
    g = G.run_gpu(sc, cams, tile=16, bg=bg, grad_images=np.ones((1200, 3)))
    assert (g["I_tri"] == -1).all()
    assert np.allclose(g["images"], np.array(bg, np.float32))
    for k, v in g["grads"].items():
        assert not v.any(), k


def test_overflow_is_reported_and_recovered():
    """A pair capacity far too small is flagged; the front end grows it and the
    retried render matches the oracle."""
    import torch
    from paper_2503_13961_amd import native as N
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log("[edge] overflow")
    sc, cams = _workload("random64")
    r = Renderer(0, pair_factor=0.01, bpair_factor=0.01)
    dev = torch.device("cuda", 0)
    p = scene_tensors(sc, dev)
    ct = torch.from_numpy(cams.cams).to(dev)
    _, state = r.forward(sc.degree, p, ct, cams.wh, check=False)
    st, cnt = r.query(state)
    assert st == N.BGT_E_OVERFLOW and cnt[0] & 1
    images, state = r.forward(sc.degree, p, ct, cams.wh, check=True)
    fr = G.oracle_frames(sc, cams, G.oracle_config())[0]
    assert np.abs(images.cpu().numpy() - fr.render()[0]).max() <= IMG_TOL


def test_invalid_arguments_enqueue_nothing():
    import torch
    from paper_2503_13961_amd import native as N
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log("[edge] invalid arguments")
    r = Renderer(0)
    sc, cams = _workload("tiny")
    dev = torch.device("cuda", 0)
    p = scene_tensors(sc, dev)
    ct = torch.from_numpy(cams.cams).to(dev)
    pr = r.prims_struct(sc.degree, p)
    vw = r.views_struct(ct, cams.wh)
    with pytest.raises(N.BgtError) as e:
        N.bgt_render_fwd(r.ctx, pr, vw, 0, 0, 0, 0)
    assert e.value.status == N.BGT_E_INVALID
    with pytest.raises(N.BgtError) as e:
        N.bgt_render_fwd(r.ctx, pr, vw, ct.data_ptr(), ct.data_ptr(), 16, 0)
    assert e.value.status == N.BGT_E_NOMEM
    bad = N.make_prims(7, sc.num_prims, *(p[k].data_ptr() for k in ("ctrl", "color_ctrl", "log_scale", "quat",
                                                                     "opacity", "sharpness")))
    with pytest.raises(N.BgtError) as e:
        N.bgt_state_size(r.ctx, bad, vw)
    assert e.value.status == N.BGT_E_INVALID
