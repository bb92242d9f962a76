"""Parity of the lattice variant (m Gaussians per flat sub-triangle edge,
rendered in place of the per-pixel Gaussians) against the oracle run in the
same mode.  The same bars as the pixel variant: integer outputs bit-exact,
images within 1e-4, gradients within 1e-3 of each tensor's largest entry.
"""
import numpy as np
import pytest

import oracle
from paper_2503_13961_amd import scenes as S
from tests import gpu_common as G
from tests.test_gpu_parity import GRAD_TOL, IMG_TOL, _workload

pytestmark = pytest.mark.gpu


def _gpu_record_index(cams, P, NL, v, r):
    """GPU record of the oracle's record r of view v (pixels, then lattice)."""
    po = G.view_offsets(cams)
    npx = int(po[v + 1] - po[v])
    r = np.asarray(r, np.int64)
    return np.where(r < npx, po[v] + r, po[-1] + (v * P) * NL + (r - npx))


@pytest.mark.parametrize("m,tile", [(4, 16), (2, 8), (3, 32)])
@pytest.mark.parametrize("name", ["tiny", "sphere_small", "ragged", "degree1", "degree5", "random64_r3_sh3"])
def test_lattice_stage_parity(name, m, tile):
    """Index map and boundary set as in the pixel variant; lattice records
    (mean, conic, colour, depth) against the oracle's; tile lists bit-exact
    after mapping record ids; images 1e-4."""
    G.log(f"[lattice_stage] workload={name} m={m} tile={tile}")
    sc, cams = _workload(name)
    g = G.run_gpu(sc, cams, tile=tile, lattice=m)
    assert g["status"] == 0, g["counters"]
    cfg = G.oracle_config(tile=tile, lattice=m)
    po, to = G.view_offsets(cams), G.tile_offsets(cams, tile)
    P = sc.num_prims
    R = oracle.GR
    for v, fr in enumerate(G.oracle_frames(sc, cams, cfg)):
        NL = fr.nlat // P
        sl = slice(po[v], po[v + 1])
        it, iu, isb, has = fr.raster()
        np.testing.assert_array_equal(g["I_tri"][sl], it)
        np.testing.assert_array_equal((g["pflags"][sl] & 1) != 0, has)
        np.testing.assert_array_equal((g["pflags"][sl] & 2) != 0, isb)
        rec, ren = fr.records(rendered=True)
        lat = np.nonzero(ren)[0]
        assert len(lat) and (lat >= fr.npx).all()
        gi = _gpu_record_index(cams, P, NL, v, lat)
        gr = g["rec"][gi]
        anchor = np.ascontiguousarray(gr[:, 11]).view(np.int32)     # the record's pixel, x | y << 16
        ax = (anchor << 16 >> 16).astype(np.float64)
        ay = (anchor >> 16).astype(np.float64)
        assert np.abs(ax + 0.5 + gr[:, 0] - rec[lat, R["MUX"]]).max() < 2e-5 * max(1.0, np.abs(rec[lat, R["MUX"]]).max() / 100)
        assert np.abs(ay + 0.5 + gr[:, 1] - rec[lat, R["MUY"]]).max() < 2e-5 * max(1.0, np.abs(rec[lat, R["MUY"]]).max() / 100)
        for j, key in ((2, "QA"), (3, "QB"), (4, "QC")):
            assert np.abs(gr[:, j] - rec[lat, R[key]]).max() <= 1e-6 * np.abs(rec[lat, R["QA"]]).max()
        for j, key in ((5, "CR"), (6, "CG"), (7, "CB")):
            assert np.abs(gr[:, j] - rec[lat, R[key]]).max() < 1e-6
        np.testing.assert_array_equal(gr[:, 9].view(np.int32), rec[lat, R["PRIM"]].astype(np.int32))
        # depth sort keys (the top 40 bits of the FP64 depth) bit-exact
        np.testing.assert_array_equal(g["gkey"][gi], rec[lat, R["DEPTH"]].view(np.uint64) >> np.uint64(24))
        for which, (cnt, start, lst) in enumerate(((g["g_count"], g["g_start"], g["g_list"]),
                                                   (g["b_count"], g["b_start"], g["b_list"]))):
            os_, ol = fr.lists(which)
            c = cnt[to[v]:to[v + 1]]
            np.testing.assert_array_equal(c, np.diff(os_))
            for t in range(len(c)):
                s0 = start[to[v] + t]
                want = _gpu_record_index(cams, P, NL, v, ol[os_[t]:os_[t + 1]])
                np.testing.assert_array_equal(lst[s0:s0 + c[t]], want)
        img = fr.render()[0]
        err = np.abs(g["images"][sl] - img).max()
        G.log(f"    view {v}: {len(lat)} lattice Gaussians, image max abs err {err:.3e}")
        assert err <= IMG_TOL


@pytest.mark.parametrize("name,m,no_b", [("random64", 4, False), ("sphere_small", 4, False), ("degree1", 2, False),
                                         ("degree5", 3, False), ("random64_r3_sh3", 4, False),
                                         ("sphere_small", 4, True), ("ragged", 3, False)])
def test_lattice_gradient_parity(name, m, no_b):
    """Backward of the lattice variant against the oracle's FP64 gradient
    (pinned by finite differences in the same mode)."""
    from paper_2503_13961_amd import native as N
    G.log(f"[lattice_grad] workload={name} m={m} no_boundary={no_b}")
    sc, cams = _workload(name)
    cfg = G.oracle_config(tile=16, lattice=m, no_boundary=no_b)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    gi = G.l1_cotangent(img_ref, S.l1_target(cams.num_pixels))
    g = G.run_gpu(sc, cams, tile=16, grad_images=gi, lean=True, lattice=m,
                  flags=N.BGT_FLAG_NO_BOUNDARY if no_b else 0)
    assert g["status"] == 0, g["counters"]
    err = np.abs(g["images"] - img_ref).max()
    G.log(f"    image max abs err {err:.3e}")
    assert err <= IMG_TOL
    ref = oracle.grad_views(frames, gi)
    if no_b:
        assert not g["grads"]["sharpness"].any()
    G.check_grads(g["grads"], ref, GRAD_TOL, skip=("sharpness",) if no_b else ())


@pytest.mark.parametrize("m", [4, 3])
def test_lattice_shared_edges_axis_camera(m):
    """A watertight sphere seen along the z axis: the lattice nodes on edges
    shared by two patches are coincident Gaussians of equal depth, which
    this camera often puts exactly on a depth-key boundary; the tile lists
    must still order every such pair as the oracle does."""
    import math
    G.log(f"[lattice_shared_edges] sphere freq 4, axis camera, m={m}")
    sc = S.lattice_scaled(S.deformed_sphere(freq=4, seed=3, f=160 / (2 * math.tan(math.pi / 6))), m=m, L=4)
    cams = S.make_cameras([(0.0, 0.0, 3.0)], [(160, 160)])
    g = G.run_gpu(sc, cams, tile=16, lattice=m)
    assert g["status"] == 0, g["counters"]
    fr = G.oracle_frames(sc, cams, G.oracle_config(tile=16, lattice=m))[0]
    rec = fr.records()
    d = rec[fr.npx:, oracle.GR["DEPTH"]]
    on_boundary = int(((d.view(np.uint64) & np.uint64(0xFFFFFF)) == 0).sum())
    os_, ol = fr.lists(0)
    NL = fr.nlat // sc.num_prims
    np.testing.assert_array_equal(g["g_count"], np.diff(os_))
    for t in range(len(os_) - 1):
        s0 = g["g_start"][t]
        want = _gpu_record_index(cams, sc.num_prims, NL, 0, ol[os_[t]:os_[t + 1]])
        np.testing.assert_array_equal(g["g_list"][s0:s0 + g["g_count"][t]], want)
    err = np.abs(g["images"] - fr.render()[0]).max()
    G.log(f"    depths on a key boundary: {on_boundary} of {fr.nlat}; image max abs err {err:.3e}")
    assert on_boundary > 100 and err <= IMG_TOL


def test_lattice_full_size_sphere():
    """One 800x800 view of the 2000-patch sphere with m = 4 (182,000 lattice
    Gaussians sized to the lattice spacing): index map bit-exact, the whole
    image within 1e-4; gradients within 1e-3 for a cotangent on 200 sampled
    pixels (so that the oracle's backward stays bounded)."""
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log("[lattice_full_size] sphere2k_1v 800x800, m=4")
    sc, cams, _ = S.workload("sphere2k_1v")
    sc = S.lattice_scaled(sc, m=4, L=4)
    rng = np.random.default_rng(5)
    gi = np.zeros((cams.num_pixels, 3), np.float32)
    pix = rng.choice(cams.num_pixels, 200, replace=False)
    gi[pix] = np.sign(rng.standard_normal((200, 3))) / gi.size
    g = G.run_gpu(sc, cams, tile=16, grad_images=gi, lean=True, lattice=4)
    assert g["status"] == 0, g["counters"]
    fr = G.oracle_frames(sc, cams, G.oracle_config(tile=16, lattice=4))[0]
    np.testing.assert_array_equal(g["I_tri"], fr.raster()[0])
    img = fr.render()[0]
    err = np.abs(g["images"] - img).max()
    G.log(f"    {fr.nlat} lattice Gaussians; image max abs err {err:.3e}")
    assert err <= IMG_TOL
    ref = fr.grad(gi.astype(np.float64))
    G.check_grads(g["grads"], ref, GRAD_TOL)


def test_lattice_training_step_lowers_the_loss():
    """The optimisation step (Eq. 9 loss, backward, Adam) on the lattice
    variant: recoloured and moved lattice Gaussians fitted to renders of the
    original scene; the loss falls and every parameter array stays finite."""
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    from paper_2503_13961_amd.train import TrainStep
    G.log("[lattice_train] sphere_small, m=4")
    sc, cams, _ = S.workload("sphere_small")
    sc = S.lattice_scaled(sc, m=4, L=4)
    dev = torch.device("cuda", 0)
    camt = torch.from_numpy(cams.cams).to(dev)
    target, _ = Renderer(0, lattice=4).forward(sc.degree, scene_tensors(sc, dev), camt, cams.wh)
    target = target.clone()
    pert = sc.copy()
    rng = np.random.default_rng(4)
    pert.color_ctrl[:] = np.clip(pert.color_ctrl + rng.normal(0, 0.1, pert.color_ctrl.shape), 0, 1)
    pert.ctrl[:] += rng.normal(0, 0.01, pert.ctrl.shape).astype(np.float32)
    step = TrainStep(Renderer(0, lattice=4), sc.degree, scene_tensors(pert, dev), camt, cams.wh, target)
    losses = [float(step()[0].cpu()) for _ in range(15)]
    G.log(f"    loss {losses[0]:.6f} .. {losses[-1]:.6f}")
    assert losses[-1] < 0.8 * losses[0]
    for k, v in step.params.items():
        assert torch.isfinite(v).all(), k
