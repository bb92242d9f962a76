"""Splitting and pruning through the C ABI against oracle/densify.py.

Integer statistics (views, texels, pixel counts), the decisions and the
output slots are bit-exact; the edge-prior sums (float atomics) are within
1e-5, the gradient sums within the gradient tolerance 1e-3 (they are sums
of backward-pass norms, which carry it); the children's nets are FP64
blossoms rounded to float: within 2 float ulps of the oracle's.
"""
import numpy as np
import pytest

import oracle
from oracle import densify as D
from paper_2503_13961_amd import scenes as S
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _stats_to_host(st):
    return {k: v.cpu().numpy() for k, v in st.t.items()}


@pytest.mark.parametrize("name", ["sphere_small", "random64"])
def test_statistics_match_oracle(name):
    import torch
    from paper_2503_13961_amd.densify import PrimStats
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log(f"[densify] statistics: {name}")
    sc, cams, _ = S.workload(name)
    dev = torch.device("cuda", 0)
    r = Renderer(0)
    params = scene_tensors(sc, dev)
    camt = torch.from_numpy(cams.cams).to(dev)
    images, state = r.forward(sc.degree, params, camt, cams.wh)
    targets = np.random.default_rng(2).random((cams.num_pixels, 3)).astype(np.float32)
    cfg = G.oracle_config(tile=16)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    gi = G.l1_cotangent(img_ref, targets)
    grads = r.backward(sc.degree, params, camt, cams.wh, images,
                       torch.from_numpy(np.ascontiguousarray(gi, np.float32)).to(dev), state)
    st = PrimStats(sc.num_prims, dev)
    st.accumulate(r, sc.degree, params, camt, cams.wh, state, torch.from_numpy(targets).to(dev), grads)
    st.accumulate(r, sc.degree, params, camt, cams.wh, state)          # visibility only
    got = _stats_to_host(st)
    ref = D.Stats(sc.num_prims)
    its = [fr.raster()[0] for fr in frames]
    ref.accumulate(its, [tuple(int(x) for x in w) for w in cams.wh], targets, oracle.grad_views(frames, gi)["ctrl"])
    ref.accumulate(its, [tuple(int(x) for x in w) for w in cams.wh])
    assert int(got["views_seen"][0]) == ref.views_seen
    np.testing.assert_array_equal(got["vis_views"], ref.vis_views)
    np.testing.assert_array_equal(got["tex"].view(np.uint64), ref.tex)
    assert not got["view_bits"].any()
    np.testing.assert_array_equal(got["edge_cnt"], ref.edge_cnt)
    np.testing.assert_array_equal(got["grad_cnt"], ref.grad_cnt)
    e = np.abs(got["edge_sum"] - ref.edge_sum).max() / max(np.abs(ref.edge_sum).max(), 1e-30)
    gsum = np.abs(got["grad_sum"] - ref.grad_sum).max() / max(np.abs(ref.grad_sum).max(), 1e-30)
    G.log(f"    visible patches {int((ref.vis_views > 0).sum())}; edge sums {e:.2e}; gradient sums {gsum:.2e}")
    assert e <= 1e-5 and gsum <= 1e-3


@pytest.mark.parametrize("degree,attrs", [(1, False), (2, False), (3, False), (5, False), (2, True)])
def test_plan_and_apply_match_oracle(degree, attrs):
    """Statistics set so that every rule fires on some patch; the decision,
    slots and count are exact and the rebuilt arrays match."""
    import torch
    from paper_2503_13961_amd import densify as DZ
    from paper_2503_13961_amd.densify import PrimStats
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log(f"[densify] plan and apply, degree {degree}")
    sc = S.random_triangles(P=300, degree=degree, seed=20 + degree)
    if attrs:   # resolution-3 maps and SH colour travel with each child
        sc = S.with_attributes(sc, attr_res=3, sh_degree=3, seed=degree)
    P = sc.num_prims
    rng = np.random.default_rng(degree)
    ref = D.Stats(P)
    ref.views_seen = 20
    ref.vis_views[:] = rng.integers(0, 21, P)
    ref.tex[:] = rng.integers(0, 1 << 16, P).astype(np.uint64)
    ref.grad_cnt[:] = rng.integers(0, 5, P)
    ref.grad_sum[:] = (rng.random(P) * 0.004 * ref.grad_cnt).astype(np.float32)
    ref.edge_cnt[:] = rng.integers(0, 50, P)
    ref.edge_sum[:] = (rng.random(P) * 26 * ref.edge_cnt).astype(np.float32)
    dev = torch.device("cuda", 0)
    r = Renderer(0)
    params = scene_tensors(sc, dev)
    st = PrimStats(P, dev)
    st.t["views_seen"][0] = ref.views_seen
    st.t["vis_views"].copy_(torch.from_numpy(ref.vis_views.astype(np.int32)))
    st.t["tex"].copy_(torch.from_numpy(ref.tex.view(np.int64)))
    st.t["grad_cnt"].copy_(torch.from_numpy(ref.grad_cnt.astype(np.int32)))
    st.t["grad_sum"].copy_(torch.from_numpy(ref.grad_sum.astype(np.float32)))
    st.t["edge_cnt"].copy_(torch.from_numpy(ref.edge_cnt.astype(np.int32)))
    st.t["edge_sum"].copy_(torch.from_numpy(ref.edge_sum.astype(np.float32)))
    action, dst, count = DZ.plan(r, degree, params, st)
    ra, rd, rc = D.plan(sc, ref)
    counts = np.bincount(ra, minlength=3)
    G.log(f"    keep {counts[0]}, split {counts[1]}, prune {counts[2]}; {P} -> {rc} patches")
    assert counts.min() > 0
    np.testing.assert_array_equal(action.cpu().numpy(), ra)
    np.testing.assert_array_equal(dst.cpu().numpy(), rd)
    assert count == rc
    new = DZ.apply(r, degree, params, action, dst, count)
    want = D.apply(sc, ra, rd)
    for k in ("ctrl", "color_ctrl"):
        got = new[k].cpu().numpy().astype(np.float64)
        ulp = np.spacing(np.abs(want[k]).astype(np.float32)).astype(np.float64)
        assert (np.abs(got - want[k]) <= 2 * ulp + 1e-30).all(), k
    for k in ("log_scale", "quat", "opacity", "sharpness") + (("sh",) if attrs else ()):
        np.testing.assert_array_equal(new[k].cpu().numpy(), want[k])


def test_split_scene_renders_the_parent_surface():
    """After splitting every patch, the children tessellate the same surface
    more finely: the foreground of the image (the union of the patches'
    projections) is unchanged except on the silhouette's rim."""
    import torch
    from paper_2503_13961_amd import densify as DZ
    from paper_2503_13961_amd.densify import PrimStats
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log("[densify] split everything: sphere_small")
    sc, cams, _ = S.workload("sphere_small")
    dev = torch.device("cuda", 0)
    r = Renderer(0)
    params = scene_tensors(sc, dev)
    st = PrimStats(sc.num_prims, dev)
    st.t["views_seen"][0] = 1
    st.t["vis_views"].fill_(1)
    st.t["tex"].fill_(-1)
    st.t["grad_cnt"].fill_(1)
    st.t["grad_sum"].fill_(1.0)
    new, action = DZ.densify(r, sc.degree, params, st, tau_a=0.0, tau_s=1e30)
    assert (action.cpu().numpy() == D.SPLIT).all()
    assert new["opacity"].shape[0] == 4 * sc.num_prims
    camt = torch.from_numpy(cams.cams).to(dev)
    _, s0 = r.forward(sc.degree, params, camt, cams.wh)
    lay = r.layout(sc.degree, params, camt, cams.wh)
    fg0 = s0[lay["I_tri"]:lay["I_tri"] + 4 * cams.num_pixels].view(torch.int32).cpu().numpy() >= 0
    r2 = Renderer(0)
    _, s1 = r2.forward(sc.degree, new, camt, cams.wh)
    lay1 = r2.layout(sc.degree, new, camt, cams.wh)
    fg1 = s1[lay1["I_tri"]:lay1["I_tri"] + 4 * cams.num_pixels].view(torch.int32).cpu().numpy() >= 0
    diff = (fg0 != fg1).mean()
    G.log(f"    foreground pixels differing: {diff:.4%} of {cams.num_pixels}")
    assert fg0.sum() > 1000 and diff < 0.01
