"""Backward passes repeated on one forward pass's state.

The blend backward stores each tile-list entry's sums in its record's slot
for the tile, for the tile's replayed prefix only (the entries up to the
largest stop index of the tile's pixels with a non-zero cotangent); the sort
writes each entry's list position to the same slot, and the parameter pass
takes a slot's sums only when that position lies in the tile's prefix.  A
second backward with a cotangent that vanishes on the pixels that composite
deepest shortens those prefixes, so sums the first pass wrote past them are
still in the state: the second pass's gradients must be those of its own
cotangent, against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2503_13961_amd import scenes as S
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,tile", [("random64", 8), ("random64", 16), ("sphere_small", 16)])
def test_second_backward_on_one_state(name, tile):
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log(f"[backward_reuse] workload={name} tile={tile}")
    sc, cams, _ = S.workload(name)
    dev = torch.device("cuda", 0)
    r = Renderer(0, tile=tile, tess_level=4, bg=(0.0, 0.0, 0.0))
    params = scene_tensors(sc, dev)
    camt = torch.from_numpy(cams.cams).to(dev)
    wh = np.ascontiguousarray(cams.wh, dtype=np.int32)
    images, state = r.forward(sc.degree, params, camt, wh)
    torch.cuda.synchronize()
    status, counters = r.query(state)
    assert status == 0 and counters[0] == 0, counters
    lay = r.layout(sc.degree, params, camt, wh)
    N = cams.num_pixels
    last = state[lay["last"]:lay["last"] + 4 * N].cpu().numpy().view(np.int32)

    cfg = G.oracle_config(tile=tile)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    target = S.l1_target(N)
    g1 = G.l1_cotangent(img_ref, target)
    # the second cotangent keeps only the pixels that stop early in their lists
    keep = last <= np.quantile(last[last > 0], 0.4)
    g2 = g1 * keep[:, None]
    # tiles whose replayed prefix the second cotangent shortens
    po, shorter = G.view_offsets(cams), 0
    for v in range(cams.n_views):
        W, H = (int(x) for x in cams.wh[v])
        tid = ((np.arange(W * H) // W) // tile) * ((W + tile - 1) // tile) + (np.arange(W * H) % W) // tile
        lv, kv = last[po[v]:po[v + 1]], keep[po[v]:po[v + 1]]
        n1 = np.zeros(tid.max() + 1, np.int64)
        n2 = np.zeros_like(n1)
        np.maximum.at(n1, tid, lv)
        np.maximum.at(n2, tid, np.where(kv, lv, 0))
        shorter += int((n2 < n1).sum())
    G.log(f"    {shorter} tiles replay a shorter prefix in the second pass")
    assert shorter > 0

    out = []
    for gi in (g1, g2, g1):
        gt = torch.from_numpy(np.ascontiguousarray(gi, dtype=np.float32)).to(dev)
        grads = r.backward(sc.degree, params, camt, wh, images, gt, state)
        torch.cuda.synchronize()
        out.append({k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()})
    ref1, ref2 = oracle.grad_views(frames, g1), oracle.grad_views(frames, g2)
    G.log("    first pass (full cotangent)")
    G.check_grads(out[0], ref1)
    G.log("    second pass (cotangent on the early-stopping pixels only)")
    G.check_grads(out[1], ref2)
    # the two cotangents' gradients differ: the check above can tell them apart
    assert any(G.grad_error(ref1[k], ref2[k]) > 0.1 for k in ref2)
    G.log("    third pass (full cotangent again)")
    G.check_grads(out[2], ref1)
