"""Gaussians whose tile range exceeds 3 x 3 tiles ("wide" records).

The backward's sums of a record in a tile go to the record's slot for that
tile, (ty mod 3) 3 + tx mod 3, which is unique only within a 3 x 3 range; a
wide record's sums are added by float atomics into nine floats of its own,
which the generation zeroes and the parameter pass reads and zeroes again.
Lattice Gaussians with log-scales set to twice the lattice spacing (m = 2)
are wide at 8 and 16 px tiles.  Checked here: such records exist, the
gradients match the oracle's, and three backward passes on one forward state
give the same gradients (the read-and-zero leaves nothing behind)."""
import numpy as np
import pytest

import oracle
from paper_2503_13961_amd import scenes as S
from tests import gpu_common as G
from tests.test_gpu_parity import GRAD_TOL, IMG_TOL, _workload

pytestmark = pytest.mark.gpu


def _wide_records(rec, tile):
    """Records whose Gaussian tile range is non-empty and exceeds 3 tiles on
    an axis (ranges: packed int16 pixel bounds in the record's last float4)."""
    r3 = rec[:, 12:14].copy().view(np.int32)
    lo = (r3 & 0xFFFF).astype(np.int16).astype(np.int64)
    hi = r3.astype(np.int64) >> 16
    ok = (lo[:, 0] <= hi[:, 0]) & (lo[:, 1] <= hi[:, 1])
    n = (hi // tile) - (lo // tile) + 1
    return int((ok & ((n[:, 0] > 3) | (n[:, 1] > 3))).sum())


@pytest.mark.parametrize("name,m,tile", [("sphere_small", 2, 8), ("random64", 2, 8), ("sphere_small", 2, 16)])
def test_wide_records_gradients(name, m, tile):
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    G.log(f"[wide_records] workload={name} m={m} tile={tile}")
    sc, cams = _workload(name)
    sc = S.lattice_scaled(sc, m=m, L=4, c=2.0)
    cfg = G.oracle_config(tile=tile, lattice=m)
    img_ref, frames = oracle.render_views(sc, cams, cfg)
    gi = G.l1_cotangent(img_ref, S.l1_target(cams.num_pixels))
    ref = oracle.grad_views(frames, gi)

    dev = torch.device("cuda", 0)
    r = Renderer(0, tile=tile, tess_level=4, bg=(0.0, 0.0, 0.0), lattice=m)
    params = scene_tensors(sc, dev)
    camt = torch.from_numpy(cams.cams).to(dev)
    wh = np.ascontiguousarray(cams.wh, dtype=np.int32)
    images, state = r.forward(sc.degree, params, camt, wh)
    torch.cuda.synchronize()
    status, counters = r.query(state)
    assert status == 0 and counters[0] == 0, counters
    err = np.abs(images.cpu().numpy().astype(np.float64) - img_ref).max()
    G.log(f"    image max abs err {err:.3e}")
    assert err <= IMG_TOL

    lay = r.layout(sc.degree, params, camt, wh)
    nrec = (lay["gkey"] - lay["rec"]) // 64
    rec = state[lay["rec"]:lay["rec"] + 64 * nrec].cpu().numpy().view(np.float32).reshape(nrec, 16)
    nwide = _wide_records(rec, tile)
    G.log(f"    {nwide} wide records of {nrec}")
    assert nwide > 0

    gt = torch.from_numpy(np.ascontiguousarray(gi, dtype=np.float32)).to(dev)
    out = []
    for _ in range(3):
        grads = r.backward(sc.degree, params, camt, wh, images, gt, state)
        torch.cuda.synchronize()
        out.append({k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()})
    G.check_grads(out[0], ref, GRAD_TOL)
    # later passes: the same sums up to the order of the float atomics
    for later in out[1:]:
        for k in out[0]:
            scale = max(np.abs(out[0][k]).max(), 1e-30)
            assert np.abs(later[k] - out[0][k]).max() <= 1e-5 * scale, k
