"""Pair-capacity overflow: reported by the next call on the context without a
device wait, and recovered by the checked training loop when it happens
inside a captured graph."""
import numpy as np
import pytest

import oracle
from paper_2503_13961_amd import scenes as S
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _setup(name="random64"):
    import torch
    from paper_2503_13961_amd.render import scene_tensors
    sc, cams, _ = S.workload(name)
    dev = torch.device("cuda", 0)
    return sc, cams, scene_tensors(sc, dev), torch.from_numpy(cams.cams).to(dev), np.ascontiguousarray(cams.wh, np.int32)


def test_next_call_reports_an_overflow():
    """An unchecked forward pass with far too small capacities records the
    overflow on the device; once the device has run it, the next forward or
    backward call on the context returns BGT_E_OVERFLOW and enqueues nothing;
    the report clears the record, and bgt_query reports the state's own bits."""
    import torch
    from paper_2503_13961_amd import native as N
    from paper_2503_13961_amd.render import Renderer
    G.log("[overflow] next call reports")
    sc, cams, p, ct, wh = _setup()
    r = Renderer(0, pair_factor=0.01, bpair_factor=0.01)
    images, state = r.forward(sc.degree, p, ct, wh, check=False)
    torch.cuda.synchronize()
    with pytest.raises(N.BgtError) as e:
        r.forward(sc.degree, p, ct, wh, state=state, images=images, check=False)
    assert e.value.status == N.BGT_E_OVERFLOW
    # reported once: this call runs (and overflows again)
    images, state = r.forward(sc.degree, p, ct, wh, state=state, images=images, check=False)
    torch.cuda.synchronize()
    gi = torch.zeros_like(images)
    with pytest.raises(N.BgtError) as e:
        r.backward(sc.degree, p, ct, wh, images, gi, state)
    assert e.value.status == N.BGT_E_OVERFLOW
    st, cnt = r.query(state)
    assert st == N.BGT_E_OVERFLOW and cnt[0] & 1
    # a checked forward grows the capacities and renders the oracle's image
    images, state = r.forward(sc.degree, p, ct, wh, check=True)
    st, cnt = r.query(state)
    assert st == N.BGT_OK and cnt[0] == 0
    fr = G.oracle_frames(sc, cams, G.oracle_config())[0]
    assert np.abs(images.cpu().numpy() - fr.render()[0]).max() <= 1e-4


def test_training_loop_recovers_from_overflow():
    """A captured training loop (forward, Eq. 9, backward, Adam) whose
    Gaussians grow while it runs (a blurrier target and a large log-scale
    learning rate), started with pair capacities that only just hold the
    initial scene: the loop's check finds the overflow, rolls back to its
    previous check, grows the capacities, captures again and repeats the
    steps.  The result matches the same loop run with ample capacity."""
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    from paper_2503_13961_amd.train import DEFAULT_LR, TrainStep
    G.log("[overflow] captured training loop")
    sc, cams, p, ct, wh = _setup()
    dev = torch.device("cuda", 0)
    blur = sc.copy()
    blur.log_scale = (blur.log_scale + np.float32(1.0)).astype(np.float32)
    tgt, _ = oracle.render_views(blur, cams, G.oracle_config())
    targets = torch.from_numpy(tgt.astype(np.float32)).to(dev)
    lr = dict(DEFAULT_LR, log_scale=0.05)
    steps = 12

    def loop(renderer, check_every):
        params = scene_tensors(sc, dev)
        ts = TrainStep(renderer, sc.degree, params, ct, wh, targets, lr=lr)
        res = ts.run(steps, check_every=check_every)
        return res, {k: v.cpu().numpy().astype(np.float64) for k, v in params.items()}, renderer

    ref_res, ref, _ = loop(Renderer(0, pair_factor=32.0), 4)
    assert ref_res == {"steps": steps, "recoveries": 0, "checks": 3}
    # capacities that just hold the initial scene: cap = pair_factor * records + 1024
    probe = Renderer(0, pair_factor=32.0)
    _, state = probe.forward(sc.degree, p, ct, wh)
    pairs = probe.query(state)[1][1]
    nrec = cams.num_pixels
    pf = (pairs - 1024) * 1.02 / nrec
    G.log(f"    initial Gaussian pairs {pairs}, pair_factor {pf:.3f}")
    res, got, r = loop(Renderer(0, pair_factor=pf), 3)
    G.log(f"    {res}, final pair_factor {r.cfg.pair_factor:.3f}")
    assert res["steps"] == steps and res["recoveries"] >= 1
    # the checked loop's trajectory is the ample-capacity one (up to the
    # float atomics' summation order)
    for k in ref:
        moved = np.abs(ref[k] - sc.arrays()[k]).max()
        err = np.abs(got[k] - ref[k]).max()
        G.log(f"    {k}: max |got - ref| {err:.2e} (largest change from the start {moved:.2e})")
        assert err <= 1e-3 * max(moved, 1e-6), k
