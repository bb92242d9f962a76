"""The torch front end (autograd Function) and the (tile, batch) autotuner."""
import numpy as np
import pytest

import oracle
from paper_2503_13961_amd import scenes as S
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def test_autograd_function_matches_oracle():
    """loss = mean|render(params) - target| through torch.autograd: the
    parameter .grad tensors equal the oracle's gradient for the same
    cotangent, and a second backward accumulates into them."""
    import torch
    from paper_2503_13961_amd.render import PARAM_NAMES, Renderer, render, scene_tensors
    G.log("[autograd] sphere_small")
    sc, cams, _ = S.workload("sphere_small")
    dev = torch.device("cuda", 0)
    r = Renderer(0)
    params = {k: v.requires_grad_(True) for k, v in scene_tensors(sc, dev).items()}
    camt = torch.from_numpy(cams.cams).to(dev)
    target = torch.from_numpy(S.l1_target(cams.num_pixels)).to(dev)
    img = render(r, sc.degree, params, camt, cams.wh)
    loss = (img - target).abs().mean()
    loss.backward(retain_graph=True)
    torch.cuda.synchronize()
    img_np = img.detach().cpu().numpy().astype(np.float64)
    # the oracle differentiates the same loss with its own image: the two
    # cotangents agree wherever |C - target| exceeds the image error, here
    # everywhere (checked), so both sides differentiate the same function
    img_ref, frames = oracle.render_views(sc, cams, G.oracle_config())
    tgt = S.l1_target(cams.num_pixels).astype(np.float64)
    gi = np.sign(img_ref - tgt) / img_ref.size
    np.testing.assert_array_equal(np.sign(img_np - tgt), np.sign(img_ref - tgt))
    ref = oracle.grad_views(frames, gi)
    first = {k: params[k].grad.detach().cpu().numpy().astype(np.float64) for k in PARAM_NAMES}
    G.check_grads(first, ref, 1e-3)
    loss.backward()
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        again = params[k].grad.detach().cpu().numpy().astype(np.float64)
        # the second pass adds its own gradient (float atomics: same sum up to ordering)
        assert G.grad_error(again - first[k], first[k]) <= 1e-5, k


def test_every_tile_and_batch_variant_agrees():
    """All (tile, batch) kernels give bit-identical images and gradients
    within 1e-5 of each other (float atomics reorder the sums)."""
    from paper_2503_13961_amd.autotune import CANDIDATES
    G.log("[variants] sphere_small")
    sc, cams, _ = S.workload("sphere_small")
    gi = np.sign(np.random.default_rng(3).standard_normal((cams.num_pixels, 3))) / (3 * cams.num_pixels)
    base = G.run_gpu(sc, cams, tile=16, batch=64, grad_images=gi, lean=True)
    for tile, batch in CANDIDATES:
        g = G.run_gpu(sc, cams, tile=tile, batch=batch, grad_images=gi, lean=True)
        np.testing.assert_array_equal(g["images"], base["images"])
        for k in base["grads"]:
            assert G.grad_error(g["grads"][k], base["grads"][k]) <= 1e-5, (tile, batch, k)


def test_autotuner_picks_a_candidate_and_caches_it(tmp_path):
    import torch
    from paper_2503_13961_amd.autotune import CANDIDATES, autotune, tuned_renderer
    from paper_2503_13961_amd.render import scene_tensors
    G.log("[autotune] sphere_small")
    sc, cams, _ = S.workload("sphere_small")
    dev = torch.device("cuda", 0)
    params = scene_tensors(sc, dev)
    camt = torch.from_numpy(cams.cams).to(dev)
    path = str(tmp_path / "tune.json")
    res = autotune(sc.degree, params, camt, cams.wh, cache_path=path, reps=3, warmup=1)
    assert not res["cached"] and (res["tile"], res["batch"]) in CANDIDATES
    assert set(res["timings"]) == {f"{t}x{b}" for t, b in CANDIDATES}
    assert res["ms"] == min(res["timings"].values()) > 0
    again = autotune(sc.degree, params, camt, cams.wh, cache_path=path)
    assert again["cached"] and (again["tile"], again["batch"]) == (res["tile"], res["batch"])
    r, rec = tuned_renderer(sc.degree, params, camt, cams.wh, cache_path=path)
    assert rec["cached"] and (r.cfg.tile, r.cfg.batch) == (res["tile"], res["batch"])
    img, _ = r.forward(sc.degree, params, camt, cams.wh)
    ref = G.run_gpu(sc, cams, lean=True)["images"]
    np.testing.assert_array_equal(img.cpu().numpy().astype(np.float64), ref)
