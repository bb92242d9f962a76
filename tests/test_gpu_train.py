"""The training step's kernels (Eq. 9 loss with its image gradient, Adam)
through the C ABI against the FP64 oracle in oracle/train.py.

Tolerances: the loss pass sums its window moments in FP64 from the same
float inputs the oracle reads, so the loss differs by the final float
rounding (1e-6 relative is ample); the per-pixel derivative maps are stored
as float between the two window passes, so the image gradient carries about
1e-7 relative error per term: 1e-5 of its largest entry.  Adam runs in FP64
on float storage: parameters within 2 float ulps of the oracle's.
"""
import numpy as np
import pytest

from oracle import train as OT
from paper_2503_13961_amd import scenes as S
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _loss_case(wh, seed):
    rng = np.random.default_rng(seed)
    n = int(sum(w * h for w, h in wh))
    x = rng.random((n, 3)).astype(np.float32)
    y = rng.random((n, 3)).astype(np.float32)
    # smooth regions too, where sigma_xy is near 0 and SSIM is most sensitive
    x[: n // 4] = 0.5
    y[: n // 8] = 0.5
    return x, y


@pytest.mark.parametrize("wh", [[(37, 29), (64, 48), (5, 3), (1, 1)], [(800, 800), (33, 17)]])
def test_loss_and_image_gradient_match_oracle(wh):
    import torch
    from paper_2503_13961_amd.render import Renderer
    from paper_2503_13961_amd.train import PhotometricLoss
    G.log(f"[loss] views {wh}")
    x, y = _loss_case(wh, 3)
    dev = torch.device("cuda", 0)
    op = PhotometricLoss(Renderer(0), np.array(wh, np.int32))
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    loss, grad = op(xt, yt)
    torch.cuda.synchronize()
    loss, grad = loss.cpu().numpy().astype(np.float64), grad.cpu().numpy().astype(np.float64)
    L, l2, ssim = OT.loss(x, y, wh)
    G.log(f"    L {loss[0]:.8f} vs {L:.8f}; L2 {loss[1]:.8f} vs {l2:.8f}; SSIM {loss[2]:.8f} vs {ssim:.8f}")
    for got, ref in zip(loss, (L, l2, ssim)):
        assert abs(got - ref) <= 1e-6 * abs(ref) + 1e-9
    ref = OT.loss_grad(x, y, wh)
    err = np.abs(grad - ref).max() / np.abs(ref).max()
    G.log(f"    image gradient max err / max|ref| = {err:.2e}")
    assert err <= 1e-5


def test_loss_without_gradient_and_lambda_ends():
    """lambda = 0 gives the mean squared error alone; lambda = 1 only
    D-SSIM; a NULL gradient pointer computes the loss alone."""
    import torch
    from paper_2503_13961_amd.render import Renderer
    from paper_2503_13961_amd.train import PhotometricLoss
    wh = [(40, 30)]
    x, y = _loss_case(wh, 4)
    dev = torch.device("cuda", 0)
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    for lam in (0.0, 1.0):
        op = PhotometricLoss(Renderer(0), np.array(wh, np.int32), lam=lam)
        loss, grad = op(xt, yt, want_grad=False)
        assert grad is None
        L = OT.loss(x, y, wh, lam=lam)[0]
        assert abs(float(loss[0].cpu()) - L) <= 1e-6 * abs(L)


def test_adam_two_steps_match_oracle():
    """Two updates of three groups (sizes 1000, 7 and 0) through the device
    step counter: t = 1 then t = 2, moments stored as float between them."""
    import torch
    from paper_2503_13961_amd import native as N
    from paper_2503_13961_amd.render import Renderer
    G.log("[adam] three groups, two steps")
    r = Renderer(0)
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(5)
    sizes, lrs = (1000, 7, 0), (1e-3, 5e-2, 1.0)
    p = [rng.normal(size=n).astype(np.float32) for n in sizes]
    m = [np.zeros(n, np.float32) for n in sizes]
    v = [np.zeros(n, np.float32) for n in sizes]
    P = [torch.from_numpy(a.copy()).to(dev) for a in p]
    Mt = [torch.zeros(n, device=dev) for n in sizes]
    Vt = [torch.zeros(n, device=dev) for n in sizes]
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    b1, b2, eps = np.float32(0.9), np.float32(0.999), np.float32(1e-8)
    for t in (1, 2):
        g = [rng.normal(size=n).astype(np.float32) * 10 ** rng.uniform(-6, 1, size=n).astype(np.float32)
             for n in sizes]
        Gt = [torch.from_numpy(a).to(dev) for a in g]
        groups = [N.bgt_adam_group(P[i].data_ptr(), Gt[i].data_ptr(), Mt[i].data_ptr(), Vt[i].data_ptr(), sizes[i],
                                   lrs[i], 0) for i in range(3)]
        N.bgt_adam_step(r.ctx, groups, float(b1), float(b2), float(eps), step.data_ptr(), 0)
        torch.cuda.synchronize()
        for i in range(3):
            pn, mn, vn = OT.adam_step(p[i], g[i], m[i], v[i], t, np.float32(lrs[i]), float(b1), float(b2), float(eps))
            p[i], m[i], v[i] = pn.astype(np.float32), mn.astype(np.float32), vn.astype(np.float32)
            got = P[i].cpu().numpy()
            ulp = np.spacing(np.abs(p[i]).astype(np.float32))
            assert (np.abs(got.astype(np.float64) - pn) <= 2 * ulp).all(), (t, i)
            assert (np.abs(Mt[i].cpu().numpy() - m[i]) <= np.spacing(np.abs(m[i]))).all()
    assert int(step.cpu()) == 2


def test_train_step_in_a_graph_matches_eager_and_lowers_the_loss():
    """Forward, Eq. 9, backward and Adam captured in one graph: each replay
    takes one optimisation step (the device step counter advances).  The
    replays' losses follow an eager run of the same steps from the same
    parameters (the backward's float atomics sum in no fixed order: 1e-3),
    and the loss of a recoloured scene against renders of the original
    falls."""
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    from paper_2503_13961_amd.train import TrainStep
    G.log("[train] sphere_small, eager steps vs graph replays")
    sc, cams, _ = S.workload("sphere_small")
    dev = torch.device("cuda", 0)
    camt = torch.from_numpy(cams.cams).to(dev)
    target, _ = Renderer(0).forward(sc.degree, scene_tensors(sc, dev), camt, cams.wh)
    target = target.clone()
    pert = sc.copy()
    rng = np.random.default_rng(0)
    pert.color_ctrl[:] = np.clip(pert.color_ctrl + rng.normal(0, 0.1, pert.color_ctrl.shape), 0, 1)
    lr = {"ctrl": 0.0, "color_ctrl": 1e-2, "log_scale": 0.0, "quat": 0.0, "opacity": 0.0, "sharpness": 0.0}
    n = 12
    eager = TrainStep(Renderer(0), sc.degree, scene_tensors(pert, dev), camt, cams.wh, target, lr=lr)
    ref = []
    for _ in range(n):
        ref.append(float(eager()[0].cpu()))
    step = TrainStep(Renderer(0), sc.degree, scene_tensors(pert, dev), camt, cams.wh, target, lr=lr)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        got = [float(step()[0].cpu())]   # eager first step, then capture the next
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            loss = step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for _ in range(n - 1):
        g.replay()
        torch.cuda.synchronize()
        got.append(float(loss[0].cpu()))
        _ = torch.ones(16, device=dev).sum().item()   # eager work between replays
    G.log(f"    eager {ref[0]:.6f} .. {ref[-1]:.6f}; replays {got[0]:.6f} .. {got[-1]:.6f}")
    assert int(step.opt.step_count.cpu()) == n
    for a, b in zip(ref, got):
        assert abs(a - b) <= 1e-3 * a, (ref, got)
    assert ref[-1] < 0.8 * ref[0]


def test_l1_cotangent_is_exact():
    """sign(C - target) * scale, 0 on ties, over a length that is not a
    multiple of 4 and from an offset slice: bit-exact."""
    import torch
    from paper_2503_13961_amd import native as N
    from paper_2503_13961_amd.render import Renderer
    rng = np.random.default_rng(9)
    n = 3 * 1001
    x = rng.random(n + 5).astype(np.float32)
    y = rng.random(n + 5).astype(np.float32)
    y[::7] = x[::7]                                      # exact ties
    dev = torch.device("cuda", 0)
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    g = torch.full((n + 5,), 7.0, device=dev)
    r = Renderer(0)
    scale = np.float32(1.0 / n)
    N.bgt_l1_cotangent(r.ctx, n, xt[3:].data_ptr(), yt[3:].data_ptr(), float(scale), g[3:].data_ptr(), 0)
    got = g.cpu().numpy()
    want = np.sign(x[3:3 + n] - y[3:3 + n]).astype(np.float32) * scale
    np.testing.assert_array_equal(got[3:3 + n], want)
    assert (got[:3] == 7.0).all() and (got[3 + n:] == 7.0).all()


def test_train_step_with_attribute_maps_and_sh():
    """A scene with resolution-3 maps and SH colour: Adam takes seven groups
    (the SH coefficients too), the step counter advances and the loss of a
    recoloured scene against renders of the original falls."""
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    from paper_2503_13961_amd.train import TrainStep
    G.log("[train] sphere_small with resolution-3 maps and SH degree 3")
    sc, cams, _ = S.workload("sphere_small")
    sc = S.with_attributes(sc, attr_res=3, sh_degree=3, seed=1)
    dev = torch.device("cuda", 0)
    camt = torch.from_numpy(cams.cams).to(dev)
    target, _ = Renderer(0).forward(sc.degree, scene_tensors(sc, dev), camt, cams.wh)
    target = target.clone()
    pert = sc.copy()
    pert.sh = (pert.sh + np.random.default_rng(0).normal(0, 0.05, pert.sh.shape)).astype(np.float32)
    params = scene_tensors(pert, dev)
    sh0 = params["sh"].clone()
    lr = {"ctrl": 0.0, "color_ctrl": 0.0, "log_scale": 0.0, "quat": 0.0, "opacity": 0.0, "sharpness": 0.0,
          "sh": 2e-3}
    step = TrainStep(Renderer(0), sc.degree, params, camt, cams.wh, target, lr=lr)
    assert len(step.opt.names) == 7
    losses = [float(step()[0].cpu()) for _ in range(8)]
    G.log(f"    loss {losses[0]:.6f} .. {losses[-1]:.6f}")
    assert int(step.opt.step_count.cpu()) == 8
    assert losses[-1] < losses[0]
    assert (params["sh"] - sh0).abs().max() > 0
