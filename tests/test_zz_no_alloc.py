"""bgt_loss_noalloc (the loss pass with the library's static workspace)
against bgt_loss with a caller-allocated workspace, through the C ABI: two
calls in a row, the second with smaller views, and the size limit."""
import numpy as np
import pytest

from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _case(wh, seed):
    rng = np.random.default_rng(seed)
    n = int(sum(w * h for w, h in wh))
    x = rng.random((n, 3)).astype(np.float32)
    y = rng.random((n, 3)).astype(np.float32)
    x[: n // 5] = 0.5   # flat regions, where SSIM is most sensitive
    return x, y


def test_noalloc_loss_matches_workspace_loss_on_two_calls():
    import torch
    from paper_2503_13961_amd import native as N
    from paper_2503_13961_amd.render import Renderer
    r = Renderer(0)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream().cuda_stream
    for wh, lam, seed in (([(800, 800), (33, 17), (5, 3)], 0.2, 1), ([(64, 48), (1, 1)], 0.7, 2)):
        G.log(f"[noalloc] views {wh} lambda {lam}")
        wh = np.array(wh, np.int32)
        views = N.make_views(wh, None)
        x, y = _case(wh, seed)
        xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
        ws = torch.empty(N.bgt_loss_workspace_size(views), dtype=torch.uint8, device=dev)
        loss_a, grad_a = torch.empty(3, device=dev), torch.empty_like(xt)
        loss_b, grad_b = torch.full((3,), -1.0, device=dev), torch.full_like(xt, -1.0)
        N.bgt_loss(r.ctx, views, xt.data_ptr(), yt.data_ptr(), lam, loss_a.data_ptr(), grad_a.data_ptr(),
                   ws.data_ptr(), ws.numel(), stream)
        N.bgt_loss_noalloc(r.ctx, views, xt.data_ptr(), yt.data_ptr(), lam, loss_b.data_ptr(), grad_b.data_ptr(),
                           stream)
        torch.cuda.synchronize()
        # the same kernels on the same inputs: identical bits
        np.testing.assert_array_equal(loss_b.cpu().numpy(), loss_a.cpu().numpy())
        np.testing.assert_array_equal(grad_b.cpu().numpy(), grad_a.cpu().numpy())
        G.log(f"    loss {loss_b.cpu().numpy()}")


def test_noalloc_loss_rejects_views_beyond_its_workspace():
    import torch
    from paper_2503_13961_amd import native as N
    from paper_2503_13961_amd.render import Renderer
    G.log("[noalloc] size limit")
    r = Renderer(0)
    wh = np.array([(2048, 2048)], np.int32)            # 151 MB of maps > 64 MiB
    views = N.make_views(wh, None)
    assert N.bgt_loss_workspace_size(views) > 64 << 20
    dev = torch.device("cuda", 0)
    x = torch.zeros((2048 * 2048, 3), device=dev)
    loss = torch.full((3,), -1.0, device=dev)
    with pytest.raises(N.BgtError) as e:
        N.bgt_loss_noalloc(r.ctx, views, x.data_ptr(), x.data_ptr(), 0.2, loss.data_ptr(), None,
                           torch.cuda.current_stream().cuda_stream)
    assert e.value.status == N.BGT_E_NOMEM
    assert "static workspace" in N.bgt_last_error(r.ctx)
    torch.cuda.synchronize()
    assert (loss.cpu().numpy() == -1.0).all()          # nothing was enqueued
