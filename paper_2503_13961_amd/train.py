"""One training step around the renderer (Sec. 3.3) on the C ABI: the
photometric loss of Eq. 9 (bgt_loss) and the Adam update (bgt_adam_step).
PyTorch only holds the device memory and supplies the stream."""
from __future__ import annotations

import numpy as np
import torch

from . import native as N
from .render import Renderer, _ptr, _stream, param_names

LAMBDA = 0.2  # weight of the D-SSIM term in Eq. 9

# The paper gives no learning rates.  Defaults: the 3DGS framework's own for
# positions, colour, log-scales and rotations; opacity here is the value
# itself rather than a logit, so it takes the colour rate, and the boundary
# sharpness the rotation rate; SH coefficients take the colour rate over 20,
# the 3DGS ratio between its higher SH bands and their DC term.
DEFAULT_LR = {"ctrl": 1.6e-4, "color_ctrl": 2.5e-3, "log_scale": 5e-3, "quat": 1e-3, "opacity": 2.5e-3,
              "sharpness": 1e-3, "sh": 2.5e-3 / 20}


class PhotometricLoss:
    """Eq. 9 over packed images [sum W H][3]: returns (loss[3] = (L, L2, SSIM),
    dL/dC).  Owns the workspace for one set of view sizes."""

    def __init__(self, renderer: Renderer, wh, lam: float = LAMBDA):
        self.renderer = renderer
        self.wh = np.ascontiguousarray(wh, dtype=np.int32).reshape(-1, 2)
        self.lam = float(lam)
        self.views = N.make_views(self.wh, None)
        nbytes = N.bgt_loss_workspace_size(self.views)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=renderer.device)
        self.loss = torch.empty(3, dtype=torch.float32, device=renderer.device)

    def __call__(self, images: torch.Tensor, targets: torch.Tensor, grad_images: torch.Tensor | None = None,
                 want_grad: bool = True):
        if want_grad and grad_images is None:
            grad_images = torch.empty_like(images)
        N.bgt_loss(self.renderer.ctx, self.views, _ptr(images), _ptr(targets), self.lam, _ptr(self.loss),
                   _ptr(grad_images) if want_grad else None, _ptr(self.workspace), self.workspace.numel(), _stream())
        return self.loss, grad_images


class LossFunction(torch.autograd.Function):
    """L = Eq. 9 (a 0-d tensor); backward scales dL/dC by the incoming
    gradient."""

    @staticmethod
    def forward(ctx, loss_op: PhotometricLoss, images, targets):
        loss, grad = loss_op(images.detach().contiguous(), targets.detach().contiguous())
        ctx.save_for_backward(grad.clone())
        return loss[0].clone()

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return None, grad * g, None


class Adam:
    """Adam over the six parameter tensors with one learning rate each
    (bgt_adam_step).  The step counter lives on the device, so a captured
    graph replays the bias correction correctly."""

    def __init__(self, renderer: Renderer, params: dict, lr: dict | None = None, betas=(0.9, 0.999),
                 eps: float = 1e-15):
        self.renderer = renderer
        self.params = params
        self.lr = dict(DEFAULT_LR if lr is None else lr)
        self.betas = (float(betas[0]), float(betas[1]))
        self.eps = float(eps)
        self.names = param_names(params)
        self.m = {k: torch.zeros_like(params[k]) for k in self.names}
        self.v = {k: torch.zeros_like(params[k]) for k in self.names}
        self.step_count = torch.zeros(1, dtype=torch.int32, device=renderer.device)

    def step(self, grads: dict):
        groups = [N.bgt_adam_group(_ptr(self.params[k]), _ptr(grads[k]), _ptr(self.m[k]), _ptr(self.v[k]),
                                   self.params[k].numel(), self.lr[k], 0) for k in self.names]
        N.bgt_adam_step(self.renderer.ctx, groups, self.betas[0], self.betas[1], self.eps, _ptr(self.step_count),
                        _stream())


class TrainStep:
    """Forward of all views, Eq. 9 against the targets, backward, Adam: one
    optimisation iteration of Sec. 3.3, every stage in the library's kernels
    (capturable in one graph once the state is sized)."""

    def __init__(self, renderer: Renderer, degree: int, params: dict, cams: torch.Tensor, wh, targets: torch.Tensor,
                 lr: dict | None = None, lam: float = LAMBDA):
        self.r, self.degree, self.params, self.cams = renderer, degree, params, cams
        self.wh = np.ascontiguousarray(wh, dtype=np.int32).reshape(-1, 2)
        self.targets = targets
        self.loss_op = PhotometricLoss(renderer, self.wh, lam)
        self.opt = Adam(renderer, params, lr)
        self.images, self.state = renderer.forward(degree, params, cams, self.wh)
        self.grad_images = torch.empty_like(self.images)
        self.grads = {k: torch.empty_like(params[k]) for k in param_names(params)}

    def __call__(self):
        self.r.forward(self.degree, self.params, self.cams, self.wh, state=self.state, images=self.images,
                       check=False)
        loss, _ = self.loss_op(self.images, self.targets, self.grad_images)
        self.r.backward(self.degree, self.params, self.cams, self.wh, self.images, self.grad_images, self.state,
                        self.grads)
        self.opt.step(self.grads)
        return loss

    # ------------------------------------------------ a checked training loop

    def _snapshot(self):
        """Device copies of everything a step changes: parameters, Adam moments, step count."""
        names = self.opt.names
        return ({k: self.params[k].clone() for k in names}, {k: self.opt.m[k].clone() for k in names},
                {k: self.opt.v[k].clone() for k in names}, self.opt.step_count.clone())

    def _restore(self, snap):
        p, m, v, t = snap
        for k in self.opt.names:
            self.params[k].copy_(p[k])
            self.opt.m[k].copy_(m[k])
            self.opt.v[k].copy_(v[k])
        self.opt.step_count.copy_(t)

    def _capture(self):
        self()  # warm-up outside the capture (first launches load the kernels)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self()
        torch.cuda.synchronize()
        return g

    def run(self, steps: int, check_every: int = 8, graph: bool = True) -> dict:
        """Take `steps` optimisation steps (replayed from one captured graph,
        or eagerly) and check for a pair-capacity overflow every `check_every`
        steps.  The pair lists are sized when the loop starts; as training
        moves the patches (larger Gaussians reach more tiles) a forward pass
        can need more, and its lists are then cut short.  The library records
        that on the device (a sticky flag in pinned memory that bgt_query
        reads), so at each check, after the group of steps: if any of them
        overflowed, the parameters, moments and step count go back to their
        values at the previous check, the capacities double, the state is
        resized, the graph is captured again and the group is taken again.
        Returns {"steps", "recoveries", "checks"}."""
        snap = self._snapshot()
        g = self._capture() if graph else None
        if g is not None:
            self._restore(snap)  # the warm-up and the captured launch both stepped
        done = recoveries = checks = 0
        while done < steps:
            n = min(check_every, steps - done)
            for _ in range(n):
                if g is not None:
                    g.replay()
                else:
                    self()
            st, _ = self.r.query(self.state)  # syncs; includes every pass since the last check
            checks += 1
            if st == N.BGT_OK:
                done += n
                snap = self._snapshot()
                continue
            recoveries += 1
            self._restore(snap)
            g = None  # the captured kernels hold the old context's capacities
            self.r._grow()
            self.images, self.state = self.r.forward(self.degree, self.params, self.cams, self.wh)
            self.grad_images = torch.empty_like(self.images)
            if graph:
                g = self._capture()
                self._restore(snap)
        torch.cuda.synchronize()
        return {"steps": done, "recoveries": recoveries, "checks": checks}
