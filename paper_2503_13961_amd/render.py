"""PyTorch front end: device memory, streams and autograd around libbgt.

PyTorch only supplies memory and the current stream; the forward and
backward passes are the library's HIP kernels (``native``).
"""
from __future__ import annotations

import numpy as np
import torch

from . import native as N

PARAM_NAMES = ("ctrl", "color_ctrl", "log_scale", "quat", "opacity", "sharpness")


def param_names(params) -> tuple:
    """The parameter arrays present: the six of every scene, plus the SH
    coefficients ("sh", [3][K][P]) of a scene with view-dependent colour."""
    return PARAM_NAMES + (("sh",) if params.get("sh") is not None and params["sh"].numel() > 0 else ())


def _grad_ptrs(grads) -> N.bgt_grads:
    return N.make_grads(*(_ptr(grads[k]) for k in PARAM_NAMES), sh=_ptr(grads["sh"]) if "sh" in grads else None)


def _ptr(t: torch.Tensor) -> int:
    assert t.is_contiguous(), "tensor must be contiguous"
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Renderer:
    """One bgt context on one device, plus the pair-capacity retry policy."""

    def __init__(self, device: int = 0, **config):
        self.device_index = int(device)
        self.device = torch.device("cuda", self.device_index)
        self._config = dict(config)
        self.cfg = N.bgt_default_config(**self._config)
        self.ctx = N.bgt_create(self.cfg, self.device_index)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None:
            N.bgt_destroy(ctx)
            self.ctx = None

    # ---------------------------------------------------------------- structs
    @staticmethod
    def prims_struct(degree, params) -> N.bgt_prims:
        P = int(params["opacity"].shape[0])
        T = int(params["log_scale"].shape[1]) if params["log_scale"].dim() == 3 else 1
        R = {1: 1, 6: 3}.get(T, 0)  # attribute-map texels T = R(R+1)/2
        sh = params.get("sh")
        shd = 0
        if sh is not None and sh.numel() > 0:
            shd = {3: 1, 8: 2, 15: 3}.get(int(sh.shape[1]), -1)
        return N.make_prims(degree, P, *(_ptr(params[k]) for k in PARAM_NAMES), attr_res=R, sh_degree=shd,
                            sh=_ptr(sh) if shd > 0 else None)

    @staticmethod
    def views_struct(cams: torch.Tensor, wh: np.ndarray) -> N.bgt_views:
        return N.make_views(wh, _ptr(cams))

    def state_bytes(self, degree, params, cams, wh) -> int:
        return N.bgt_state_size(self.ctx, self.prims_struct(degree, params), self.views_struct(cams, wh))

    def layout(self, degree, params, cams, wh) -> dict:
        return N.bgt_state_layout(self.ctx, self.prims_struct(degree, params), self.views_struct(cams, wh))

    def _grow(self):
        """Double the pair capacities (new context with the same settings)."""
        self._config["pair_factor"] = float(self.cfg.pair_factor) * 2
        self._config["bpair_factor"] = float(self.cfg.bpair_factor) * 2
        old = self.ctx
        self.cfg = N.bgt_default_config(**self._config)
        self.ctx = N.bgt_create(self.cfg, self.device_index)
        N.bgt_destroy(old)

    # ---------------------------------------------------------------- passes
    def forward(self, degree, params, cams, wh, state=None, images=None, check=True):
        """Render all views; returns (images [sum WH][3], state)."""
        wh = np.ascontiguousarray(wh, dtype=np.int32).reshape(-1, 2)
        npx = int((wh[:, 0].astype(np.int64) * wh[:, 1]).sum())
        for _ in range(8):
            nbytes = self.state_bytes(degree, params, cams, wh)
            if state is None or state.numel() < nbytes:
                state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            if images is None:
                images = torch.empty((npx, 3), dtype=torch.float32, device=self.device)
            try:
                N.bgt_render_fwd(self.ctx, self.prims_struct(degree, params), self.views_struct(cams, wh),
                                 _ptr(images), _ptr(state), state.numel(), _stream())
            except N.BgtError as err:  # an earlier unchecked pass on this context overflowed
                if err.status != N.BGT_E_OVERFLOW or not check:
                    raise
                self._grow()
                continue
            if not check:
                return images, state
            st, _ = N.bgt_query(self.ctx, _ptr(state), state.numel(), _stream())
            if st == N.BGT_OK:
                return images, state
            self._grow()
        raise N.BgtError(N.BGT_E_OVERFLOW, "pair capacity still exceeded after 8 doublings")

    def backward(self, degree, params, cams, wh, images, grad_images, state, grads=None):
        wh = np.ascontiguousarray(wh, dtype=np.int32).reshape(-1, 2)
        if grads is None:
            grads = {k: torch.empty_like(params[k]) for k in param_names(params)}
        g = _grad_ptrs(grads)
        N.bgt_render_bwd(self.ctx, self.prims_struct(degree, params), self.views_struct(cams, wh), _ptr(images),
                         _ptr(grad_images), _ptr(state), state.numel(), g, _stream())
        return grads

    def query(self, state):
        return N.bgt_query(self.ctx, _ptr(state), state.numel(), _stream())

    def tessellate(self, degree, params, L=None):
        L = int(self.cfg.tess_level)
        P = int(params["opacity"].shape[0])
        VL = (L + 1) * (L + 2) // 2
        out = torch.empty((3, VL, P), dtype=torch.float32, device=self.device)
        N.bgt_tessellate(self.ctx, self.prims_struct(degree, params), _ptr(out), _stream())
        return out


class RenderFunction(torch.autograd.Function):
    """images = render(BG-Triangle parameters); backward = bgt_render_bwd."""

    @staticmethod
    def forward(ctx, renderer, degree, cams, wh, ctrl, color_ctrl, log_scale, quat, opacity, sharpness, sh=None):
        params = dict(zip(PARAM_NAMES, (ctrl, color_ctrl, log_scale, quat, opacity, sharpness)))
        if sh is not None:
            params["sh"] = sh
        params = {k: v.detach().contiguous() for k, v in params.items()}
        images, state = renderer.forward(degree, params, cams, wh)
        ctx.renderer, ctx.degree, ctx.wh, ctx.state = renderer, degree, wh, state
        ctx.names = param_names(params)
        ctx.save_for_backward(*(params[k] for k in ctx.names), cams, images)
        return images

    @staticmethod
    def backward(ctx, grad_images):
        *ps, cams, images = ctx.saved_tensors
        params = dict(zip(ctx.names, ps))
        grads = ctx.renderer.backward(ctx.degree, params, cams, ctx.wh, images, grad_images.contiguous(), ctx.state)
        return (None, None, None, None) + tuple(grads[k] for k in PARAM_NAMES) + (grads.get("sh"),)


def render(renderer: Renderer, degree: int, params: dict, cams: torch.Tensor, wh) -> torch.Tensor:
    return RenderFunction.apply(renderer, degree, cams, wh, *(params[k] for k in PARAM_NAMES), params.get("sh"))


def scene_tensors(scene, device) -> dict:
    """Upload a scenes.Scene to device tensors (float32, contiguous)."""
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(device)
            for k, v in scene.arrays().items()}
