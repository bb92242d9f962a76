"""Splitting and pruning (Sec. 3.3) on the C ABI: per-patch statistics
gathered while training, the per-patch decision, and the rebuilt parameter
arrays.  PyTorch holds the device memory."""
from __future__ import annotations

import torch

from . import native as N
from .render import Renderer, _grad_ptrs, _ptr, _stream, param_names


class PrimStats:
    """Device accumulators of P patches (bgt_prim_stats), zero at creation."""

    FIELDS = (("views_seen", torch.int32, 1), ("vis_views", torch.int32, None), ("tex", torch.int64, None),
              ("view_bits", torch.int64, None), ("grad_sum", torch.float32, None), ("grad_cnt", torch.int32, None),
              ("edge_sum", torch.float32, None), ("edge_cnt", torch.int32, None))

    def __init__(self, num_prims: int, device):
        self.P = int(num_prims)
        self.t = {name: torch.zeros(n or self.P, dtype=dt, device=device) for name, dt, n in self.FIELDS}

    def clear(self):
        for v in self.t.values():
            v.zero_()

    def struct(self) -> N.bgt_prim_stats:
        return N.bgt_prim_stats(*(_ptr(self.t[name]) for name, _, _ in self.FIELDS))

    def accumulate(self, renderer: Renderer, degree, params, cams, wh, state, targets=None, grads=None):
        """One rendered batch: `state` from renderer.forward of the same
        params and views, `targets` the training images, `grads` the
        backward pass's output (dict), either may be None."""
        g = None if grads is None else _grad_ptrs(grads)
        N.bgt_stats_accumulate(renderer.ctx, renderer.prims_struct(degree, params), renderer.views_struct(cams, wh),
                               _ptr(state), state.numel(), None if targets is None else _ptr(targets), g,
                               self.struct(), _stream())


def plan(renderer: Renderer, degree, params, stats: PrimStats, **thresholds):
    """(action[P], dst_index[P], count) on the device; count synchronizes."""
    dev = renderer.device
    action = torch.empty(stats.P, dtype=torch.int32, device=dev)
    dst = torch.empty(stats.P, dtype=torch.int32, device=dev)
    count = torch.empty(1, dtype=torch.int32, device=dev)
    N.bgt_densify_plan(renderer.ctx, renderer.prims_struct(degree, params), stats.struct(),
                       N.bgt_default_densify_config(**thresholds), _ptr(action), _ptr(dst), _ptr(count), _stream())
    return action, dst, int(count.item())


def apply(renderer: Renderer, degree, params, action, dst_index, count) -> dict:
    """The rebuilt parameter tensors (count patches)."""
    out = {}
    for k in param_names(params):
        shape = list(params[k].shape)
        shape[-1] = count
        out[k] = torch.empty(shape, dtype=torch.float32, device=renderer.device)
    N.bgt_densify_apply(renderer.ctx, renderer.prims_struct(degree, params), _ptr(action), _ptr(dst_index), count,
                        _grad_ptrs(out), _stream())
    return out


def densify(renderer: Renderer, degree, params, stats: PrimStats, **thresholds):
    """Plan and apply: returns (new params, action)."""
    action, dst, count = plan(renderer, degree, params, stats, **thresholds)
    return apply(renderer, degree, params, action, dst, count), action
