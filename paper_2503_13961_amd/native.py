"""ctypes binding of libbgt.so: the C ABI declared in include/bgt.h.

Argument marshalling only; every step of the rendering runs in the HIP
kernels of the library.  Importing this module fails loudly when the
library has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbgt.so")

BGT_OK, BGT_E_INVALID, BGT_E_NOMEM, BGT_E_OVERFLOW, BGT_E_HIP, BGT_E_UNSUPPORTED = range(6)
BGT_MAX_VIEWS = 64
BGT_FLAG_NO_BOUNDARY = 1  # bgt_config.flags: the variant without blending coefficients (w = 1)
BGT_STATE_FIELDS = 29
STATE_FIELD_NAMES = ["counters", "zbuf", "I_tri", "I_uv", "pflags", "rec", "gkey", "T_final", "last",
                     "verts", "g_count", "g_start", "g_cursor", "b_count", "b_start", "b_cursor",
                     "g_keys", "g_list", "b_keys", "b_list", "gslot", "gpos", "t_end", "gwide", "dbound", "brec64",
                     "big_tris", "scan", "end"]
EXPORTS = ["bgt_default_config", "bgt_validate_config", "bgt_validate_prims", "bgt_validate_views",
           "bgt_create", "bgt_destroy", "bgt_last_error", "bgt_tessellate", "bgt_state_size",
           "bgt_state_layout", "bgt_render_fwd", "bgt_render_bwd", "bgt_query", "bgt_profile",
           "bgt_stage_times", "bgt_loss_workspace_size", "bgt_loss", "bgt_loss_noalloc", "bgt_l1_cotangent",
           "bgt_adam_step",
           "bgt_default_densify_config", "bgt_stats_accumulate", "bgt_densify_plan", "bgt_densify_apply"]
BGT_NUM_STAGES = 6
STAGE_NAMES = ["raster", "generation", "binning", "blend_fwd", "blend_bwd", "param_bwd"]


class BgtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"bgt status {status}: {msg}")
        self.status = status


class bgt_prims(C.Structure):
    _fields_ = [("degree", C.c_int32), ("num_prims", C.c_int32), ("attr_res", C.c_int32),
                ("sh_degree", C.c_int32), ("ctrl", C.c_void_p), ("color_ctrl", C.c_void_p),
                ("log_scale", C.c_void_p), ("quat", C.c_void_p), ("opacity", C.c_void_p),
                ("sharpness", C.c_void_p), ("sh", C.c_void_p)]


class bgt_grads(C.Structure):
    _fields_ = [("ctrl", C.c_void_p), ("color_ctrl", C.c_void_p), ("log_scale", C.c_void_p),
                ("quat", C.c_void_p), ("opacity", C.c_void_p), ("sharpness", C.c_void_p),
                ("sh", C.c_void_p)]


class bgt_views(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("reserved", C.c_int32), ("wh", C.POINTER(C.c_int32)),
                ("cams", C.c_void_p)]


class bgt_config(C.Structure):
    _fields_ = [("tess_level", C.c_int32), ("tile", C.c_int32), ("batch", C.c_int32),
                ("flags", C.c_int32), ("z_near", C.c_float), ("g_min", C.c_float),
                ("t_min", C.c_float), ("alpha_max", C.c_float), ("dilation", C.c_float),
                ("r_ref", C.c_float), ("bg", C.c_float * 3), ("pair_factor", C.c_float),
                ("bpair_factor", C.c_float), ("lattice", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["bg"] = tuple(self.bg)
        return d


class bgt_adam_group(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("lr", C.c_float), ("reserved", C.c_int32)]


BGT_MAX_ADAM_GROUPS = 8


class bgt_prim_stats(C.Structure):
    _fields_ = [("views_seen", C.c_void_p), ("vis_views", C.c_void_p), ("tex", C.c_void_p),
                ("view_bits", C.c_void_p), ("grad_sum", C.c_void_p), ("grad_cnt", C.c_void_p),
                ("edge_sum", C.c_void_p), ("edge_cnt", C.c_void_p)]


class bgt_densify_config(C.Structure):
    _fields_ = [("tau_g", C.c_float), ("tau_b", C.c_float), ("tau_v", C.c_float), ("tau_r", C.c_float),
                ("tau_a", C.c_float), ("tau_s", C.c_float)]

_lib = None


def lib():
    """Load libbgt.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
        L.bgt_default_config.argtypes = [C.POINTER(bgt_config)]
        L.bgt_default_config.restype = None
        L.bgt_validate_config.argtypes = [C.POINTER(bgt_config)]
        L.bgt_validate_prims.argtypes = [C.POINTER(bgt_prims), C.POINTER(bgt_config)]
        L.bgt_validate_views.argtypes = [C.POINTER(bgt_views)]
        L.bgt_create.argtypes = [C.POINTER(bgt_config), C.c_int, C.POINTER(vp)]
        L.bgt_destroy.argtypes = [vp]
        L.bgt_destroy.restype = None
        L.bgt_last_error.argtypes = [vp]
        L.bgt_last_error.restype = C.c_char_p
        L.bgt_tessellate.argtypes = [vp, C.POINTER(bgt_prims), vp, vp]
        L.bgt_state_size.argtypes = [vp, C.POINTER(bgt_prims), C.POINTER(bgt_views), C.POINTER(C.c_size_t)]
        L.bgt_state_layout.argtypes = [vp, C.POINTER(bgt_prims), C.POINTER(bgt_views), i64p]
        L.bgt_render_fwd.argtypes = [vp, C.POINTER(bgt_prims), C.POINTER(bgt_views), vp, vp, C.c_size_t, vp]
        L.bgt_render_bwd.argtypes = [vp, C.POINTER(bgt_prims), C.POINTER(bgt_views), vp, vp, vp, C.c_size_t,
                                     C.POINTER(bgt_grads), vp]
        L.bgt_query.argtypes = [vp, vp, C.c_size_t, i64p, vp]
        L.bgt_loss_workspace_size.argtypes = [C.POINTER(bgt_views), C.POINTER(C.c_size_t)]
        L.bgt_loss.argtypes = [vp, C.POINTER(bgt_views), vp, vp, C.c_float, vp, vp, vp, C.c_size_t, vp]
        L.bgt_loss_noalloc.argtypes = [vp, C.POINTER(bgt_views), vp, vp, C.c_float, vp, vp, vp]
        L.bgt_l1_cotangent.argtypes = [vp, C.c_int64, vp, vp, C.c_float, vp, vp]
        L.bgt_adam_step.argtypes = [vp, C.POINTER(bgt_adam_group), C.c_int32, C.c_float, C.c_float, C.c_float,
                                    vp, vp]
        L.bgt_default_densify_config.argtypes = [C.POINTER(bgt_densify_config)]
        L.bgt_default_densify_config.restype = None
        L.bgt_stats_accumulate.argtypes = [vp, C.POINTER(bgt_prims), C.POINTER(bgt_views), vp, C.c_size_t, vp,
                                           C.POINTER(bgt_grads), C.POINTER(bgt_prim_stats), vp]
        L.bgt_densify_plan.argtypes = [vp, C.POINTER(bgt_prims), C.POINTER(bgt_prim_stats),
                                       C.POINTER(bgt_densify_config), vp, vp, vp, vp]
        L.bgt_densify_apply.argtypes = [vp, C.POINTER(bgt_prims), vp, vp, C.c_int32, C.POINTER(bgt_grads), vp]
        L.bgt_profile.argtypes = [vp, C.c_int]
        L.bgt_stage_times.argtypes = [vp, C.POINTER(C.c_float)]
        _lib = L
    return _lib


# ------------------------------------------------------------ thin wrappers (same names)

def bgt_default_config(**overrides) -> bgt_config:
    c = bgt_config()
    lib().bgt_default_config(C.byref(c))
    fields = {f[0] for f in bgt_config._fields_}
    for k, v in overrides.items():
        if k not in fields:  # a ctypes structure would take it as a plain attribute
            raise TypeError(f"bgt_config has no field {k!r} (fields: {sorted(fields)})")
        if k == "bg":
            c.bg = (C.c_float * 3)(*v)
        else:
            setattr(c, k, v)
    return c


def bgt_validate_config(cfg: bgt_config) -> int:
    return lib().bgt_validate_config(C.byref(cfg))


def bgt_validate_prims(prims: bgt_prims, cfg: bgt_config) -> int:
    return lib().bgt_validate_prims(C.byref(prims), C.byref(cfg))


def bgt_validate_views(views: bgt_views) -> int:
    return lib().bgt_validate_views(C.byref(views))


def bgt_create(cfg: bgt_config | None, device: int) -> C.c_void_p:
    h = C.c_void_p()
    st = lib().bgt_create(C.byref(cfg) if cfg is not None else None, device, C.byref(h))
    if st != BGT_OK:
        raise BgtError(st, "bgt_create failed")
    return h


def bgt_destroy(ctx) -> None:
    lib().bgt_destroy(ctx)


def bgt_last_error(ctx) -> str:
    return lib().bgt_last_error(ctx).decode()


def _check(ctx, st):
    if st != BGT_OK:
        raise BgtError(st, bgt_last_error(ctx))
    return st


def bgt_tessellate(ctx, prims: bgt_prims, verts_ptr: int, stream: int = 0) -> int:
    return _check(ctx, lib().bgt_tessellate(ctx, C.byref(prims), verts_ptr, stream))


def bgt_state_size(ctx, prims: bgt_prims, views: bgt_views) -> int:
    n = C.c_size_t()
    _check(ctx, lib().bgt_state_size(ctx, C.byref(prims), C.byref(views), C.byref(n)))
    return int(n.value)


def bgt_state_layout(ctx, prims: bgt_prims, views: bgt_views) -> dict:
    off = (C.c_int64 * BGT_STATE_FIELDS)()
    _check(ctx, lib().bgt_state_layout(ctx, C.byref(prims), C.byref(views), off))
    return dict(zip(STATE_FIELD_NAMES, [int(x) for x in off]))


def bgt_render_fwd(ctx, prims, views, images_ptr, state_ptr, state_bytes, stream=0) -> int:
    return _check(ctx, lib().bgt_render_fwd(ctx, C.byref(prims), C.byref(views), images_ptr, state_ptr,
                                            state_bytes, stream))


def bgt_render_bwd(ctx, prims, views, images_ptr, grad_images_ptr, state_ptr, state_bytes, grads: bgt_grads,
                   stream=0) -> int:
    return _check(ctx, lib().bgt_render_bwd(ctx, C.byref(prims), C.byref(views), images_ptr, grad_images_ptr,
                                            state_ptr, state_bytes, C.byref(grads), stream))


def bgt_query(ctx, state_ptr, state_bytes, stream=0):
    """Returns (status, counters[10]); status may be BGT_E_OVERFLOW."""
    out = (C.c_int64 * 10)()
    st = lib().bgt_query(ctx, state_ptr, state_bytes, out, stream)
    if st not in (BGT_OK, BGT_E_OVERFLOW):
        raise BgtError(st, bgt_last_error(ctx))
    return st, [int(x) for x in out]


def bgt_loss_workspace_size(views: bgt_views) -> int:
    n = C.c_size_t()
    st = lib().bgt_loss_workspace_size(C.byref(views), C.byref(n))
    if st != BGT_OK:
        raise BgtError(st, "invalid views")
    return int(n.value)


def bgt_loss(ctx, views, images_ptr, targets_ptr, lam, loss_ptr, grad_images_ptr, workspace_ptr, workspace_bytes,
             stream=0) -> int:
    return _check(ctx, lib().bgt_loss(ctx, C.byref(views), images_ptr, targets_ptr, lam, loss_ptr, grad_images_ptr,
                                      workspace_ptr, workspace_bytes, stream))


def bgt_loss_noalloc(ctx, views, images_ptr, targets_ptr, lam, loss_ptr, grad_images_ptr, stream=0) -> int:
    return _check(ctx, lib().bgt_loss_noalloc(ctx, C.byref(views), images_ptr, targets_ptr, lam, loss_ptr,
                                              grad_images_ptr, stream))


def bgt_l1_cotangent(ctx, n, images_ptr, targets_ptr, scale, grad_ptr, stream=0) -> int:
    return _check(ctx, lib().bgt_l1_cotangent(ctx, n, images_ptr, targets_ptr, scale, grad_ptr, stream))


def bgt_adam_step(ctx, groups, beta1, beta2, eps, step_ptr, stream=0) -> int:
    """groups: sequence of bgt_adam_group (host)."""
    arr = (bgt_adam_group * max(len(groups), 1))(*groups)
    return _check(ctx, lib().bgt_adam_step(ctx, arr, len(groups), beta1, beta2, eps, step_ptr, stream))


def bgt_default_densify_config(**overrides) -> bgt_densify_config:
    c = bgt_densify_config()
    lib().bgt_default_densify_config(C.byref(c))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def bgt_stats_accumulate(ctx, prims, views, state_ptr, state_bytes, targets_ptr, grads, stats: bgt_prim_stats,
                         stream=0) -> int:
    """grads: bgt_grads or None; targets_ptr: device pointer or None."""
    return _check(ctx, lib().bgt_stats_accumulate(ctx, C.byref(prims), C.byref(views), state_ptr, state_bytes,
                                                  targets_ptr, C.byref(grads) if grads is not None else None,
                                                  C.byref(stats), stream))


def bgt_densify_plan(ctx, prims, stats: bgt_prim_stats, cfg: bgt_densify_config, action_ptr, dst_index_ptr,
                     count_ptr, stream=0) -> int:
    return _check(ctx, lib().bgt_densify_plan(ctx, C.byref(prims), C.byref(stats), C.byref(cfg), action_ptr,
                                              dst_index_ptr, count_ptr, stream))


def bgt_densify_apply(ctx, prims, action_ptr, dst_index_ptr, dst_prims, dst: bgt_grads, stream=0) -> int:
    return _check(ctx, lib().bgt_densify_apply(ctx, C.byref(prims), action_ptr, dst_index_ptr, dst_prims,
                                               C.byref(dst), stream))


def bgt_profile(ctx, enable: bool) -> int:
    return _check(ctx, lib().bgt_profile(ctx, 1 if enable else 0))


def bgt_stage_times(ctx) -> dict:
    ms = (C.c_float * BGT_NUM_STAGES)()
    _check(ctx, lib().bgt_stage_times(ctx, ms))
    return dict(zip(STAGE_NAMES, [float(x) for x in ms]))


# ------------------------------------------------------------ struct builders

def make_prims(degree, num_prims, ctrl, color_ctrl, log_scale, quat, opacity, sharpness, attr_res=1, sh_degree=0,
               sh=None):
    """Pointers are integers (device addresses)."""
    return bgt_prims(degree, num_prims, attr_res, sh_degree, ctrl, color_ctrl, log_scale, quat, opacity, sharpness,
                     sh)


def make_views(wh_int32_array, cams_ptr):
    """wh: host numpy int32 [V][2] (kept alive by the caller); cams: device pointer."""
    n = int(wh_int32_array.shape[0])
    p = wh_int32_array.ctypes.data_as(C.POINTER(C.c_int32))
    return bgt_views(n, 0, p, cams_ptr)


def make_grads(ctrl, color_ctrl, log_scale, quat, opacity, sharpness, sh=None):
    return bgt_grads(ctrl, color_ctrl, log_scale, quat, opacity, sharpness, sh)
