"""CPU FP64 oracle of the BG-Triangle rendering path (ctypes over bgt_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline of the benchmark may use it; the product path never does.  It
shares no code with the HIP implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bgt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.orc_bernstein.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp]
        L.orc_surface.argtypes = [C.c_int, dp, C.c_double, C.c_double, C.c_double, dp]
        L.orc_tessellate.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_tessellate.restype = C.c_int
        L.orc_frame_create.argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int, C.c_int,
                                       C.c_void_p, ip, dp]
        L.orc_frame_create.restype = C.c_void_p
        L.orc_frame_free.argtypes = [C.c_void_p]
        L.orc_frame_dims.argtypes = [C.c_void_p, ip]
        L.orc_frame_raster.argtypes = [C.c_void_p, ip, dp, C.c_void_p, C.c_void_p]
        L.orc_frame_records.argtypes = [C.c_void_p, dp, C.c_void_p]
        L.orc_frame_lists.argtypes = [C.c_void_p, C.c_int, ip, ip]
        L.orc_frame_render.argtypes = [C.c_void_p, ip, C.c_int, dp, dp, ip, ip]
        L.orc_frame_render.restype = C.c_int
        L.orc_pixel_trace.argtypes = [C.c_void_p, C.c_int, C.c_int, ip, dp, dp, dp]
        L.orc_pixel_trace.restype = C.c_int
        L.orc_frame_grad.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_sh_basis.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_sh_basis.restype = None
        L.orc_theta.argtypes = [C.c_int, C.c_double, C.c_double, ip, dp]
        L.orc_theta.restype = C.c_int
        L.orc_frame_grad.restype = C.c_int
        L.orc_frame_zkeys.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_frame_zkeys.restype = None
        L.orc_gamma_star.argtypes = [C.c_void_p, C.c_int, C.c_int, dp, ip]
        L.orc_gamma_star.restype = C.c_int
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


class _Scene(C.Structure):
    _fields_ = [("degree", C.c_int), ("num_prims", C.c_int), ("attr_res", C.c_int),
                ("ctrl", C.c_void_p), ("color_ctrl", C.c_void_p), ("log_scale", C.c_void_p),
                ("quat", C.c_void_p), ("opacity", C.c_void_p), ("sharpness", C.c_void_p),
                ("sh_degree", C.c_int), ("sh", C.c_void_p)]


class _Config(C.Structure):
    _fields_ = [("L", C.c_int), ("tile", C.c_int), ("z_near", C.c_double), ("g_min", C.c_double),
                ("t_min", C.c_double), ("alpha_max", C.c_double), ("dilation", C.c_double),
                ("r_ref", C.c_double), ("bg", C.c_double * 3), ("no_boundary", C.c_int),
                ("lattice", C.c_int), ("exact_keys", C.c_int)]


@dataclass
class Config:
    """Rendering constants (readings where the paper is silent)."""
    L: int = 4
    tile: int = 16
    z_near: float = 0.2
    g_min: float = 2.0 ** -15
    t_min: float = 2.0 ** -15
    alpha_max: float = 0.99
    dilation: float = 0.3
    r_ref: float = 1e-2
    bg: tuple = (0.0, 0.0, 0.0)
    no_boundary: bool = False  # the ablation variant without blending coefficients (w = 1)
    lattice: int = 0           # m >= 2: m Gaussians per flat sub-triangle edge instead of one per pixel
    exact_keys: bool = False   # untruncated FP64 depth keys (to show what the 40-bit truncation changes)

    def c(self) -> _Config:
        return _Config(self.L, self.tile, self.z_near, self.g_min, self.t_min, self.alpha_max,
                       self.dilation, self.r_ref, (C.c_double * 3)(*self.bg), int(self.no_boundary),
                       int(self.lattice), int(self.exact_keys))

    @property
    def kappa2(self) -> float:
        return 2.0 * math.log(1.0 / self.g_min)


GR = dict(MUX=0, MUY=1, QA=2, QB=3, QC=4, CR=5, CG=6, CB=7, DEPTH=8, SIGMA=9, SA=10, SB=11,
          SC=12, PRIM=13, RX=14, RY=15, SX=16, SY=17, SZ=18, TX=19, TY=20, TZ=21)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _c_scene(scene):
    keep = {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in scene.arrays().items()}
    shd = int(getattr(scene, "sh_degree", 0))
    s = _Scene(scene.degree, scene.num_prims, scene.attr_res,
               *(keep[k].ctypes.data for k in ("ctrl", "color_ctrl", "log_scale", "quat",
                                               "opacity", "sharpness")),
               shd, keep["sh"].ctypes.data if shd > 0 else None)
    return s, keep


def theta(R, u, v):
    """Texel indices and weights of Eq. 5's interpolation at (u, v)."""
    ti, tw = np.zeros(3, np.int32), np.zeros(3)
    n = lib().orc_theta(int(R), float(u), float(v), _ip(ti), _dp(tw))
    return ti[:n], tw[:n]


def sh_basis(D, d):
    """Real SH of bands 1..D at the unit vector d and their Cartesian
    gradients ([K], [K][3])."""
    K = (D + 1) ** 2 - 1
    Y, dY = np.zeros(max(K, 1)), np.zeros((max(K, 1), 3))
    lib().orc_sh_basis(D, float(d[0]), float(d[1]), float(d[2]), _dp(Y), _dp(dY))
    return Y[:K], dY[:K]


def bernstein(n, u, v, w):
    B = np.zeros((n + 1) * (n + 2) // 2)
    lib().orc_bernstein(n, u, v, w, _dp(B))
    return B


def surface(n, cp, u, v, w):
    cp = np.ascontiguousarray(cp, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(3)
    lib().orc_surface(n, _dp(cp), u, v, w, _dp(out))
    return out


def tessellate(scene, L=4):
    VL = (L + 1) * (L + 2) // 2
    out = np.zeros((3, VL, scene.num_prims))
    s, keep = _c_scene(scene)
    rc = lib().orc_tessellate(C.byref(s), L, _dp(out))
    if rc:
        raise ValueError("orc_tessellate failed")
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


class Frame:
    """One view of a scene, rasterized and turned into Gaussians in FP64."""

    def __init__(self, scene, cam, W, H, cfg: Config | None = None, I_tri=None, I_uv=None):
        self.cfg = cfg or Config()
        self.scene = scene
        self.W, self.H = int(W), int(H)
        self._s, self._keep = _c_scene(scene)
        self._cam = np.ascontiguousarray(cam, dtype=np.float32).reshape(16)
        self._cc = self.cfg.c()
        it = None if I_tri is None else np.ascontiguousarray(I_tri, dtype=np.int32)
        iu = None if I_uv is None else np.ascontiguousarray(I_uv, dtype=np.float64)
        self._hold = (it, iu)
        h = lib().orc_frame_create(C.byref(self._s), self._cam.ctypes.data_as(C.POINTER(C.c_float)),
                                   self.W, self.H, C.byref(self._cc),
                                   _ip(it) if it is not None else None,
                                   _dp(iu) if iu is not None else None)
        if not h:
            raise ValueError("orc_frame_create failed")
        self._h = h
        d = np.zeros(8, np.int32)
        lib().orc_frame_dims(h, _ip(d))
        self.tiles_x, self.tiles_y = int(d[2]), int(d[3])
        self.n_gpairs, self.n_bpairs = int(d[4]), int(d[5])
        self.nlat = int(d[7])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_frame_free(h)
            self._h = None

    @property
    def npx(self):
        return self.W * self.H

    def raster(self):
        it = np.zeros(self.npx, np.int32)
        iu = np.zeros((self.npx, 2))
        isb = np.zeros(self.npx, np.uint8)
        val = np.zeros(self.npx, np.uint8)
        lib().orc_frame_raster(self._h, _ip(it), _dp(iu), isb.ctypes.data, val.ctypes.data)
        return it, iu, isb.astype(bool), val.astype(bool)

    def zkeys(self):
        """Depth-key bits of each pixel's winner: the FP64 pattern of 1/z,
        truncated to its high 40 bits unless the frame uses exact keys."""
        out = np.zeros(self.npx, np.uint64)
        lib().orc_frame_zkeys(self._h, out.ctypes.data)
        return out

    def records(self, rendered=False):
        """Records [H*W + nlat][GR]: one per pixel (the pixel's Gaussian, or
        in the lattice variant its boundary point only), then the lattice
        Gaussians; with `rendered`, also which records are rendered."""
        r = np.zeros((self.npx + self.nlat, len(GR)))
        ren = np.zeros(self.npx + self.nlat, np.uint8)
        lib().orc_frame_records(self._h, _dp(r), ren.ctypes.data)
        return (r, ren.astype(bool)) if rendered else r

    def lists(self, which=0):
        nt = self.tiles_x * self.tiles_y
        start = np.zeros(nt + 1, np.int32)
        n = self.n_gpairs if which == 0 else self.n_bpairs
        lst = np.zeros(max(n, 1), np.int32)
        lib().orc_frame_lists(self._h, which, _ip(start), _ip(lst))
        return start, lst[:n]

    def render(self, pixels=None):
        if pixels is None:
            n = self.npx
            pp = None
        else:
            pixels = np.ascontiguousarray(pixels, dtype=np.int32)
            n = len(pixels)
            pp = _ip(pixels)
        img = np.zeros((n, 3))
        T = np.zeros(n)
        vis = np.zeros(n, np.int32)
        nc = np.zeros(n, np.int32)
        rc = lib().orc_frame_render(self._h, pp, n, _dp(img), _dp(T), _ip(vis), _ip(nc))
        if rc:
            raise ValueError("render failed")
        return img, T, vis, nc

    def trace(self, pix, cap=4096):
        g = np.zeros(cap, np.int32)
        a = np.zeros(cap)
        T = np.zeros(cap)
        w = np.zeros(cap)
        n = lib().orc_pixel_trace(self._h, int(pix), cap, _ip(g), _dp(a), _dp(T), _dp(w))
        n = min(n, cap)
        return g[:n], a[:n], T[:n], w[:n]

    def gamma_star(self, pix, prim):
        """gamma* of primitive `prim` at pixel `pix` and the record index of
        the boundary point its gradient is routed to (-1: none in range)."""
        g = np.zeros(1)
        a = np.zeros(1, np.int32)
        if lib().orc_gamma_star(self._h, int(pix), int(prim), _dp(g), _ip(a)):
            raise ValueError("gamma_star failed")
        return float(g[0]), int(a[0])

    def grad(self, grad_image):
        sc = self.scene
        ncp = (sc.degree + 1) * (sc.degree + 2) // 2
        P = sc.num_prims
        gi = np.ascontiguousarray(grad_image, dtype=np.float64).reshape(self.npx, 3)
        T = sc.attr_res * (sc.attr_res + 1) // 2
        shd = int(getattr(sc, "sh_degree", 0))
        out = dict(ctrl=np.zeros((3, ncp, P)), color_ctrl=np.zeros((3, ncp, P)),
                   log_scale=np.zeros((3, T, P)), quat=np.zeros((4, T, P)),
                   opacity=np.zeros(P), sharpness=np.zeros(P))
        if shd > 0:
            out["sh"] = np.zeros((3, (shd + 1) ** 2 - 1, P))
        rc = lib().orc_frame_grad(self._h, _dp(gi), _dp(out["ctrl"]), _dp(out["color_ctrl"]),
                                  _dp(out["log_scale"]), _dp(out["quat"]), _dp(out["opacity"]),
                                  _dp(out["sharpness"]), _dp(out["sh"]) if shd > 0 else None)
        if rc:
            raise ValueError("grad failed")
        return out


def render_views(scene, cams, cfg: Config | None = None):
    """Render every view; returns packed HWC images [sum(W*H)][3] and frames."""
    imgs, frames = [], []
    for v in range(cams.n_views):
        W, H = (int(x) for x in cams.wh[v])
        fr = Frame(scene, cams.cams[v], W, H, cfg)
        imgs.append(fr.render()[0])
        frames.append(fr)
    return np.concatenate(imgs, axis=0), frames


def grad_views(frames, grad_image):
    """Sum of per-view parameter gradients for a packed grad image."""
    tot = None
    off = 0
    for fr in frames:
        g = fr.grad(grad_image[off:off + fr.npx])
        off += fr.npx
        tot = g if tot is None else {k: tot[k] + g[k] for k in tot}
    return tot
