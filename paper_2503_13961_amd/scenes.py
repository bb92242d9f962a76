"""Seeded synthetic inputs: Bezier-triangle scenes and pinhole cameras.

This module only draws inputs.  It holds none of the rendering arithmetic,
and both the HIP path and the CPU oracle take their inputs from here.

Layouts match the C ABI (structure-of-arrays, float32):

* ``ctrl``, ``color_ctrl``: ``[3][ncp][P]`` with ``ncp = (n+1)(n+2)/2``.
  The control-point index follows the double sum of Eq. 1:
  ``i = 0..n`` outer, ``j = 0..n-i`` inner, ``k = n-i-j``; ``u`` pairs with
  ``i``, ``v`` with ``j`` and ``w`` with ``k``.
* ``log_scale``: ``[3][T][P]``, ``quat``: ``[4][T][P]`` as ``(w, x, y, z)``,
  with ``T = R(R+1)/2`` texels of the attribute map (``R`` 1 or 3; texel
  ``t`` enumerates the nodes ``(a, b)``, ``a + b <= R - 1``, ``a`` outer).
* ``opacity``, ``sharpness``: ``[P]``.
* ``sh``: ``[3][K][P]``, the view-dependent colour's SH coefficients of bands
  1..D (``K = (D+1)^2 - 1``, ``D = sh_degree``), absent when ``D = 0``.
* cameras: ``cams`` float32 ``[V][16]`` = world-to-camera ``R`` (row-major
  3x3), ``t`` (3), ``fx, fy, cx, cy``; ``wh`` int32 ``[V][2]`` = width, height.
  Axes follow OpenCV (x right, y down, z forward); the vertical field of
  view sets ``fx = fy = H / (2 tan(fov/2))`` and ``(cx, cy) = (W/2, H/2)``.

The scene recipes stand in for the paper's datasets (NeRF-Synthetic, masked
Tanks and Temples), which are not available: a deformed geodesic sphere of
quadratic patches stands in for a closed object seen from cameras on a
sphere facing its centre (the camera layout of the toy experiments in Sec. 4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def cp_indices(n: int):
    """(i, j, k) triples of a degree-n Bezier triangle in Eq. 1 order."""
    return [(i, j, n - i - j) for i in range(n + 1) for j in range(n - i + 1)]


def num_ctrl(n: int) -> int:
    return (n + 1) * (n + 2) // 2


@dataclass
class Scene:
    degree: int
    ctrl: np.ndarray          # [3][ncp][P] f32
    color_ctrl: np.ndarray    # [3][ncp][P] f32
    log_scale: np.ndarray     # [3][T][P] f32
    quat: np.ndarray          # [4][T][P] f32
    opacity: np.ndarray       # [P] f32
    sharpness: np.ndarray     # [P] f32
    attr_res: int = 1
    name: str = ""
    sh_degree: int = 0
    sh: np.ndarray | None = None   # [3][K][P] f32 when sh_degree > 0

    @property
    def num_prims(self) -> int:
        return int(self.ctrl.shape[2])

    def arrays(self):
        d = dict(ctrl=self.ctrl, color_ctrl=self.color_ctrl,
                 log_scale=self.log_scale, quat=self.quat,
                 opacity=self.opacity, sharpness=self.sharpness)
        if self.sh_degree > 0:
            d["sh"] = self.sh
        return d

    def copy(self) -> "Scene":
        return Scene(self.degree, self.ctrl.copy(), self.color_ctrl.copy(),
                     self.log_scale.copy(), self.quat.copy(),
                     self.opacity.copy(), self.sharpness.copy(),
                     self.attr_res, self.name, self.sh_degree,
                     None if self.sh is None else self.sh.copy())

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.degree, np.ascontiguousarray(self.ctrl[:, :, idx]),
                     np.ascontiguousarray(self.color_ctrl[:, :, idx]),
                     np.ascontiguousarray(self.log_scale[:, :, idx]),
                     np.ascontiguousarray(self.quat[:, :, idx]),
                     np.ascontiguousarray(self.opacity[idx]),
                     np.ascontiguousarray(self.sharpness[idx]),
                     self.attr_res, self.name + "[subset]", self.sh_degree,
                     None if self.sh is None else np.ascontiguousarray(self.sh[:, :, idx]))

    def save(self, path):
        np.savez(path, degree=self.degree, attr_res=self.attr_res, sh_degree=self.sh_degree,
                 **self.arrays())

    @staticmethod
    def load(path) -> "Scene":
        z = np.load(path)  # allow_pickle stays False
        shd = int(z["sh_degree"]) if "sh_degree" in z else 0
        return Scene(int(z["degree"]), z["ctrl"], z["color_ctrl"],
                     z["log_scale"], z["quat"], z["opacity"], z["sharpness"],
                     int(z["attr_res"]), "", shd, z["sh"] if shd > 0 else None)


@dataclass
class Cameras:
    cams: np.ndarray   # [V][16] f32
    wh: np.ndarray     # [V][2] i32
    eyes: list = field(default_factory=list)

    @property
    def n_views(self) -> int:
        return int(self.cams.shape[0])

    @property
    def num_pixels(self) -> int:
        return int(np.sum(self.wh[:, 0].astype(np.int64) * self.wh[:, 1]))

    def view(self, v: int) -> "Cameras":
        return Cameras(np.ascontiguousarray(self.cams[v:v + 1]),
                       np.ascontiguousarray(self.wh[v:v + 1]),
                       self.eyes[v:v + 1] if self.eyes else [])


# ---------------------------------------------------------------- cameras

def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)):
    """World-to-camera rotation and translation, OpenCV axes."""
    eye = np.asarray(eye, np.float64)
    zc = np.asarray(target, np.float64) - eye
    zc /= np.linalg.norm(zc)
    xc = np.cross(zc, np.asarray(up, np.float64))
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    R = np.stack([xc, yc, zc])
    t = -R @ eye
    return R, t


def make_cameras(eyes, sizes, fov_deg=60.0, target=(0.0, 0.0, 0.0)) -> Cameras:
    cams = np.zeros((len(eyes), 16), np.float32)
    wh = np.zeros((len(eyes), 2), np.int32)
    for v, (eye, (W, H)) in enumerate(zip(eyes, sizes)):
        R, t = look_at(eye, target)
        f = H / (2.0 * math.tan(math.radians(fov_deg) / 2.0))
        cams[v, 0:9] = R.reshape(-1)
        cams[v, 9:12] = t
        cams[v, 12:16] = (f, f, W / 2.0, H / 2.0)
        wh[v] = (W, H)
    return Cameras(cams, wh, [tuple(map(float, e)) for e in eyes])


def fibonacci_eyes(n: int, radius: float):
    """n eyes on a sphere: y_i = 1-(2i+1)/n, azimuth i*pi*(3-sqrt5)."""
    out = []
    for i in range(n):
        y = 1.0 - (2 * i + 1) / n
        r = math.sqrt(max(0.0, 1.0 - y * y))
        phi = i * math.pi * (3.0 - math.sqrt(5.0))
        out.append((radius * r * math.cos(phi), radius * y, radius * r * math.sin(phi)))
    return out


# ---------------------------------------------------------------- attributes

def _random_quats(rng, P):
    q = rng.normal(size=(P, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _attributes(rng, P, ncp, s_ref, opacity, sharpness):
    """Colour control points, log-scales, rotations, opacity, sharpness.

    Draw order is fixed: colours, log-scales, quaternions, then opacity and
    sharpness when they are random.
    """
    color = rng.random((P, ncp, 3))
    log_scale = math.log(s_ref) + rng.uniform(-0.3, 0.3, size=(P, 3))
    quat = _random_quats(rng, P)
    if isinstance(opacity, tuple):
        op = rng.uniform(opacity[0], opacity[1], size=P)
    else:
        op = np.full(P, float(opacity))
    if isinstance(sharpness, tuple):
        sh = rng.uniform(sharpness[0], sharpness[1], size=P)
    else:
        sh = np.full(P, float(sharpness))
    return color, log_scale, quat, op, sh


def _pack(degree, ctrl_pn3, color_pn3, log_scale_p3, quat_p4, op, sh, name):
    f32 = np.float32
    return Scene(
        degree=degree,
        ctrl=np.ascontiguousarray(np.transpose(ctrl_pn3, (2, 1, 0)), dtype=f32),
        color_ctrl=np.ascontiguousarray(np.transpose(color_pn3, (2, 1, 0)), dtype=f32),
        log_scale=np.ascontiguousarray(log_scale_p3.T[:, None, :], dtype=f32),
        quat=np.ascontiguousarray(quat_p4.T[:, None, :], dtype=f32),
        opacity=np.ascontiguousarray(op, dtype=f32),
        sharpness=np.ascontiguousarray(sh, dtype=f32),
        attr_res=1, name=name)


# ---------------------------------------------------------------- scenes

def random_triangles(P=64, degree=2, seed=0, s_ref=None, opacity=0.8,
                     sharpness=10.0, d_cam=4.0, f=128 / (2 * math.tan(math.pi / 6))):
    """Every control point drawn independently from U[-1,1]^3."""
    rng = np.random.default_rng(seed)
    ncp = num_ctrl(degree)
    ctrl = rng.uniform(-1.0, 1.0, size=(P, ncp, 3))
    if s_ref is None:
        s_ref = d_cam / f
    color, ls, q, op, sh = _attributes(rng, P, ncp, s_ref, opacity, sharpness)
    return _pack(degree, ctrl, color, ls, q, op, sh, f"random{P}_n{degree}")


def _icosahedron():
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, phi, 0], [1, phi, 0], [-1, -phi, 0], [1, -phi, 0],
                  [0, -1, phi], [0, 1, phi], [0, -1, -phi], [0, 1, -phi],
                  [phi, 0, -1], [phi, 0, 1], [-phi, 0, -1], [-phi, 0, 1]], np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
         [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
         [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
         [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    faces = []
    for a, b, c in f:
        n = np.cross(v[b] - v[a], v[c] - v[a])
        if np.dot(n, v[a] + v[b] + v[c]) < 0:
            b, c = c, b
        faces.append((a, b, c))
    return v, faces


def deformed_sphere(freq=10, degree=2, seed=0, noise=0.05, radius=1.0,
                    s_ref=None, opacity=(0.3, 1.0), sharpness=10.0,
                    d_cam=2.0, f=800 / (2 * math.tan(math.pi / 6))):
    """Geodesic (class I) icosphere of 20*freq^2 Bezier triangles.

    Control nodes sit on the shared (degree*freq)-lattice of each face, are
    projected to the unit sphere and displaced radially once per node by
    ``1 + N(0, noise^2)``, so neighbouring patches share their edge control
    points and the surface is watertight.
    """
    rng = np.random.default_rng(seed)
    V, faces = _icosahedron()
    m = degree * freq
    node_id = {}
    node_dir = []

    def node(face, a, b):
        A, B, C = (V[i] for i in face)
        c = m - a - b
        p = (a * A + b * B + c * C) / m
        p = p / np.linalg.norm(p)
        key = tuple(np.round(p * 1e9).astype(np.int64))
        if key not in node_id:
            node_id[key] = len(node_dir)
            node_dir.append(p)
        return node_id[key]

    tris = []  # each: list of node ids in Eq.1 order
    cps = cp_indices(degree)
    for face in faces:
        small = []
        for a in range(freq):
            for b in range(freq - a):
                c = freq - 1 - a - b
                small.append(((a + 1, b, c), (a, b + 1, c), (a, b, c + 1)))
        for a in range(freq - 1):
            for b in range(freq - 1 - a):
                c = freq - 2 - a - b
                small.append(((a, b + 1, c + 1), (a + 1, b, c + 1), (a + 1, b + 1, c)))
        for U, Vv, W in small:
            ids = []
            for (i, j, k) in cps:
                la = i * U[0] + j * Vv[0] + k * W[0]
                lb = i * U[1] + j * Vv[1] + k * W[1]
                ids.append(node((face), la, lb))
            tris.append(ids)
    dirs = np.array(node_dir)
    rad = radius * (1.0 + noise * rng.normal(size=len(dirs)))
    pos = dirs * rad[:, None]
    P = len(tris)
    ncp = len(cps)
    ctrl = pos[np.array(tris)]  # [P][ncp][3]
    if s_ref is None:
        s_ref = d_cam / f
    color, ls, q, op, sh = _attributes(rng, P, ncp, s_ref, opacity, sharpness)
    return _pack(degree, ctrl, color, ls, q, op, sh, f"sphere_nu{freq}_n{degree}")


def box_triangles(P=20000, degree=3, seed=0, box=4.0, size_range=(0.01, 0.3),
                  sharpness=(1.0, 20.0), opacity=(0.3, 1.0), s_ref=None,
                  d_cam=8.0, f=1600 / (2 * math.tan(math.pi / 6))):
    """Randomly placed, sized and oriented patches in a cube of side ``box``.

    Corners are ``centre + size * rotation @ e_k`` with ``e_k`` on the unit
    circle at 90, 210 and 330 degrees; the other control points are the flat
    lattice positions plus ``N(0, (0.1 size)^2)``.
    """
    rng = np.random.default_rng(seed)
    ncp = num_ctrl(degree)
    centre = rng.uniform(-box / 2, box / 2, size=(P, 3))
    size = np.exp(rng.uniform(math.log(size_range[0]), math.log(size_range[1]), size=P))
    qs = _random_quats(rng, P)
    ang = np.radians([90.0, 210.0, 330.0])
    e = np.stack([np.cos(ang), np.sin(ang), np.zeros(3)], axis=1)  # [3][3]
    ctrl = np.zeros((P, ncp, 3))
    noise = rng.normal(size=(P, ncp, 3))
    for p in range(P):
        w, x, y, z = qs[p]
        Rm = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                       [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                       [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        corners = centre[p] + size[p] * (e @ Rm.T)  # U, V, W
        for idx, (i, j, k) in enumerate(cp_indices(degree)):
            flat = (i * corners[0] + j * corners[1] + k * corners[2]) / degree
            corner = (i == degree) or (j == degree) or (k == degree)
            ctrl[p, idx] = flat if corner else flat + 0.1 * size[p] * noise[p, idx]
    if s_ref is None:
        s_ref = d_cam / f
    color, ls, q, op, sh = _attributes(rng, P, ncp, s_ref, opacity, sharpness)
    return _pack(degree, ctrl, color, ls, q, op, sh, f"box{P}_n{degree}")


def flat_patch(corners, degree=1, color=(1.0, 1.0, 1.0), log_scale=-6.0,
               opacity=0.8, sharpness=10.0):
    """Single planar patch with control points on the flat lattice."""
    corners = np.asarray(corners, np.float64)
    ncp = num_ctrl(degree)
    ctrl = np.zeros((1, ncp, 3))
    for idx, (i, j, k) in enumerate(cp_indices(degree)):
        ctrl[0, idx] = (i * corners[0] + j * corners[1] + k * corners[2]) / degree
    col = np.tile(np.asarray(color, np.float64), (1, ncp, 1))
    ls = np.full((1, 3), float(log_scale))
    q = np.array([[1.0, 0.0, 0.0, 0.0]])
    return _pack(degree, ctrl, col, ls, q, np.array([opacity]), np.array([sharpness]),
                 "flat")


def concat(scenes):
    d = scenes[0].degree
    assert all(s.degree == d for s in scenes)
    return Scene(d, np.concatenate([s.ctrl for s in scenes], axis=2),
                 np.concatenate([s.color_ctrl for s in scenes], axis=2),
                 np.concatenate([s.log_scale for s in scenes], axis=2),
                 np.concatenate([s.quat for s in scenes], axis=2),
                 np.concatenate([s.opacity for s in scenes]),
                 np.concatenate([s.sharpness for s in scenes]), 1, "concat")


# ---------------------------------------------------------------- workloads

def workload(name: str, seed: int = 0):
    """Named workloads: returns (scene, cameras, description)."""
    if name == "tiny":
        sc = random_triangles(P=16, degree=2, seed=seed)
        cams = make_cameras([(0.0, 0.0, 4.0)], [(70, 53)])
        return sc, cams, "16 random quadratic patches, one 70x53 view"
    if name == "random64":
        sc = random_triangles(P=64, degree=2, seed=seed)
        cams = make_cameras([(0.0, 0.0, 4.0)], [(128, 128)])
        return sc, cams, "64 random quadratic patches, one 128x128 view, fov 60"
    if name == "sphere2k_1v":
        sc = deformed_sphere(freq=10, seed=seed)
        cams = make_cameras([(0.0, 0.0, 3.0)], [(800, 800)])
        return sc, cams, "2000-patch deformed sphere, one 800x800 view"
    if name == "sphere2k_16v_mixed":
        sc = deformed_sphere(freq=10, seed=seed)
        eyes = fibonacci_eyes(16, 3.0)
        sizes = [(400 + round(400 * i / 15),) * 2 for i in range(16)]
        return sc, make_cameras(eyes, sizes), "2000-patch sphere, 16 views 400..800 square"
    if name == "sphere2k_16v_800":
        sc = deformed_sphere(freq=10, seed=seed)
        eyes = fibonacci_eyes(16, 3.0)
        return sc, make_cameras(eyes, [(800, 800)] * 16), "2000-patch sphere, 16 views 800x800"
    if name == "box20k_cubic":
        sc = box_triangles(P=20000, degree=3, seed=seed)
        cams = make_cameras([(0.0, 0.0, 8.0)], [(1600, 1600)])
        return sc, cams, "20000 cubic patches in a 4^3 box, one 1600x1600 view"
    if name == "sphere50k_32v":
        sc = deformed_sphere(freq=50, seed=seed, f=768 / (2 * math.tan(math.pi / 6)))
        eyes = fibonacci_eyes(32, 3.0)
        return sc, make_cameras(eyes, [(1024, 768)] * 32), "50000-patch sphere, 32 views 1024x768"
    if name.startswith("sphere_small"):
        # small sphere views for parity tests: ragged sizes spanning several tiles
        sc = deformed_sphere(freq=4, seed=seed, f=90 / (2 * math.tan(math.pi / 6)))
        eyes = fibonacci_eyes(3, 3.0)
        return sc, make_cameras(eyes, [(97, 90), (64, 64), (130, 75)]), \
            "320-patch sphere, 3 ragged views"
    raise KeyError(name)


def lattice_scaled(scene: Scene, m: int = 4, L: int = 4, c: float = 0.6) -> Scene:
    """The scene with Gaussians sized for the lattice variant (m Gaussians
    per flat sub-triangle edge at tessellation level L): the log-scales of
    patch p shifted so that their mean is log(c h_p), h_p = the mean length
    of its three corner edges over L (m - 1), the lattice spacing, so that
    neighbouring lattice Gaussians overlap and cover the patch.  The
    per-axis offsets (the anisotropy) and the rotations are kept."""
    n = scene.degree
    ids = cp_indices(n)
    corner = [ids.index((n, 0, 0)), ids.index((0, n, 0)), ids.index((0, 0, n))]
    X = scene.ctrl[:, corner, :].astype(np.float64)            # [3][3 corners][P]
    edges = [np.linalg.norm(X[:, a] - X[:, b], axis=0) for a, b in ((0, 1), (1, 2), (2, 0))]
    h = (edges[0] + edges[1] + edges[2]) / 3.0 / (L * (m - 1))
    out = scene.copy()
    ls = scene.log_scale.astype(np.float64)
    ls = ls - ls.mean(axis=(0, 1), keepdims=True) + np.log(c * h)[None, None, :]
    out.log_scale = np.ascontiguousarray(ls, dtype=np.float32)
    out.name = scene.name + f"_lattice{m}"
    return out


def l1_target(num_pixels: int, seed: int = 0) -> np.ndarray:
    """Random target image for the L1 cotangent, U[0,1] per pixel-channel."""
    return np.random.default_rng(1000 + seed).random((num_pixels, 3)).astype(np.float32)


def num_sh(sh_degree: int) -> int:
    """SH coefficients per colour channel in bands 1..D."""
    return (sh_degree + 1) ** 2 - 1


def with_attributes(scene: Scene, attr_res=3, sh_degree=3, seed=0, scale_jitter=0.2, quat_jitter=0.2,
                    sh_std=0.1) -> Scene:
    """The scene with resolution-`attr_res` rotation and scale maps and SH
    colour of degree `sh_degree`.  Each texel takes its patch's log-scales
    plus U(-scale_jitter, scale_jitter) and its quaternion plus
    N(0, quat_jitter^2) per component; SH coefficients are N(0, sh_std^2)
    divided by the band index.  Draw order: log-scales, quaternions, SH."""
    rng = np.random.default_rng(seed)
    P = scene.num_prims
    T = attr_res * (attr_res + 1) // 2
    out = scene.copy()
    out.attr_res = attr_res
    base_ls = scene.log_scale[:, 0, :].astype(np.float64)
    base_q = scene.quat[:, 0, :].astype(np.float64)
    ls = base_ls[:, None, :] + (rng.uniform(-scale_jitter, scale_jitter, size=(3, T, P)) if T > 1 else 0.0)
    q = base_q[:, None, :] + (rng.normal(0.0, quat_jitter, size=(4, T, P)) if T > 1 else 0.0)
    out.log_scale = np.ascontiguousarray(ls, dtype=np.float32)
    out.quat = np.ascontiguousarray(q, dtype=np.float32)
    out.sh_degree = sh_degree
    if sh_degree > 0:
        K = num_sh(sh_degree)
        band = np.array([int(math.isqrt(k + 1)) for k in range(K)], np.float64)   # k + 1 = l^2 + (m + l)
        out.sh = np.ascontiguousarray(rng.normal(0.0, sh_std, size=(3, K, P)) / band[None, :, None],
                                      dtype=np.float32)
    else:
        out.sh = None
    out.name = scene.name + f"_R{attr_res}_SH{sh_degree}"
    return out
