"""Small test-side utilities (no rendering arithmetic of the method)."""
import math

import numpy as np

from paper_2503_13961_amd import scenes as S


def camera_from(R, t, f, W, H, cx=None, cy=None):
    cam = np.zeros(16, np.float32)
    cam[0:9] = np.asarray(R, np.float64).reshape(-1)
    cam[9:12] = t
    cam[12:16] = (f, f, W / 2.0 if cx is None else cx, H / 2.0 if cy is None else cy)
    return cam


def axis_camera(W, H, f):
    """Camera at the world origin looking down +z (identity rotation)."""
    return camera_from(np.eye(3), np.zeros(3), f, W, H)


def pixel_ray_point(cam, px, py, z):
    """World point at camera depth z on the ray through pixel-space (px, py)."""
    R = cam[:9].astype(np.float64).reshape(3, 3)
    t = cam[9:12].astype(np.float64)
    fx, fy, cx, cy = (float(v) for v in cam[12:16])
    xc = np.array([(px - cx) / fx * z, (py - cy) / fy * z, z])
    return R.T @ (xc - t)


def flat_patch_scene(corners, degree=1, color=(1, 1, 1), log_scale=-6.0, opacity=0.8,
                     sharpness=10.0):
    return S.flat_patch(corners, degree, color, log_scale, opacity, sharpness)


def decasteljau(cp, n, u, v, w):
    """Triangular de Casteljau recursion; cp indexed by (i, j) in Eq. 1 order."""
    idx = {ijk: m for m, ijk in enumerate(S.cp_indices(n))}
    pts = {(i, j, k): np.asarray(cp[idx[(i, j, k)]], np.float64) for (i, j, k) in idx}
    for r in range(n, 0, -1):
        nxt = {}
        for i in range(r):
            for j in range(r - i):
                k = r - 1 - i - j
                nxt[(i, j, k)] = u * pts[(i + 1, j, k)] + v * pts[(i, j + 1, k)] + w * pts[(i, j, k + 1)]
        pts = nxt
    return pts[(0, 0, 0)]


def bezier_curve(cps, t):
    """Univariate Bezier curve by de Casteljau."""
    pts = [np.asarray(p, np.float64) for p in cps]
    while len(pts) > 1:
        pts = [(1 - t) * a + t * b for a, b in zip(pts[:-1], pts[1:])]
    return pts[0]


def elevate(cp, n):
    """Degree elevation n -> n+1 of a Bezier triangle (control net [ncp][3])."""
    idx = {ijk: m for m, ijk in enumerate(S.cp_indices(n))}
    out = []
    for (i, j, k) in S.cp_indices(n + 1):
        acc = np.zeros(3)
        if i > 0:
            acc += i * np.asarray(cp[idx[(i - 1, j, k)]])
        if j > 0:
            acc += j * np.asarray(cp[idx[(i, j - 1, k)]])
        if k > 0:
            acc += k * np.asarray(cp[idx[(i, j, k - 1)]])
        out.append(acc / (n + 1))
    return np.array(out)


def scene_ctrl(scene, p):
    """[ncp][3] float64 control net of primitive p."""
    return scene.ctrl[:, :, p].T.astype(np.float64)
