"""FP64 reference of the splitting and pruning step (Sec. 3.3, Splitting and
Pruning; implementation details, Splitting and Pruning).  Test
infrastructure only, like the rest of oracle/.

Readings where the paper is silent:
  - Splitting cuts a patch at its edge midpoints into four patches of the
    same degree: three corner patches and the middle one, whose domain is the
    parent's domain triangle turned by a half turn (its u corner is the
    midpoint opposite u).  Their control nets are the parent's blossom at the
    sub-domain corners, so each child reproduces its part of the parent
    surface (and colour) exactly.  Per-patch attributes (attribute-map
    texels, opacity, sharpness, SH coefficients) are copied.
  - Position gradient: the mean over a patch's control points of |dL/dp|,
    accumulated over the calls in which the patch is visible, and averaged.
  - Edge prior: the Sobel gradient magnitude of the training image's grey
    level (mean of R, G, B on the 0..255 scale the threshold 13 implies;
    0 on the image border), summed over the pixels the patch wins in I_id and
    averaged over them.
  - Visibility count ratio: the number of rendered views in which the patch
    wins at least one pixel, over the number of views rendered.
  - Visibility texture: one texel per flat sub-triangle of the tessellation
    (L^2 cells over the patch's (u, v) domain, the cell being the one I_tri
    names); its ratio is the share of texels seen in any view.
  - Area: the four planar triangles through the surface points at the
    corners and edge midpoints.  Aspect ratio: the box of the corner
    triangle aligned with its longest edge, i.e. that edge's length over the
    triangle's height on it.
  - A patch that meets a pruning criterion is removed and not split.
"""
from __future__ import annotations

import math

import numpy as np

# thresholds of the implementation details
TAU_G = 0.0018   # mean position gradient
TAU_B = 13.0     # mean edge prior
TAU_V = 0.08     # visibility count ratio
TAU_R = 0.4      # visibility texture ratio
TAU_A = 3e-4     # area
TAU_S = 10.0     # aspect ratio

KEEP, SPLIT, PRUNE = 0, 1, 2


def ctrl_index(n, i, j):
    """Linear index of p_ijk in the order of Eq. 1's sum (i outer, j inner)."""
    return sum(n - a + 1 for a in range(i)) + j


def _blossom(net, n, pts):
    """Blossom of a degree-n net (dict (i, j) -> value) at the n barycentric
    points `pts`: one de Casteljau step per point."""
    cur = dict(net)
    deg = n
    for (a, b, c) in pts:
        nxt = {}
        for i in range(deg):
            for j in range(deg - i):
                nxt[(i, j)] = a * cur[(i + 1, j)] + b * cur[(i, j + 1)] + c * cur[(i, j)]
        cur, deg = nxt, deg - 1
    return cur[(0, 0)]


# domain corners (u, v, w) of the four children, in the order corner u,
# corner v, corner w, middle
CHILD_CORNERS = (
    ((1.0, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.0, 0.5)),
    ((0.5, 0.5, 0.0), (0.0, 1.0, 0.0), (0.0, 0.5, 0.5)),
    ((0.5, 0.0, 0.5), (0.0, 0.5, 0.5), (0.0, 0.0, 1.0)),
    ((0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0)),
)


def subdivide(cp, n):
    """Control nets [4][ncp][d] of the four children of a degree-n net
    cp [ncp][d] (any number d of channels)."""
    cp = np.asarray(cp, np.float64)
    net = {}
    for i in range(n + 1):
        for j in range(n - i + 1):
            net[(i, j)] = cp[ctrl_index(n, i, j)]
    out = np.zeros((4,) + cp.shape)
    for c, (A, B, Cc) in enumerate(CHILD_CORNERS):
        for i in range(n + 1):
            for j in range(n - i + 1):
                k = n - i - j
                out[c, ctrl_index(n, i, j)] = _blossom(net, n, [A] * i + [B] * j + [Cc] * k)
    return out


def _surface(cp, n, u, v, w):
    s = np.zeros(cp.shape[1])
    for i in range(n + 1):
        for j in range(n - i + 1):
            k = n - i - j
            coef = math.factorial(n) / (math.factorial(i) * math.factorial(j) * math.factorial(k))
            s += coef * u ** i * v ** j * w ** k * cp[ctrl_index(n, i, j)]
    return s


def area4(cp, n):
    """Sum of the areas of the four planar triangles through the corner and
    edge-midpoint surface points."""
    cp = np.asarray(cp, np.float64)
    P = {k: _surface(cp, n, *uvw) for k, uvw in {
        "u": (1, 0, 0), "v": (0, 1, 0), "w": (0, 0, 1),
        "uv": (0.5, 0.5, 0), "vw": (0, 0.5, 0.5), "wu": (0.5, 0, 0.5)}.items()}

    def tri(a, b, c):
        return 0.5 * np.linalg.norm(np.cross(P[b] - P[a], P[c] - P[a]))
    return tri("u", "uv", "wu") + tri("uv", "v", "vw") + tri("wu", "vw", "w") + tri("vw", "wu", "uv")


def aspect(cp, n):
    """Longest corner edge over the corner triangle's height on it."""
    cp = np.asarray(cp, np.float64)
    A, B, C = cp[ctrl_index(n, n, 0)], cp[ctrl_index(n, 0, n)], cp[ctrl_index(n, 0, 0)]
    edges = [np.linalg.norm(B - A), np.linalg.norm(C - B), np.linalg.norm(A - C)]
    twice_area = np.linalg.norm(np.cross(B - A, C - A))
    L = max(edges)
    return math.inf if twice_area == 0.0 else L * L / twice_area


def sobel_edges(img, W, H):
    """Sobel gradient magnitude of the grey level (0..255) of one view's
    image [H*W][3]; 0 on the border."""
    g = np.asarray(img, np.float64).reshape(H, W, 3).mean(axis=2) * 255.0
    out = np.zeros((H, W))
    if H >= 3 and W >= 3:
        gx = (g[:-2, 2:] + 2 * g[1:-1, 2:] + g[2:, 2:]) - (g[:-2, :-2] + 2 * g[1:-1, :-2] + g[2:, :-2])
        gy = (g[2:, :-2] + 2 * g[2:, 1:-1] + g[2:, 2:]) - (g[:-2, :-2] + 2 * g[:-2, 1:-1] + g[:-2, 2:])
        out[1:-1, 1:-1] = np.sqrt(gx * gx + gy * gy)
    return out.ravel()


class Stats:
    """Per-patch accumulators over the training calls."""

    def __init__(self, P, L=4):
        self.L2 = L * L
        self.views_seen = 0
        self.vis_views = np.zeros(P, np.int64)
        self.tex = np.zeros(P, np.uint64)
        self.grad_sum = np.zeros(P)
        self.grad_cnt = np.zeros(P, np.int64)
        self.edge_sum = np.zeros(P)
        self.edge_cnt = np.zeros(P, np.int64)

    def accumulate(self, I_tri_views, wh, targets=None, d_ctrl=None):
        """I_tri of each view (list of [H*W] int arrays), targets packed
        [sum W H][3] or None, d_ctrl [3][ncp][P] or None."""
        P = len(self.vis_views)
        seen = np.zeros(P, bool)
        off = 0
        for it, (W, H) in zip(I_tri_views, wh):
            it = np.asarray(it)
            fg = it >= 0
            g, s = it[fg] // self.L2, it[fg] % self.L2
            vis = np.zeros(P, bool)
            vis[g] = True
            self.vis_views += vis
            seen |= vis
            for gg, ss in zip(g, s):
                self.tex[gg] |= np.uint64(1) << np.uint64(ss)
            if targets is not None:
                e = sobel_edges(targets[off:off + W * H], W, H)[fg]
                np.add.at(self.edge_sum, g, e)
                np.add.at(self.edge_cnt, g, 1)
            off += W * H
        self.views_seen += len(wh)
        if d_ctrl is not None:
            norms = np.sqrt((np.asarray(d_ctrl, np.float64) ** 2).sum(axis=0)).mean(axis=0)   # [P]
            self.grad_sum[seen] += norms[seen]
            self.grad_cnt[seen] += 1

    def tex_ratio(self):
        return np.array([bin(int(t)).count("1") for t in self.tex]) / self.L2


def plan(scene, stats: Stats):
    """Action per patch (KEEP, SPLIT, PRUNE) and the children's first slots."""
    P, n = scene.num_prims, scene.degree
    act = np.full(P, KEEP, np.int32)
    tr = stats.tex_ratio()
    for p in range(P):
        cp = scene.ctrl[:, :, p].T.astype(np.float64)
        vis_ratio = stats.vis_views[p] / max(stats.views_seen, 1)
        if (vis_ratio < TAU_V or tr[p] < TAU_R or area4(cp, n) < TAU_A or aspect(cp, n) > TAU_S):
            act[p] = PRUNE
            continue
        g_avg = stats.grad_sum[p] / stats.grad_cnt[p] if stats.grad_cnt[p] else 0.0
        e_avg = stats.edge_sum[p] / stats.edge_cnt[p] if stats.edge_cnt[p] else 0.0
        if g_avg > TAU_G or e_avg > TAU_B:
            act[p] = SPLIT
    slots = np.where(act == KEEP, 1, np.where(act == SPLIT, 4, 0))
    return act, np.concatenate([[0], np.cumsum(slots)[:-1]]).astype(np.int32), int(slots.sum())


def apply(scene, act, dst):
    """New arrays (ctrl, color_ctrl, log_scale, quat, opacity, sharpness):
    kept patches copied, split patches replaced by their four children, in
    patch order."""
    n = scene.degree
    has_sh = getattr(scene, "sh_degree", 0) > 0
    out = {k: [] for k in ("ctrl", "color_ctrl", "log_scale", "quat", "opacity", "sharpness", "sh")}
    for p in range(scene.num_prims):
        if act[p] == PRUNE:
            continue
        nets = [scene.ctrl[:, :, p].T.astype(np.float64)], [scene.color_ctrl[:, :, p].T.astype(np.float64)]
        if act[p] == SPLIT:
            nets = list(subdivide(nets[0][0], n)), list(subdivide(nets[1][0], n))
        for c, cc in zip(*nets):
            out["ctrl"].append(c.T)
            out["color_ctrl"].append(cc.T)
            out["log_scale"].append(scene.log_scale[:, :, p])
            out["quat"].append(scene.quat[:, :, p])
            out["opacity"].append(scene.opacity[p])
            out["sharpness"].append(scene.sharpness[p])
            if has_sh:
                out["sh"].append(scene.sh[:, :, p])
    res = {"ctrl": np.stack(out["ctrl"], axis=-1), "color_ctrl": np.stack(out["color_ctrl"], axis=-1),
           "log_scale": np.stack(out["log_scale"], axis=-1), "quat": np.stack(out["quat"], axis=-1),
           "opacity": np.array(out["opacity"]), "sharpness": np.array(out["sharpness"])}
    if has_sh:
        res["sh"] = np.stack(out["sh"], axis=-1)
    return res
