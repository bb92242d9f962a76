"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and read its state back; build the matching oracle configuration."""
import sys

import numpy as np

import oracle
from paper_2503_13961_amd import scenes as S

F32 = lambda x: float(np.float32(x))


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_config(tile=16, L=4, bg=(0.0, 0.0, 0.0), **kw):
    """The oracle's constants set to the float32 values the library uses."""
    d = dict(L=L, tile=tile, z_near=F32(0.2), g_min=2.0 ** -15, t_min=2.0 ** -15, alpha_max=F32(0.99),
             dilation=F32(0.3), r_ref=F32(1e-2), bg=tuple(F32(b) for b in bg))
    d.update(kw)
    return oracle.Config(**d)


def run_gpu(scene, cams, tile=16, L=4, bg=(0.0, 0.0, 0.0), grad_images=None, renderer=None, lean=False, **cfg):
    """Forward (and optionally backward) through the C ABI; returns host arrays
    (with lean=True only the images, index map and pixel flags of the state)."""
    import torch
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    dev = torch.device("cuda", 0)
    r = renderer or Renderer(0, tile=tile, tess_level=L, bg=bg, **cfg)
    params = scene_tensors(scene, dev)
    camt = torch.from_numpy(cams.cams).to(dev)
    wh = np.ascontiguousarray(cams.wh, dtype=np.int32)
    images, state = r.forward(scene.degree, params, camt, wh)
    torch.cuda.synchronize()
    lay = r.layout(scene.degree, params, camt, wh)
    N = cams.num_pixels

    def sec(name, dtype, count):  # one state section, copied to the host
        o = lay[name]
        return state[o:o + np.dtype(dtype).itemsize * count].cpu().numpy().view(dtype)

    ntiles = sum(((int(w) + tile - 1) // tile) * ((int(h) + tile - 1) // tile) for w, h in cams.wh)
    m = int(cfg.get("lattice", 0))        # lattice variant: records of the lattice Gaussians follow the pixels'
    NL = (L * (m - 1) + 1) * (L * (m - 1) + 2) // 2 if m >= 2 else 0
    NR = N + cams.n_views * scene.num_prims * NL
    out = dict(images=images.cpu().numpy().astype(np.float64), I_tri=sec("I_tri", np.int32, N),
               pflags=sec("pflags", np.uint8, N))
    if not lean:
        out.update(I_uv=sec("I_uv", np.float32, 2 * N).reshape(N, 2), rec=sec("rec", np.float32, 16 * NR).reshape(NR, 16), gkey=sec("gkey", np.uint64, NR),
                   T_final=sec("T_final", np.float32, N), last=sec("last", np.int32, N),
                   g_count=sec("g_count", np.int32, ntiles), g_start=sec("g_start", np.int32, ntiles),
                   b_count=sec("b_count", np.int32, ntiles), b_start=sec("b_start", np.int32, ntiles))
        gtot = int(out["g_start"][-1] + out["g_count"][-1]) if ntiles else 0
        btot = int(out["b_start"][-1] + out["b_count"][-1]) if ntiles else 0
        out["g_list"] = sec("g_list", np.uint32, gtot).astype(np.int64)
        out["b_list"] = sec("b_list", np.uint32, btot).astype(np.int64)
    status, counters = r.query(state)
    out["counters"] = counters
    out["status"] = status
    if grad_images is not None:
        gi = torch.from_numpy(np.ascontiguousarray(grad_images, dtype=np.float32)).to(dev)
        grads = r.backward(scene.degree, params, camt, wh, images, gi, state)
        torch.cuda.synchronize()
        out["grads"] = {k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()}
    return out


def oracle_frames(scene, cams, cfg):
    return [oracle.Frame(scene, cams.cams[v], int(cams.wh[v, 0]), int(cams.wh[v, 1]), cfg)
            for v in range(cams.n_views)]


def view_offsets(cams):
    n = cams.wh[:, 0].astype(np.int64) * cams.wh[:, 1]
    return np.concatenate([[0], np.cumsum(n)])


def tile_offsets(cams, tile):
    n = [((int(w) + tile - 1) // tile) * ((int(h) + tile - 1) // tile) for w, h in cams.wh]
    return np.concatenate([[0], np.cumsum(n)])


def l1_cotangent(image, target):
    return np.sign(image - target) / image.size


def grad_error(g, ref):
    """Worst absolute error relative to the tensor's largest reference entry."""
    scale = np.abs(ref).max()
    return float(np.abs(g - ref).max() / scale) if scale > 0 else float(np.abs(g).max())


# Per-element gradient tolerance: |g - ref| <= GRAD_REL * max(|ref|, GRAD_FLOOR
# * max|ref|) for every element of a tensor.  Entries at least 1/20 of the
# tensor's largest are held to 1e-3 of themselves; smaller ones to 5e-5 of the
# largest.  The floor is set by the discrete cut-offs of the rendering (the
# support G >= g_min and the stop at T < T_min, both 2^-15): where FP32 and
# FP64 fall on different sides of one, a pixel's term moves by up to about
# 3e-5 of its size, and an entry whose terms cancel keeps that as an absolute
# error of up to about 3e-5 of the largest entries.
GRAD_REL = 1e-3
GRAD_FLOOR = 5e-2


def grad_rel_error(g, ref, floor=GRAD_FLOOR):
    """Worst per-element relative error |g - ref| / max(|ref|, floor max|ref|)."""
    g, ref = np.asarray(g, np.float64).reshape(-1), np.asarray(ref, np.float64).reshape(-1)
    scale = np.abs(ref).max(initial=0.0)
    if scale == 0:
        return float(np.abs(g).max(initial=0.0))
    return float((np.abs(g - ref) / np.maximum(np.abs(ref), floor * scale)).max())


def check_grads(got, ref, tol=GRAD_REL, skip=()):
    """Assert both gradient measures for every array: the worst error over
    the tensor's largest entry, and the per-element relative error above."""
    for k in ref:
        if k in skip:
            continue
        g, r = np.asarray(got[k], np.float64).reshape(ref[k].shape), ref[k]
        e, el = grad_error(g, r), grad_rel_error(g, r)
        log(f"    {k}: max err / max|ref| = {e:.2e}, per element {el:.2e}  (max|ref| {np.abs(r).max():.2e})")
        assert e <= tol and el <= tol, (k, e, el)
