"""Tile-size and LDS-batch autotuner for the batched renderer.

The blend kernels come in (tile, batch) variants: 8, 16 or 32 px square
tiles, with 32, 64 or 128 Gaussians staged per LDS batch (at most one per
pixel of the tile).  Which one is fastest depends on the Gaussians' screen
size against the tile (pairs per Gaussian, boundary points per tile) and on
how many tiles there are to fill the chip.  The tuner times one whole
forward + backward per candidate on the caller's own scene and cameras and
keeps the fastest.  Results are cached in a JSON file keyed by the GPU
architecture, the Bezier degree, the patch count and the view sizes; the
scene content is not part of the key, so a cached choice is a good guess for
a scene of the same kind and size, not a measurement of it.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import torch

from .render import Renderer, param_names

CANDIDATES = ((8, 32), (8, 64), (16, 32), (16, 64), (16, 128), (32, 32), (32, 64), (32, 128))


def default_cache_path() -> str:
    return os.environ.get("BGT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "bgt", "autotune.json"))


def shape_key(degree: int, num_prims: int, wh: np.ndarray, device: int = 0) -> str:
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    wh = np.ascontiguousarray(wh, dtype=np.int32).reshape(-1, 2)
    views = hashlib.sha1(wh.tobytes()).hexdigest()[:16]
    return f"{arch}|n{degree}|P{num_prims}|V{len(wh)}|{views}"


def _load(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path, key, entry):
    d = _load(path)
    d[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_candidate(degree, params, cams, wh, tile, batch, device=0, reps=5, warmup=2, seed=0, **config):
    """Median ms of one forward + backward with this (tile, batch), eager."""
    wh = np.ascontiguousarray(wh, dtype=np.int32).reshape(-1, 2)
    r = Renderer(device, tile=tile, batch=batch, **config)
    images, state = r.forward(degree, params, cams, wh, check=True)
    g = torch.Generator(device="cpu").manual_seed(seed)
    # an L1-like cotangent: every pixel replays its whole list
    gi = (torch.randint(0, 2, images.shape, generator=g).float() * 2 - 1).div_(images.numel()).to(images.device)
    grads = {k: torch.empty_like(params[k]) for k in param_names(params)}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * (reps + warmup))]
    for i in range(warmup + reps):
        ev[2 * i].record()
        r.forward(degree, params, cams, wh, state=state, images=images, check=False)
        r.backward(degree, params, cams, wh, images, gi, state, grads=grads)
        ev[2 * i + 1].record()
    torch.cuda.synchronize()
    ms = sorted(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(warmup, warmup + reps))
    del r, state, images, grads
    return ms[len(ms) // 2]


def autotune(degree, params, cams, wh, device=0, candidates=CANDIDATES, reps=5, warmup=2, cache=True,
             cache_path=None, **config) -> dict:
    """Fastest (tile, batch) for this scene shape; returns
    {"tile", "batch", "ms", "timings": {"TxK": ms}, "cached": bool, "seconds"}."""
    wh = np.ascontiguousarray(wh, dtype=np.int32).reshape(-1, 2)
    P = int(params["opacity"].shape[0])
    key = shape_key(degree, P, wh, device)
    if config:  # the renderer's variant (lattice, flags, ...) changes the best choice
        key += "|" + ",".join(f"{k}={config[k]}" for k in sorted(config))
    path = cache_path or default_cache_path()
    if cache:
        hit = _load(path).get(key)
        if hit and (int(hit.get("tile", 0)), int(hit.get("batch", 0))) in set(candidates):
            return dict(hit, cached=True)
    t0 = time.perf_counter()
    timings = {}
    for tile, batch in candidates:
        timings[f"{tile}x{batch}"] = time_candidate(degree, params, cams, wh, tile, batch, device=device, reps=reps,
                                                    warmup=warmup, **config)
    best = min(timings, key=timings.get)
    tile, batch = (int(x) for x in best.split("x"))
    entry = {"tile": tile, "batch": batch, "ms": timings[best], "timings": timings,
             "seconds": round(time.perf_counter() - t0, 3)}
    if cache:
        try:
            _store(path, key, entry)
        except OSError:
            pass  # a read-only home: the choice still holds for this process
    return dict(entry, cached=False)


def tuned_renderer(degree, params, cams, wh, device=0, **kw) -> tuple[Renderer, dict]:
    """A Renderer with the autotuned (tile, batch) and the tuner's record."""
    config = {k: v for k, v in kw.items() if k not in ("candidates", "reps", "warmup", "cache", "cache_path")}
    res = autotune(degree, params, cams, wh, device=device, **kw)
    return Renderer(device, tile=res["tile"], batch=res["batch"], **config), res
