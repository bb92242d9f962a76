#!/usr/bin/env python
"""Throughput of the BG-Triangle rasterizer (forward + backward) on one MI355X.

A step is one pass of the whole path over one batch: tessellation, raster,
sub-primitive generation, tile binning, discontinuity-aware blending, the
L1-loss cotangent and the backward pass to every BG-Triangle parameter.
Workload: the 2000-patch deformed sphere seen by 16 cameras on a sphere of
radius 3 at 800x800 (10.24 Mpx per step), all views in one batched launch
sequence captured in a hipGraph.  The same kernels launched view after view
are timed beside it.  Inputs are resident in HBM before the timed region.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpixels/s at 800×800, 16 views batched vs per-view, at 1e-4 error"
IMG_TOL, GRAD_TOL = 1e-4, 1e-3
GRAD_FLOOR = 5e-2  # per-element gradient error is relative to max(|ref|, GRAD_FLOOR * max|ref|)
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile", default="auto", help="8, 16, 32 or auto (the autotuner picks tile and batch)")
    ap.add_argument("--batch", type=int, default=64, help="Gaussians per LDS batch when --tile is given")
    ap.add_argument("--workload", default="sphere2k_16v_800")
    ap.add_argument("--lattice", type=int, default=0,
                    help="time the lattice variant with this many Gaussians per sub-triangle edge (for profiling)")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip timing the variant without blending coefficients")
    ap.add_argument("--no-densify", action="store_true", help="skip timing the splitting-and-pruning kernels")
    ap.add_argument("--no-train-step", action="store_true",
                    help="skip timing the optimisation step (fwd + Eq. 9 loss + bwd + Adam)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip timing the other configurations")
    ap.add_argument("--cpu-views", type=int, default=16, help="views in the oracle's timed sample")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the batched graph replays (for rocprofv3); prints the JSON line")
    ap.add_argument("--eager", action="store_true",
                    help="with --profile-run: launch the steps eagerly instead of replaying the graph")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first run a plain device-to-device copy of this many MiB (counter calibration)")
    return ap.parse_args()


class Step:
    """Pre-allocated buffers and the launch sequence of one fwd+bwd step."""

    def __init__(self, renderer, degree, params, camt, wh, target):
        import torch
        from paper_2503_13961_amd import native as N
        self.torch, self.N = torch, N
        self.r, self.degree, self.params, self.camt, self.wh = renderer, degree, params, camt, wh
        self.npx = int((wh[:, 0].astype(np.int64) * wh[:, 1]).sum())
        dev = camt.device
        self.images = torch.empty((self.npx, 3), dtype=torch.float32, device=dev)
        self.gimg = torch.empty_like(self.images)
        self.target = target
        self.grads = {k: torch.empty_like(v) for k, v in params.items()}
        # size the state (and its pair capacities) with a checked eager pass
        _, self.state = renderer.forward(degree, params, camt, wh, images=self.images, check=True)

    def __call__(self):
        torch = self.torch
        self.r.forward(self.degree, self.params, self.camt, self.wh, state=self.state, images=self.images,
                       check=False)
        self.N.bgt_l1_cotangent(self.r.ctx, self.gimg.numel(), self.images.data_ptr(), self.target.data_ptr(),
                                1.0 / self.gimg.numel(), self.gimg.data_ptr(), torch.cuda.current_stream().cuda_stream)
        self.r.backward(self.degree, self.params, self.camt, self.wh, self.images, self.gimg, self.state,
                        grads=self.grads)


class PerViewStep:
    """The same kernels launched once per view (16 separate pipelines)."""

    def __init__(self, renderer, degree, params, camt, wh, target):
        import torch
        self.torch = torch
        off = np.concatenate([[0], np.cumsum(wh[:, 0].astype(np.int64) * wh[:, 1])])
        self.steps = [Step(renderer, degree, params, camt[v:v + 1].contiguous(), wh[v:v + 1].copy(),
                           target[off[v]:off[v + 1]]) for v in range(len(wh))]
        self.grads = {k: torch.empty_like(v) for k, v in params.items()}
        self.npx = int(off[-1])

    def __call__(self):
        torch = self.torch
        for s in self.steps:
            s.r.forward(s.degree, s.params, s.camt, s.wh, state=s.state, images=s.images, check=False)
        for s in self.steps:
            s.N.bgt_l1_cotangent(s.r.ctx, s.gimg.numel(), s.images.data_ptr(), s.target.data_ptr(),
                                 1.0 / (3 * self.npx), s.gimg.data_ptr(), torch.cuda.current_stream().cuda_stream)
        for g in self.grads.values():
            g.zero_()
        for s in self.steps:
            s.r.backward(s.degree, s.params, s.camt, s.wh, s.images, s.gimg, s.state, grads=s.grads)
            for k, g in self.grads.items():
                g.add_(s.grads[k])


def capture(step):
    import torch
    step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    return g


def time_replays(g, steps, warmup):
    import torch
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def stage_profile(step, n=5):
    """Per-stage kernel durations (ms) from the library's HIP events, eager."""
    import torch
    from paper_2503_13961_amd import native as N
    r = step.r
    N.bgt_profile(r.ctx, True)
    acc = None
    for _ in range(n):
        step()
        t = N.bgt_stage_times(r.ctx)
        acc = t if acc is None else {k: acc[k] + t[k] for k in acc}
    N.bgt_profile(r.ctx, False)
    torch.cuda.synchronize()
    return {k: v / n for k, v in acc.items()}


def algorithmic(counters, npx, ntiles, P, ncp):
    """Algorithmic HBM bytes of each blend kernel per launch (each essential
    read or write counted once):
      forward : per Gaussian pair 4 B list entry + 48 B record (mean offset,
                conic, colour, opacity, id, pixel range); per boundary pair
                4 B + 16 B (position, radius, id); per pixel 4 B id read,
                12 B image, 4 B transmittance, 4 B stop index written;
                per tile 16 B of list ranges.
      backward: the forward's reads again, plus per pixel 12 B image and
                12 B cotangent read, per Gaussian pair its 36 B of sums
                written (9 floats), per boundary pair a 12 B gradient
                read-modify-write."""
    gp, bp = counters[1], counters[2]
    fwd = gp * (4 + 48) + bp * (4 + 16) + npx * (4 + 12 + 4 + 4) + ntiles * 16
    bwd = gp * (4 + 48 + 36) + bp * (4 + 16 + 2 * 12) + npx * (4 + 4 + 12 + 12) + ntiles * 16
    return {"blend_fwd": fwd, "blend_bwd": bwd}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and its logical CPU count."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name or platform.processor() or platform.machine(), os.cpu_count()


def oracle_config(**mode):
    """The oracle's constants at the float32 values the library uses."""
    import oracle
    return oracle.Config(z_near=float(np.float32(0.2)), alpha_max=float(np.float32(0.99)),
                         dilation=float(np.float32(0.3)), r_ref=float(np.float32(1e-2)), **mode)


def reference_leg(scene, cams, images, grads, target, scale, nviews):
    """The FP64 oracle on the first `nviews` views of the workload, forward and
    backward: every pixel of its image, and the dense gradient of the timed
    step's L1 loss with the oracle's own cotangent sign(C - target) * scale.
    Its forward + backward time is the CPU baseline.  Against it, the timed
    replay's own outputs: every pixel of every view, and (when all views are
    taken) the replay's gradients per element.  The two L1 cotangents differ
    exactly where the target lies between the two images (|C_oracle -
    target| below the image error there); the patches whose Gaussians reach
    those pixels differentiate a different loss on the two sides and are
    left out of the gradient comparison, and counted."""
    import oracle
    cfg = oracle_config()
    off = np.concatenate([[0], np.cumsum(cams.wh[:, 0].astype(np.int64) * cams.wh[:, 1])])
    t_oracle, px, img_err, ref, ambiguous, excluded = 0.0, 0, 0.0, None, 0, set()
    for v in range(nviews):
        W, H = int(cams.wh[v, 0]), int(cams.wh[v, 1])
        sl = slice(off[v], off[v + 1])
        t0 = time.perf_counter()
        fr = oracle.Frame(scene, cams.cams[v], W, H, cfg)
        img = fr.render()[0]
        gi = np.sign(img - target[sl]) * scale
        g = fr.grad(gi)
        t_oracle += time.perf_counter() - t0
        px += W * H
        ref = g if ref is None else {k: ref[k] + g[k] for k in ref}
        err = float(np.abs(images[sl] - img).max())
        img_err = max(img_err, err)
        amb = np.nonzero((np.sign(images[sl] - target[sl]) != np.sign(img - target[sl])).any(axis=1))[0]
        ambiguous += len(amb)
        if len(amb):
            prim = fr.records()[:, oracle.GR["PRIM"]].astype(np.int64)
            for q in amb:
                excluded.update(int(prim[x]) for x in fr.trace(int(q))[0])
        del fr
    cores = oracle.num_threads()
    cpu, logical = cpu_model()
    out = {"cpu_baseline": {"value": px / t_oracle / 1e6, "unit": "Mpixels/s", "cores": cores, "kind": "oracle",
                            "sample": f"{nviews} of the {cams.n_views} views ({px} px), forward + backward, FP64, "
                                      f"OpenMP", "seconds": round(t_oracle, 3), "cpu": cpu,
                            "logical_cpus": logical},
           "image_max_abs_err": img_err, "image_pixels_checked": px}
    if nviews == cams.n_views and grads is not None:
        P = scene.num_prims
        keep = np.ones(P, bool)
        keep[sorted(excluded)] = False
        gr = {}
        for k, r in ref.items():
            got = np.asarray(grads[k], np.float64).reshape(r.shape)
            scale_k = np.abs(r).max()
            err = np.abs(got - r) / max(scale_k, 1e-300)
            rel = np.abs(got - r) / np.maximum(np.abs(r), GRAD_FLOOR * scale_k)
            gr[k] = {"max_err_over_max": float(err[..., keep].max(initial=0.0)),
                     "per_element_rel": float(rel[..., keep].max(initial=0.0)),
                     "max_err_over_max_incl_excluded": float(err.max(initial=0.0))}
        out["grads"] = gr
        out["ambiguous_channels"] = int(ambiguous)
        out["patches_excluded"] = int((~keep).sum())
    return out


def profiled(workload, kernel):
    """(HBM bytes, SQ counters) per launch of `kernel` from the committed
    rocprofv3 summary of this workload; (None, {}) when there is none or the
    library sources changed since it was taken."""
    from paper_2503_13961_amd import profiling
    m = profiling.read_counters(os.path.join(ROOT, "profiles", f"kernels_{workload}.md"))
    if not m or m.get("source_sha256") != profiling.source_digest():
        return None, {}
    b = m.get("bytes", {}).get(kernel) or {}
    traffic = None if b.get("fetch") is None or b.get("write") is None else b["fetch"] + b["write"]
    return traffic, m.get("sq", {}).get(kernel, {})


def copy_bandwidth(dev, mib=1024, reps=5):
    """Device-to-device copy of `mib` MiB, read + written bytes per second (GB/s)."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def path_bytes(counters, npx, ntiles, backward=True):
    """Algorithmic HBM bytes of one whole fwd+bwd step, each buffer the method
    must produce or consume counted once per essential read or write: per
    pixel the index map and (u, v) written and read, image, transmittance
    and stop index written, the backward's reads; per foreground pixel its
    Gaussian written; per boundary pixel its list entries, record and
    gradient (read back by the parameter pass); per Gaussian-tile pair the key
    emitted, sorted, the value and the record read in the forward and again
    in the backward, with its 36 bytes of sums written there and read by the
    parameter pass; per boundary pair the same with its 16-byte record and a
    12-byte gradient read-modify-write; per tile its list ranges."""
    gp, bp, fg, nb = counters[1], counters[2], counters[3], counters[4]
    fwd = npx * (12 + 12 + 20) + fg * 44 + nb * (4 + 4 + 16) + gp * (12 + 24 + 4 + 44) + bp * (12 + 24 + 4 + 16) \
        + ntiles * 24
    bwd = npx * 24 + nb * (24 + 12) + gp * (4 + 44 + 2 * 36) + bp * (4 + 16 + 24)
    return fwd + (bwd if backward else 0)


def parity_check(scene, cams, images, samples=6000, seed=0, views=None, **mode):
    """Image parity of the timed replay's output on sampled pixels of every
    view (or of `views`); `mode` sets the oracle's variant (e.g. lattice=4)."""
    import oracle
    cfg = oracle_config(**mode)
    rng = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(cams.wh[:, 0].astype(np.int64) * cams.wh[:, 1])])
    worst = 0.0
    for v in (range(cams.n_views) if views is None else views):
        W, H = int(cams.wh[v, 0]), int(cams.wh[v, 1])
        fr = oracle.Frame(scene, cams.cams[v], W, H, cfg)
        pix = rng.choice(W * H, size=min(samples // cams.n_views, W * H), replace=False).astype(np.int32)
        ref = fr.render(pix)[0]
        worst = max(worst, float(np.abs(images[off[v] + pix] - ref).max()))
    return worst


class ForwardStep:
    """The forward pass alone (all stages up to the image)."""

    def __init__(self, renderer, degree, params, camt, wh):
        self.r, self.degree, self.params, self.camt, self.wh = renderer, degree, params, camt, wh
        self.npx = int((wh[:, 0].astype(np.int64) * wh[:, 1]).sum())
        self.images, self.state = renderer.forward(degree, params, camt, wh, check=True)

    def __call__(self):
        self.r.forward(self.degree, self.params, self.camt, self.wh, state=self.state, images=self.images,
                       check=False)


# The workload list's configurations, each timed at its own size (the metric
# line above is the 16 x 800^2 batch) with the (tile, batch) the autotuner
# picks: (name, forward only, autotuner candidates ("all" or a list), views
# whose every pixel is checked against the oracle (None: all), sampled
# pixels in each other view)
CONFIGS = [
    ("random64", True, "all", None, 0),
    ("sphere2k_1v", False, "all", None, 0),
    ("sphere2k_16v_mixed", False, "all", None, 0),
    ("box20k_cubic", False, "all", None, 0),
    ("sphere50k_32v", False, [(8, 64), (16, 64), (32, 64)], [0], 1500),
]


def time_configs(dev, steps, warmup, parity=True):
    """Mpixels/s, HBM fraction of the algorithmic bytes and image parity of
    every configuration of the workload list (the last one autotuned over
    tile sizes 8, 16 and 32)."""
    import torch
    from paper_2503_13961_amd import scenes as S
    from paper_2503_13961_amd.render import Renderer, scene_tensors
    out = {}
    for name, fwd_only, cands, full_views, per_view in CONFIGS:
        scene, cams, desc = S.workload(name)
        params = scene_tensors(scene, dev)
        camt = torch.from_numpy(cams.cams).to(dev)
        wh = np.ascontiguousarray(cams.wh, dtype=np.int32)
        rec = {"what": desc + (", forward only" if fwd_only else ", forward + L1 cotangent + backward")}
        if cands:
            from paper_2503_13961_amd.autotune import CANDIDATES, autotune
            tune = autotune(scene.degree, params, camt, wh, candidates=CANDIDATES if cands == "all" else cands,
                            cache=False)
            tile, batch = tune["tile"], tune["batch"]
            rec["autotune_ms"] = {k: round(v, 4) for k, v in tune["timings"].items()}
        else:
            tile, batch = 16, 64
        r = Renderer(0, tile=tile, batch=batch)
        if fwd_only:
            step = ForwardStep(r, scene.degree, params, camt, wh)
        else:
            step = Step(r, scene.degree, params, camt, wh, torch.from_numpy(S.l1_target(cams.num_pixels)).to(dev))
        _, counters = r.query(step.state)
        g = capture(step)
        ms = time_replays(g, steps, warmup)
        npx = step.npx
        ntiles = sum(((int(w) + tile - 1) // tile) * ((int(h) + tile - 1) // tile) for w, h in wh)
        pb = path_bytes(counters, npx, ntiles, backward=not fwd_only)
        rec.update({"views": int(cams.n_views), "pixels": npx, "prims": scene.num_prims, "degree": scene.degree,
                    "tile": tile, "batch": batch, "ms_per_step": round(ms, 4),
                    "value": round(npx / (ms * 1e-3) / 1e6, 2), "unit": "Mpixels/s",
                    "algorithmic_bytes": int(pb), "hbm_frac": round(pb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
        if parity:
            img = step.images.detach().cpu().numpy()
            views = range(cams.n_views) if full_views is None else full_views
            err = full_frame_error(scene, cams, img, views)
            rec["image_max_abs_err_full_views"] = err
            rec["full_views"] = len(views)
            if per_view:
                rest = [v for v in range(cams.n_views) if v not in set(views)]
                es = parity_check(scene, cams, img, samples=per_view * cams.n_views, views=rest)
                rec["image_max_abs_err_sampled"] = es
                rec["sampled"] = f"{per_view} px in each of the other {len(rest)} views"
                err = max(err, es)
            rec["image_ok"] = bool(err <= IMG_TOL)
        log(f"[bench] config {name}: {rec}")
        out[name] = rec
        del g, step, r
        torch.cuda.synchronize()
    return out


def full_frame_error(scene, cams, images, views):
    """Largest |image - oracle| over every pixel of the given views."""
    import oracle
    cfg = oracle_config()
    off = np.concatenate([[0], np.cumsum(cams.wh[:, 0].astype(np.int64) * cams.wh[:, 1])])
    worst = 0.0
    for v in views:
        W, H = int(cams.wh[v, 0]), int(cams.wh[v, 1])
        fr = oracle.Frame(scene, cams.cams[v], W, H, cfg)
        worst = max(worst, float(np.abs(images[off[v]:off[v + 1]] - fr.render()[0]).max()))
        del fr
    return worst


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(views would shard across GPUs with one all-reduce of the parameter gradients).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2503_13961_amd import scenes as S
    from paper_2503_13961_amd.render import Renderer, scene_tensors

    dev = torch.device("cuda", 0)
    scene, cams, desc = S.workload(args.workload)
    if args.lattice:
        scene = S.lattice_scaled(scene, m=args.lattice, L=4)
        desc += f", lattice variant m={args.lattice}"
    log(f"[bench] {desc}")
    params = scene_tensors(scene, dev)
    camt = torch.from_numpy(cams.cams).to(dev)
    wh = np.ascontiguousarray(cams.wh, dtype=np.int32)
    target = torch.from_numpy(S.l1_target(cams.num_pixels)).to(dev)
    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {args.copy_probe_mb} MiB read + written")
        del src, dst
    tune = None
    if args.tile == "auto":
        from paper_2503_13961_amd.autotune import autotune
        tune = autotune(scene.degree, params, camt, wh, cache=False)
        tile, batch = tune["tile"], tune["batch"]
        log(f"[bench] autotuned tile {tile}, batch {batch} in {tune['seconds']} s: {tune['timings']}")
    else:
        tile, batch = int(args.tile), args.batch
    r = Renderer(0, tile=tile, batch=batch, lattice=args.lattice)
    step = Step(r, scene.degree, params, camt, wh, target)
    if args.profile_run and args.eager:
        for _ in range(args.warmup + args.steps):
            step()
        torch.cuda.synchronize()
        log("[bench] eager profile steps done")
        print(json.dumps({"profile_run": "eager", "steps": args.steps + args.warmup}), flush=True)
        return
    st, counters = r.query(step.state)
    log(f"[bench] counters {counters}")
    g = capture(step)
    log("[bench] graph captured")
    ms = time_replays(g, args.steps, args.warmup)
    npx = step.npx
    value = npx / (ms * 1e-3) / 1e6
    log(f"[bench] batched: {ms:.3f} ms/step, {value:.1f} Mpix/s")
    out = {"metric": METRIC, "value": round(value, 2), "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"{args.workload}: {desc}", "views": int(cams.n_views),
                      "width": int(wh[0, 0]), "height": int(wh[0, 1]), "pixels": npx,
                      "prims": scene.num_prims, "degree": scene.degree, "tile": tile, "batch": batch,
                      "autotuned": tune is not None, "batched": True, "hipgraph": True}}
    if tune is not None:
        out["autotune_ms"] = {k: round(v, 4) for k, v in tune["timings"].items()}
    images_batched = step.images.detach().cpu().numpy()
    grads_batched = {k: v.detach().cpu().numpy() for k, v in step.grads.items()}  # the replay's own gradients
    if args.profile_run:
        print(json.dumps(out), flush=True)
        return
    if not args.no_per_view:
        pv = PerViewStep(Renderer(0, tile=tile, batch=batch), scene.degree, params, camt, wh, target)
        gpv = capture(pv)
        ms_pv = time_replays(gpv, args.steps, args.warmup)
        imgs_pv = torch.cat([s.images for s in pv.steps]).cpu().numpy()
        same = bool(np.array_equal(imgs_pv, images_batched))
        gdiff = max(float((pv.grads[k] - step.grads[k]).abs().max() / step.grads[k].abs().max().clamp_min(1e-30))
                    for k in step.grads)
        out["per_view"] = {"ms_per_step": round(ms_pv, 4), "value": round(npx / (ms_pv * 1e-3) / 1e6, 2),
                           "batched_speedup": round(ms_pv / ms, 3), "images_bitwise_equal": same,
                           "grad_max_rel_diff": gdiff}
        log(f"[bench] per-view: {ms_pv:.3f} ms/step; images equal {same}; grad diff {gdiff:.2e}")
        del pv, gpv
    if not args.no_variants:
        # each variant with the (tile, batch) the autotuner picks for it (with
        # --tile given, the main step's)
        def variant_config(degree, vparams, **config):
            if args.tile != "auto":
                return tile, batch, None
            from paper_2503_13961_amd.autotune import autotune
            tv = autotune(degree, vparams, camt, wh, cache=False, **config)
            return tv["tile"], tv["batch"], {k: round(v, 4) for k, v in tv["timings"].items()}

        # the ablation variant without blending coefficients (w = 1): same
        # scene and kernels, no boundary points, lists or gamma* maps
        from paper_2503_13961_amd import native as N
        vt, vb, vtune = variant_config(scene.degree, params, flags=N.BGT_FLAG_NO_BOUNDARY)
        vs = Step(Renderer(0, tile=vt, batch=vb, flags=N.BGT_FLAG_NO_BOUNDARY), scene.degree, params, camt, wh,
                  target)
        gv = capture(vs)
        ms_v = time_replays(gv, args.steps, args.warmup)
        out["variants"] = {"no_boundary": {"ms_per_step": round(ms_v, 4), "value": round(npx / (ms_v * 1e-3) / 1e6, 2),
                                           "tile": vt, "batch": vb, "autotune_ms": vtune,
                                           "what": "w = 1 for every Gaussian (ablation w/o B)"}}
        log(f"[bench] variant without blending coefficients: {ms_v:.3f} ms/step (tile {vt}, batch {vb})")
        del vs, gv
        # the paper's full model: resolution-3 rotation and scale maps, SH colour of degree 3
        full = S.with_attributes(scene, attr_res=3, sh_degree=3)
        fparams = scene_tensors(full, dev)
        vt, vb, vtune = variant_config(full.degree, fparams)
        vs = Step(Renderer(0, tile=vt, batch=vb), full.degree, fparams, camt, wh, target)
        gv = capture(vs)
        ms_v = time_replays(gv, args.steps, args.warmup)
        ast = stage_profile(vs)
        out["variants"]["attr_maps_r3_sh3"] = {
            "ms_per_step": round(ms_v, 4), "value": round(npx / (ms_v * 1e-3) / 1e6, 2),
            "tile": vt, "batch": vb, "autotune_ms": vtune,
            "stage_ms": {k: round(v, 4) for k, v in ast.items()},
            "what": "resolution-3 rotation and scale maps and degree-3 SH colour (the paper's full model)"}
        log(f"[bench] variant with resolution-3 maps and SH degree 3: {ms_v:.3f} ms/step (tile {vt}, batch {vb})")
        del vs, gv
        # the lattice variant: m = 4 Gaussians per flat sub-triangle edge
        # (91 per patch and view) in place of the per-pixel Gaussians, sized
        # to the lattice spacing; the image of the last replay is checked on
        # sampled pixels of four views
        lat = S.lattice_scaled(scene, m=4, L=4)
        lparams = scene_tensors(lat, dev)
        vt, vb, vtune = variant_config(lat.degree, lparams, lattice=4)
        vs = Step(Renderer(0, tile=vt, batch=vb, lattice=4), lat.degree, lparams, camt, wh, target)
        gv = capture(vs)
        ms_v = time_replays(gv, args.steps, args.warmup)
        _, lc = vs.r.query(vs.state)
        lst = stage_profile(vs)
        lerr = None
        if not args.no_parity:
            lerr = parity_check(lat, cams, vs.images.detach().cpu().numpy(), samples=4000,
                                views=range(0, cams.n_views, max(1, cams.n_views // 4)), lattice=4)
        out["variants"]["lattice_m4"] = {
            "ms_per_step": round(ms_v, 4), "value": round(npx / (ms_v * 1e-3) / 1e6, 2),
            "tile": vt, "batch": vb, "autotune_ms": vtune,
            "gaussians": int(cams.n_views * scene.num_prims * 91), "gauss_pairs": int(lc[1]),
            "image_max_abs_err_sampled": lerr, "stage_ms": {k: round(v, 4) for k, v in lst.items()},
            "what": "4 Gaussians per flat sub-triangle edge (91 per patch and view) instead of one per pixel, "
                    "log-scales set to 0.6 x the lattice spacing"}
        log(f"[bench] lattice variant: {ms_v:.3f} ms/step (tile {vt}, batch {vb}), {lc[1]} pairs, "
            f"sampled image err {lerr}")
        del vs, gv
    if not args.no_train_step:
        # one optimisation iteration of Sec. 3.3 on the same views: forward,
        # Eq. 9 (L2 + D-SSIM) against the target images, backward, Adam
        from paper_2503_13961_amd.train import TrainStep

        class FixedSceneTrainStep(TrainStep):
            """Restores the parameters before each step, so that every timed
            replay renders the workload's scene (the random target would
            otherwise drive the scales and opacities away from it)."""

            def __call__(self):
                for k, v in params.items():
                    self.params[k].copy_(v)
                return super().__call__()

        ts = FixedSceneTrainStep(Renderer(0, tile=tile, batch=batch), scene.degree,
                                 {k: v.clone() for k, v in params.items()}, camt, wh, target)
        gt = capture(ts)
        ms_t = time_replays(gt, args.steps, args.warmup)
        out["training_step"] = {"ms_per_step": round(ms_t, 4), "value": round(npx / (ms_t * 1e-3) / 1e6, 2),
                                "what": "forward + Eq. 9 loss (L2 + D-SSIM) + backward + Adam, one graph; "
                                        "parameters restored from a copy first (six small device copies)"}
        log(f"[bench] training step: {ms_t:.3f} ms")
        del ts, gt
    if not args.no_densify:
        # splitting and pruning: statistics of one rendered batch (every
        # iteration), then the decision and the rebuilt arrays (every few
        # hundred iterations in the paper's schedule)
        from paper_2503_13961_amd import densify as DZ
        pst = DZ.PrimStats(scene.num_prims, dev)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        pst.accumulate(r, scene.degree, params, camt, wh, step.state, target, step.grads)
        e0.record()
        for _ in range(args.steps):
            pst.accumulate(r, scene.degree, params, camt, wh, step.state, target, step.grads)
        e1.record()
        new, action = DZ.densify(r, scene.degree, params, pst)
        e2.record()
        torch.cuda.synchronize()
        acts = np.bincount(action.cpu().numpy(), minlength=3)
        out["densify"] = {"stats_ms": round(e0.elapsed_time(e1) / args.steps, 4),
                          "plan_apply_ms": round(e1.elapsed_time(e2), 4),
                          "keep_split_prune": [int(x) for x in acts], "prims_after": int(new["opacity"].shape[0]),
                          "what": "statistics of one 16-view batch (visibility, texels, edge prior, gradient "
                                  "norms); decision + rebuilt arrays (includes one host read of the count)"}
        log(f"[bench] densify: {out['densify']}")
        del pst, new
    if not args.no_configs:
        out["configs"] = time_configs(dev, args.steps, args.warmup, parity=not args.no_parity)
    stages = stage_profile(step)
    out["stage_ms"] = {k: round(v, 4) for k, v in stages.items()}
    log(f"[bench] stages {out['stage_ms']}")
    ntiles = sum(((int(w) + tile - 1) // tile) * ((int(h) + tile - 1) // tile) for w, h in wh)
    alg = algorithmic(counters, npx, ntiles, scene.num_prims, (scene.degree + 1) * (scene.degree + 2) // 2)
    dom = max(("blend_fwd", "blend_bwd"), key=lambda k: stages[k])
    achieved = alg[dom] / (stages[dom] * 1e-3) / 1e9
    kname = f"bgt::k_{dom}<{tile}, {batch}>"
    traffic, sq = profiled(args.workload, kname)
    issue = 256 * 2.4e9 * stages[dom] * 1e-3   # wave-instruction slots of the launch (one per CU per cycle)
    out["roofline"] = {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": None if traffic is None else round(traffic / 1e9, 4),
                       "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                       "algorithmic_bytes": int(alg[dom]), "kernel_ms": round(stages[dom], 4),
                       "valu_issue_frac": round(sq["SQ_INSTS_VALU"] / issue, 3) if "SQ_INSTS_VALU" in sq else None,
                       "lds_issue_frac": round(sq["SQ_INSTS_LDS"] / issue, 3) if "SQ_INSTS_LDS" in sq else None}
    # the whole step against the HBM roofline, and a measured copy bandwidth
    pb = path_bytes(counters, npx, ntiles)
    cp = copy_bandwidth(dev)
    out["path_roofline"] = {"algorithmic_bytes": int(pb), "achieved": round(pb / (ms * 1e-3) / 1e9, 1),
                            "unit": "GB/s", "frac": round(pb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "copy_gbs_measured": round(cp, 1),
                            "frac_of_copy": round(pb / (ms * 1e-3) / 1e9 / cp, 4)}
    out["counters"] = {"gauss_pairs": counters[1], "boundary_pairs": counters[2], "foreground_px": counters[3],
                       "boundary_px": counters[4]}
    if not (args.no_parity and args.no_cpu_baseline):
        nv = cams.n_views if not args.no_parity else min(args.cpu_views, cams.n_views)
        ref = reference_leg(scene, cams, images_batched, grads_batched, S.l1_target(cams.num_pixels),
                            1.0 / (3 * npx), nv)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = ref["cpu_baseline"]
            log(f"[bench] cpu baseline {ref['cpu_baseline']}")
        if not args.no_parity:
            gw = max(max(v["max_err_over_max"], v["per_element_rel"]) for v in ref["grads"].values())
            out["parity"] = {"image_max_abs_err": ref["image_max_abs_err"], "image_pixels": ref["image_pixels_checked"],
                             "image_tolerance": IMG_TOL, "grads": ref["grads"], "grad_tolerance": GRAD_TOL,
                             "grad_floor": GRAD_FLOOR, "ambiguous_l1_channels": ref["ambiguous_channels"],
                             "patches_excluded": ref["patches_excluded"],
                             "what": "every pixel of the timed replay's images and the replay's own gradients "
                                     "(dense L1 cotangent) against the FP64 oracle; per-element error relative "
                                     "to max(|ref|, floor * max|ref|)",
                             "ok": bool(ref["image_max_abs_err"] <= IMG_TOL and gw <= GRAD_TOL)}
            log(f"[bench] parity: image {ref['image_max_abs_err']:.2e} on {ref['image_pixels_checked']} px; "
                f"gradients {ref['grads']}; excluded patches {ref['patches_excluded']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
