"""Summaries of rocprofv3 runs of the renderer (kernel trace and counters).

    python -m paper_2503_13961_amd.profiling --workload NAME --command "..." \
        --trace DIR [--fetch DIR --write DIR] [--counters DIR ...] --md OUT.md

DIR is a rocprofv3 output directory written with ``--output-format csv``
(``*_kernel_stats.csv`` / ``*_kernel_trace.csv`` for the trace,
``*_counter_collection.csv`` for ``--pmc``).  The FETCH_SIZE and WRITE_SIZE
passes are calibrated with a plain device copy of known size run in the same
process (``bench.py --copy-probe-mb``): the scale of each counter is the
probe's true byte count over what the counter read for it.

The summary ends with one machine-readable line (bytes per dispatch and the
SHA-256 of the library sources), so a reader can tell whether the counters
still describe the kernels it runs (``source_digest()``, ``read_counters()``).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def source_digest() -> str:
    """SHA-256 over the library's HIP/C++ sources and its public header."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*"))) + [os.path.join(ROOT, "include", "bgt.h")]
    for f in files:
        if os.path.isfile(f):
            h.update(os.path.basename(f).encode())
            with open(f, "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def _one(dirname, suffix):
    hits = sorted(glob.glob(os.path.join(dirname, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {dirname}")
    return hits[0]


def _short(name: str) -> str:
    n = name.split("(")[0].replace("void ", "").strip()
    return n


def kernel_stats(trace_dir):
    """{kernel: {calls, avg_us, total_ms, pct}} from a --kernel-trace --stats run."""
    out = {}
    with open(_one(trace_dir, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            out[_short(r["Name"])] = {"calls": int(r["Calls"]), "avg_us": float(r["AverageNs"]) / 1e3,
                                      "total_ms": float(r["TotalDurationNs"]) / 1e6,
                                      "pct": float(r["Percentage"])}
    return out


def counters(pmc_dir):
    """{kernel: {counter: mean per dispatch}} and the per-dispatch rows."""
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    rows = []
    with open(_one(pmc_dir, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            k = _short(r["Kernel_Name"])
            v = float(r["Counter_Value"])
            agg[k][r["Counter_Name"]].append(v)
            rows.append((k, r["Counter_Name"], v, int(r.get("Grid_Size", 0) or 0)))
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in agg.items()}, rows


def probe_scale(rows, counter, probe_bytes):
    """True bytes over the counter's reading for the largest device copy
    (the probe): FETCH for the copy's reads, WRITE for its writes."""
    best = 0.0
    for k, c, v, _ in rows:
        if c == counter and "copyBuffer" in k:
            best = max(best, v)
    return probe_bytes / (best * 1024.0) if best > 0 else None


def summarize(workload, command, trace, fetch=None, write=None, extra=(), probe_mb=1024):
    res = {"workload": workload, "command": command, "source_sha256": source_digest(),
           "kernels": kernel_stats(trace)}
    probe = probe_mb * (1 << 20)
    if fetch:
        fc, frows = counters(fetch)
        res["fetch_scale"] = probe_scale(frows, "FETCH_SIZE", probe)
        for k, d in fc.items():
            if "FETCH_SIZE" in d:
                res["kernels"].setdefault(k, {})["fetch_bytes"] = d["FETCH_SIZE"] * 1024 * (res["fetch_scale"] or 1)
    if write:
        wc, wrows = counters(write)
        res["write_scale"] = probe_scale(wrows, "WRITE_SIZE", probe)
        for k, d in wc.items():
            if "WRITE_SIZE" in d:
                res["kernels"].setdefault(k, {})["write_bytes"] = d["WRITE_SIZE"] * 1024 * (res["write_scale"] or 1)
    for e in extra:
        ec, _ = counters(e)
        for k, d in ec.items():
            res["kernels"].setdefault(k, {}).update(d)
    return res


def markdown(res, focus=("k_blend_bwd", "k_blend_fwd", "k_gen", "k_param_bwd")):
    L = [f"# Kernel profile: {res['workload']}", "",
         "Made by (rocprofv3 writes CSV under the `-d` directory):", "", "```", res["command"], "```", "",
         f"Library sources: sha256 `{res['source_sha256'][:16]}`", ""]
    if res.get("fetch_scale") or res.get("write_scale"):
        L += [f"Counter calibration with a 1 GiB device copy in the same process: FETCH_SIZE x "
              f"{res.get('fetch_scale') or float('nan'):.3f}, WRITE_SIZE x {res.get('write_scale') or float('nan'):.3f}.", ""]
    L += ["| kernel | calls | avg (us) | share of GPU time |", "|---|---|---|---|"]
    ks = sorted(((k, v) for k, v in res["kernels"].items() if "calls" in v), key=lambda kv: -kv[1]["total_ms"])
    for k, v in ks[:20]:
        name = k if len(k) <= 60 else k[:57] + "..."
        L.append(f"| `{name}` | {v['calls']} | {v['avg_us']:.1f} | {v['pct']:.1f}% |")
    rows = [(k, v) for k, v in res["kernels"].items() if any(f in k for f in focus)]
    if rows:
        cols = sorted({c for _, v in rows for c in v if c not in ("calls", "avg_us", "total_ms", "pct")})
        if cols:
            L += ["", "Per dispatch (bytes calibrated as above; SQ counters summed over the GPU):", "",
                  "| kernel | " + " | ".join(cols) + " |", "|---|" + "---|" * len(cols)]
            for k, v in rows:
                cells = []
                for c in cols:
                    x = v.get(c)
                    cells.append("" if x is None else (f"{x / 1e6:.1f} MB" if c.endswith("_bytes") else f"{x:.4g}"))
                L.append(f"| `{k}` | " + " | ".join(cells) + " |")
    # one machine-readable line: bytes per dispatch, for readers that check
    # the source digest before using them
    mach = {"source_sha256": res["source_sha256"], "workload": res["workload"],
            "bytes": {k: {"fetch": v.get("fetch_bytes"), "write": v.get("write_bytes"), "avg_us": v.get("avg_us")}
                      for k, v in res["kernels"].items()
                      if k.startswith("bgt::") and ("fetch_bytes" in v or "write_bytes" in v)},
            "sq": {k: {c: x for c, x in v.items() if c.startswith("SQ_")}
                   for k, v in res["kernels"].items() if k.startswith("bgt::") and any(c.startswith("SQ_") for c in v)}}
    L += ["", "<!-- counters " + json.dumps(mach, sort_keys=True) + " -->"]
    return "\n".join(L) + "\n"


def read_counters(md_path):
    """The machine-readable line of a summary written by markdown(), or None."""
    try:
        with open(md_path) as f:
            for line in f:
                if line.startswith("<!-- counters "):
                    return json.loads(line[len("<!-- counters "):].rsplit("-->", 1)[0])
    except OSError:
        return None
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--counters", nargs="*", default=[])
    ap.add_argument("--probe-mb", type=int, default=1024)
    ap.add_argument("--md", required=True)
    a = ap.parse_args()
    res = summarize(a.workload, a.command, a.trace, a.fetch, a.write, a.counters, a.probe_mb)
    with open(a.md, "w") as f:
        f.write(markdown(res))


if __name__ == "__main__":
    main()
