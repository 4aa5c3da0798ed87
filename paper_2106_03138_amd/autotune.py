"""Autotuner of the batched launch: for each size class (by m: <= 64, <= 128,
<= 256, <= 512) pick the kernel variant and workgroups per compute unit with
the lowest measured time on a synthetic batch of that class, and cache the
choice as JSON per device.

    python -m paper_2106_03138_amd.autotune [--count 512] [--out PATH]

The variants change only how the work is laid out (threads per workgroup,
columns per wavefront in the trailing update, whether the panel rows sit in
registers, concurrency), never the factorization's decisions: they differ in
summation order only, so tuning cannot change what is computed beyond rounding.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import _lib
from .api import Batch, BatchPlan
from . import inputs as I

CLASS_BOUNDS = [(32, 64), (65, 128), (129, 256), (257, 512)]
CANDIDATES = [(v, w) for v in (0, 1, 2) for w in (0, 1, 2)]
DEFAULT = [(0, 0), (0, 0), (1, 0), (1, 0)]
HERE = os.path.dirname(os.path.abspath(__file__))


def cache_path(device_name: str) -> str:
    """tuned/<device>.json beside the package (overridable with QRDM_TUNE_CACHE)."""
    env = os.environ.get("QRDM_TUNE_CACHE")
    if env:
        return env
    safe = "".join(ch if ch.isalnum() else "_" for ch in device_name)
    return os.path.join(HERE, "tuned", f"{safe}.json")


def _device_name():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def load(device_name: str | None = None):
    """The cached per-class choice [(variant, wgs_per_cu)] * 4, or the defaults."""
    try:
        path = cache_path(device_name or _device_name())
        with open(path) as f:
            d = json.load(f)
        return [tuple(d["classes"][i]["choice"]) for i in range(_lib.BATCH_CLASSES)]
    except (OSError, KeyError, ValueError, IndexError):
        return list(DEFAULT)


def _time_plan(batch, pristine, tune, reps):
    import torch
    plan = BatchPlan(batch, tune=[tune] * _lib.BATCH_CLASSES)
    batch.data.copy_(pristine)
    plan.factor(use_graph=True)  # capture + warm up
    times = []
    for _ in range(reps):
        batch.data.copy_(pristine)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.factor(use_graph=True)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    plan.close()
    return float(np.median(times))


def tune(count: int = 512, reps: int = 3, seed: int = 1, verbose: bool = True):
    """Measure every candidate for every class; returns the JSON-ready record."""
    import torch
    torch.cuda.init()
    rec = {"device": _device_name(), "count_per_class": count, "reps": reps, "classes": []}
    for c, (lo, hi) in enumerate(CLASS_BOUNDS):
        mats, shapes = I.batch(count, seed=seed + c, mmin=lo, mmax=hi, nmin=min(16, lo))
        b = Batch([(m, n) for m, n, _ in shapes])
        b.load(mats)
        pristine = b.data.clone()
        res = []
        for cand in CANDIDATES:
            ms = _time_plan(b, pristine, cand, reps)
            res.append({"variant": cand[0], "wgs_per_cu": cand[1], "ms": round(ms, 4)})
            if verbose:
                print(f"class {c} (m {lo}..{hi}) variant {cand[0]} wgs/cu {cand[1]}: {ms:.3f} ms", flush=True)
        best = min(res, key=lambda r: r["ms"])
        rec["classes"].append({"m_range": [lo, hi], "choice": [best["variant"], best["wgs_per_cu"]],
                               "results": res})
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    _lib.load()
    t0 = time.time()
    rec = tune(args.count, args.reps)
    rec["seconds"] = round(time.time() - t0, 1)
    out = args.out or cache_path(rec["device"])
    os.makedirs(os.path.dirname(out), exist_ok=True)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
