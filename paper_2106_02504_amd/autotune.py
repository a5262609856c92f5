"""Autotuner for batched generation: picks the lanes per segment and the
segment length (generator steps per segment, i.e. draws per lane = 12 *
seg_blocks / lanes) of a Plan by timing the batched launch on the GPU.

Every candidate produces bit-identical values (the tests check this), so the
choice only affects speed.  Results are cached in a JSON file keyed by the
device (architecture name and compute-unit count), the library version and
step kernel, and a coarse signature of the workload (number of requests,
total values and the luxury levels present, each rounded to a power of two),
so a serving loop or a benchmark tunes once per shape.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np
import torch

from . import Plan, lib, step_kernel

DEFAULT_LANES = (1, 2, 4, 8, 16, 32, 64)
DEFAULT_SEG_BLOCKS = (512, 1024, 2048, 4096, 8192)


def cache_path() -> str:
    return os.environ.get("RLX_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "rlx", "autotune.json"))


def signature(requests) -> str:
    n = int(requests.shape[0])
    total = int(requests["count"].sum())
    levels = sorted(set(int(p) for p in np.unique(requests["p"])))

    def p2(v):
        return 0 if v <= 0 else int(round(math.log2(v)))
    return f"n2^{p2(n)}-v2^{p2(total)}-p{'.'.join(map(str, levels))}"


def device_key(device) -> str:
    """Cache key of the device and library: architecture name and compute
    units (the marketing name is generic on this stack), the library version
    and the step kernel the plans will use."""
    pr = torch.cuda.get_device_properties(device)
    arch = getattr(pr, "gcnArchName", "") or torch.cuda.get_device_name(device)
    return f"{arch}|cu{pr.multi_processor_count}|{lib().rlx_version().decode()}|step{step_kernel()}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(doc: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(doc, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home directory only loses the cache


def time_plan(plan: Plan, states: torch.Tensor, out: torch.Tensor, reps: int = 5) -> float:
    """Average milliseconds of one batched launch (HIP events on the
    current stream)."""
    gen = plan.generate_f64 if out.dtype == torch.float64 else plan.generate_u64
    gen(states, out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        gen(states, out)
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(requests, states: torch.Tensor, out: torch.Tensor, lanes=DEFAULT_LANES,
         seg_blocks=DEFAULT_SEG_BLOCKS, reps: int = 5, use_cache: bool = True) -> dict:
    """Return {"lanes", "seg_blocks", "ms", "table"} for these requests: the
    cached pick for the workload signature, or the fastest candidate."""
    key = f"{device_key(states.device)}|{signature(requests)}"
    doc = _load() if use_cache else {}
    if use_cache and key in doc:
        return dict(doc[key], cached=True)
    table = []
    for g in lanes:
        for s in seg_blocks:
            plan = Plan(requests, lanes=g, seg_blocks=s, device=states.device)
            ms = time_plan(plan, states, out, reps)
            plan.close()
            table.append({"lanes": g, "seg_blocks": s, "ms": ms})
    best = min(table, key=lambda r: r["ms"])
    res = {"lanes": best["lanes"], "seg_blocks": best["seg_blocks"], "ms": best["ms"], "table": table,
           "tuned_at": time.time()}
    if use_cache:
        doc[key] = res
        _store(doc)
    return dict(res, cached=False)
