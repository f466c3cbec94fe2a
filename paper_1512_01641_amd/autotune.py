"""Autotuner of the plan's launch parameters.

Times the whole path (score + align through nwm_mine) for candidate values of
each launch parameter in turn (coordinate descent from the current values),
keeps the fastest, and caches the choice per device and workload signature in
a JSON file.  The parameters change launch shapes only: results are the same
for every choice.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

SPACE = {
    "fill_waves_per_cu": [0, 2, 4, 6, 8],
    "merge_waves_per_cu": [0, 8, 16, 24],
    "score_xcd_map": [1, 0],
    "dp_hot_percent": [50, 0, 25, 75],
    # tile shape of the compacted contraction: K words per round (32 or 64)
    "score_kgroup": [1, 2],
    # S staging of the NW fill: LDS ring of 64 x 64 cells per wave with four
    # strips per workgroup (hand-offs in LDS), the same ring one strip per
    # workgroup, or 16 cells per lane in registers
    "fill_staging": [0, 2, 1],
    # source-side expansion: one fused kernel per row tile, or merge + list build
    "expand_fused": [1, 0],
}


def signature(miner) -> str:
    """Device and workload shape: architecture, pairs, log2 of the cells,
    vocabulary, operand precision."""
    props = torch.cuda.get_device_properties(miner.ctx.device)
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    b = miner.batch
    cells = int(np.dot(b.n.astype(np.int64), b.m.astype(np.int64)))
    return "%s|B%d|cells2^%d|V%d|prec%d" % (arch, b.B, round(math.log2(max(cells, 1))), b.V,
                                             miner.plan.prec)


def time_mine(miner, scorer, gap, threshold, reps=5, graph=False) -> float:
    """Median ms of one score + align pass (one warm-up pass first)."""
    dev = miner.ctx.device
    miner.mine(scorer, gap, threshold, graph=graph)
    torch.cuda.synchronize(dev)
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record()
        miner.mine(scorer, gap, threshold, graph=graph)
        e.record()
        e.synchronize()
        out.append(a.elapsed_time(e))
    return float(np.median(out))


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def autotune(miner, scorer, gap: float, threshold: float, space=None, reps: int = 5, cache_path=None,
             min_gain: float = 0.01, graph: bool = True) -> dict:
    """Pick and apply the fastest launch parameters for this miner's plan.

    Times the path the way it is run: by default as the captured graph of
    nwm_mine (its overlapped multi-stream schedule; every parameter change
    recaptures), graph=False for eager launches.  Returns {"params": {...},
    "ms": best time, "cached": bool}.  A value replaces the current best only
    when it is faster by more than min_gain (relative), so timing noise does
    not move the choice."""
    space = SPACE if space is None else space
    plan = miner.plan
    sig = signature(miner)
    cache = _load(cache_path)
    todo = dict(space)
    if sig in cache:
        for k, v in cache[sig]["params"].items():
            if k in space:
                plan.set_param(k, v)
        # a cached choice covers the parameters it names; any parameter added
        # to the search space since is tuned from there
        todo = {k: v for k, v in space.items() if k not in cache[sig]["params"]}
        if not todo:
            return {"params": {k: cache[sig]["params"][k] for k in space}, "ms": cache[sig]["ms"], "cached": True}
    best = {k: plan.get_param(k) for k in space}
    best_ms = time_mine(miner, scorer, gap, threshold, reps, graph=graph)
    for k, values in todo.items():
        for v in values:
            if v == best[k]:
                continue
            plan.set_param(k, v)
            ms = time_mine(miner, scorer, gap, threshold, reps, graph=graph)
            if ms < best_ms * (1.0 - min_gain):
                best_ms, best[k] = ms, v
        plan.set_param(k, best[k])
    if cache_path:
        cache = _load(cache_path)
        cache[sig] = {"params": best, "ms": best_ms}
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return {"params": dict(best), "ms": best_ms, "cached": False}
