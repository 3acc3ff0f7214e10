"""Execution-parameter autotuner.

Times a few training iterations of the caller's own workload for every
candidate setting of the execution options that do not change results
(waves per tile of the forward and backward compositing, HIP-graph replay)
and returns the fastest.  Results are cached on disk, keyed by the device
name and the workload shape.
"""
from __future__ import annotations

import json
import os
import time

import torch

from .train import Trainer, TrainConfig

CANDIDATES = [dict(fwd=0, bwd=2, graph=False), dict(fwd=0, bwd=4, graph=False),
              dict(fwd=4, bwd=2, graph=False), dict(fwd=4, bwd=4, graph=False),
              dict(fwd=0, bwd=2, graph=True), dict(fwd=4, bwd=2, graph=True)]

_DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gsta_autotune.json")


def workload_key(n, degree, height, width, views_per_step) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{dev}|n={n}|D={degree}|{height}x{width}|vb={views_per_step}"


def tune(params0, degree, cams, targets, order, ctx, base_cfg: TrainConfig, iters: int = 30,
         cache_path: str | None = _DEFAULT_CACHE, candidates=None, log=None):
    """Fastest {fwd, bwd, graph} for this workload (timing `iters` iterations each)."""
    n = params0.shape[1]
    key = workload_key(n, degree, cams[0].height, cams[0].width, base_cfg.views_per_step)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        return cache[key]
    best, best_t = None, float("inf")
    timings = []
    for cand in candidates or CANDIDATES:
        if cand["graph"] and base_cfg.views_per_step > 1:
            continue
        ctx.set_waves(fwd=cand["fwd"], bwd=cand["bwd"])
        cfg = TrainConfig(**{**base_cfg.__dict__, "graph": cand["graph"],
                             "device_sched": cand["graph"] or base_cfg.device_sched})
        tr = Trainer(params0, degree, cams, targets, cfg, order, ctx=ctx)
        tr.run(min(len(cams), 32))            # warm-up (captures graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr.run(iters)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / iters
        timings.append((cand, dt))
        if log:
            log(f"autotune {cand}: {dt * 1e3:.3f} ms/iter")
        if dt < best_t:
            best, best_t = cand, dt
    ctx.set_waves(fwd=best["fwd"], bwd=best["bwd"])
    if cache_path:
        cache[key] = best
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            json.dump(cache, open(cache_path, "w"), indent=1)
        except OSError:
            pass
    return best
