"""Execution-parameter autotuner.

Two levels, both on the caller's own workload and neither changing results:
the library's gsta_autotune times the compositing launch options (forward
waves per tile, the backward variant -- per pixel with 1, 2 or 4 waves per
tile, or per splat -- and the backward segment length) on the
first views of the workload and keeps the fastest on the context; this
module then times whole training iterations eagerly and replayed from HIP
graphs and picks the faster.  Results are cached on disk, keyed by the
device name and the workload shape.
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import _lib
from .core import camera_array, n_rows
from .train import Trainer, TrainConfig

_DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "gsta_autotune.json")


def workload_key(n, degree, height, width, views_per_step) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    return f"{dev}|n={n}|D={degree}|{height}x{width}|vb={views_per_step}"


def apply(ctx, choice: dict):
    ctx.set_waves(fwd=choice["fwd"], bwd=choice["bwd"])
    ctx.set_option(_lib.OPT_BWD_VARIANT, choice.get("variant", 0))
    ctx.set_option(_lib.OPT_BWD_SEGMENT, choice["segment"])


def tune_options(params0, degree, cams, ctx, views: int = 1, repeats: int = 3, bg=(0.0, 0.0, 0.0),
                 frozen=None) -> dict:
    """gsta_autotune on the first `views` cameras (with the freeze map
    `frozen`, a [n] uint8 device tensor, if given): sets and returns the
    fastest {fwd, bwd, variant, segment} with their times."""
    P = torch.from_numpy(params0).float().cuda()
    H, W = cams[0].height, cams[0].width
    img = torch.empty((views, 3, H, W), device="cuda")
    dL = torch.full_like(img, 1.0 / img.numel())
    grad = torch.empty_like(P)
    t = ctx.autotune(P, degree, camera_array(cams[:views]), bg, img, dL, grad, repeats, frozen=frozen)
    return dict(fwd=t["fwd_waves"], bwd=t["bwd_waves"], variant=t["bwd_variant"], segment=t["bwd_segment"],
                fwd_ms=t["fwd_ms"], step_ms=t["step_ms"], candidates=t["candidates"])


def tune(params0, degree, cams, targets, order, ctx, base_cfg: TrainConfig, iters: int = 30,
         cache_path: str | None = _DEFAULT_CACHE, log=None) -> dict:
    """Fastest launch options (gsta_autotune) and the faster of eager and
    graph-replayed training iterations for this workload: returns {fwd,
    bwd, variant, segment, graph} and leaves the options set on ctx."""
    n = params0.shape[1]
    assert params0.shape[0] == n_rows(degree)
    key = workload_key(n, degree, cams[0].height, cams[0].width, base_cfg.views_per_step)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        apply(ctx, cache[key])
        return cache[key]
    opts = tune_options(params0, degree, cams, ctx, views=max(1, base_cfg.views_per_step))
    if log:
        log(f"autotune launch options: {opts}")
    best, best_t = None, float("inf")
    graph_ok = base_cfg.views_per_step == 1 or base_cfg.batches is not None
    for graph in ([False, True] if graph_ok else [False]):
        cfg = TrainConfig(**{**base_cfg.__dict__, "graph": graph, "device_sched": graph or base_cfg.device_sched})
        tr = Trainer(params0, degree, cams, targets, cfg, order, ctx=ctx)
        tr.run(min(len(cams), 32))            # warm-up (captures the graphs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr.run(iters)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / iters
        if log:
            log(f"autotune graph={graph}: {dt * 1e3:.3f} ms/iter")
        if dt < best_t:
            best, best_t = graph, dt
    choice = dict(fwd=opts["fwd"], bwd=opts["bwd"], variant=opts["variant"], segment=opts["segment"], graph=best)
    apply(ctx, choice)
    if cache_path:
        cache[key] = choice
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            json.dump(cache, open(cache_path, "w"), indent=1)
        except OSError:
            pass
    return choice
