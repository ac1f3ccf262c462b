"""Autotuner for the batched, persistent, graph-captured training step.

Searches tile edge T in {8, 16, 32}, Gaussians-per-LDS-batch S in
{32, 64, 128, 256} and, for T = 16 and 32, pixels per lane P in {1, 2, 4}
(one lane renders P pixels of its tile, so a tile takes T*T/P lanes).  Every candidate runs the same iterations from the same
optimiser state (restored between candidates), each as a captured HIP graph, every
iteration timed with events on the launch stream; the candidate with the
lowest mean step time wins (the standard deviation is reported beside it).  Results are cached in a
JSON file keyed by GPU architecture, the view-set resolutions and the
Gaussian count; an unreadable cache entry is ignored and the search reruns.

The paper chooses S per tile as ceil(sqrt(N P)) rounded to a wave multiple
and capped at 128 from a latency model (Sec. 4.2); here S is one value per
launch, chosen by measurement, and the model only orders the candidates.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import pipeline as P
from .batched import BatchedStep, ViewSet

TILES = (8, 16, 32)
BATCHES = (32, 64, 128, 256)
LANE_PIXELS = (1, 2, 4)


def cache_key(resolutions, n: int) -> str:
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    res = "_".join(f"{w}x{h}" for w, h in resolutions)
    return f"{arch}|{res}|n{int(round(math.log2(max(n, 1))))}"


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path: str, data: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def capacity_for(model: P.Model, n: int, viewset: ViewSet, view_rows, iters, slack=1.15):
    """Intersection and tile-row capacities covering the given iterations
    (largest counts times `slack`; synchronises)."""
    f = P.Frame(n, viewset.widths, viewset.heights, viewset.tile, capacity=1, cull=viewset.cull)
    kmax = rmax = 0
    for i in iters:
        P.project(model.params, f, view_rows(i).reshape(-1))
        kmax = max(kmax, int(f.tiles.to(torch.int64).sum().item()))
        rmax = max(rmax, P.tile_rows(f))
    del f
    return int(kmax * slack) + 4096, int(rmax * slack) + 4096


def time_candidate(model: P.Model, n: int, resolutions, tile: int, lds: int, view_rows, targets,
                   iters, capacity, ppl: int | None = None, cull: int = 0) -> float:
    saved = [t.clone() for t in (model.params, model.m, model.v, model.step)]
    vs = ViewSet(resolutions, tile, ppl, cull)
    step = BatchedStep(model, n, vs, capacity[0], lds_batch=lds, persistent=True,
                       row_capacity=capacity[1])
    step.load(view_rows(iters[0]), targets(iters[0]))
    step.capture()
    for i in iters[:2]:                        # warm replays
        step.load(view_rows(i), targets(i))
        step.run()
    torch.cuda.synchronize()
    for t, s0 in zip((model.params, model.m, model.v, model.step), saved):
        t.copy_(s0)
    # each iteration bracketed by events on the launch stream
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in iters]
    for (e0, e1), i in zip(ev, iters):
        step.load(view_rows(i), targets(i))
        e0.record()
        step.run()
        e1.record()
    torch.cuda.synchronize()
    ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    if step.status():
        ms = [float("inf")] * len(ms)          # capacity exceeded: not a valid candidate
    for t, s0 in zip((model.params, model.m, model.v, model.step), saved):
        t.copy_(s0)
    del step
    torch.cuda.empty_cache()
    return ms


def autotune(model: P.Model, n: int, resolutions, view_rows, targets, iters, cache_path=None,
             tiles=TILES, batches=BATCHES, lane_pixels=LANE_PIXELS, log=print, cull: int = 0) -> dict:
    key = cache_key(resolutions, n) + f"|c{int(cull)}"
    cache = load_cache(cache_path) if cache_path else {}
    hit = cache.get(key)
    if (isinstance(hit, dict) and hit.get("tile") in tiles and hit.get("lds_batch") in batches
            and hit.get("pixels_per_lane") in lane_pixels + (1,)):
        return dict(hit, cached=True)
    table, spread = {}, {}
    for T in tiles:
        cap = capacity_for(model, n, ViewSet(resolutions, T, cull=cull), view_rows, iters)
        for ppl in ((1,) if T == 8 else lane_pixels):
            for S in batches:
                ms = time_candidate(model, n, resolutions, T, S, view_rows, targets, iters, cap, ppl, cull)
                key_c = f"T{T}_S{S}_P{ppl}"
                table[key_c] = float(sum(ms) / len(ms))
                spread[key_c] = float(math.sqrt(sum((x - table[key_c]) ** 2 for x in ms) / len(ms))
                                      if math.isfinite(table[key_c]) else float("inf"))
                log(f"autotune T={T} S={S} P={ppl}: {table[key_c]:.3f} +- {spread[key_c]:.3f} ms/step "
                    f"({len(ms)} iterations)")
    best = min(table, key=table.get)
    T, S, ppl = (int(x[1:]) for x in best.split("_"))
    res = {"tile": T, "lds_batch": S, "pixels_per_lane": ppl, "ms": table[best], "table_ms": table,
           "table_std_ms": spread, "iterations": len(iters), "cached": False}
    if cache_path:
        cache[key] = {k: v for k, v in res.items() if k != "cached"}
        save_cache(cache_path, cache)
    return res
