"""Launch-shape autotuner for the batched step.

Results do not depend on the launch shape (images, transmittances and last
contributors are bitwise identical across tile shapes and dispatch modes, and the
forward that joins separately composited chunks of long tile lists differs from
the walk in order by rounding only; the number of Gaussians staged per LDS batch
changes nothing but the staging), so the tuner only measures: for every
candidate (tile shape, persistent or grid dispatch, joined forward or not) at
64 Gaussians per batch it builds a workspace sized for the scene, replays a few
steps and keeps the fastest; then it times the winner with 32, 128 and 256
Gaussians per batch.  Results are cached in a JSON file keyed by GPU
architecture, image size, view count and a Gaussian-count bucket.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import pipeline as pl

TILES = ((16, 16), (8, 8), (16, 32), (32, 16))
BATCHES = (32, 64, 128, 256)
CACHE = os.path.join(os.path.expanduser("~"), ".cache", "splat_gfx950_autotune.json")


def _key(ds) -> str:
    arch = torch.cuda.get_device_properties(ds.opacity.device).gcnArchName.split(":")[0]
    gb = 2 ** int(round(math.log2(max(1, ds.n_gauss))))
    return f"{arch}|{ds.W}x{ds.H}|V{ds.n_views}|G~{gb}"


def _load_cache():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time(ds, xi, delta, targets, st, steps):
    step = pl.BatchedStep(ds, xi, delta, targets, st)
    step.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del step
    torch.cuda.empty_cache()
    return ms


def _settings(c):
    return pl.make_settings(tile=tuple(c["tile"]), persistent=c["persistent"], split_fwd=c.get("split_fwd", 0),
                            batch=c.get("batch", 64))


def autotune(ds, xi, delta, targets, steps=3, tiles=TILES, modes=(False, True), joined=(0, 1),
             batches=BATCHES, use_cache=True):
    """Return (settings, report) of the fastest launch shape for this scene's batched step."""
    key = _key(ds)
    cache = _load_cache() if use_cache else {}
    if use_cache and key in cache:
        c = cache[key]
        return _settings(c), dict(cached=True, **c)
    results = []
    for tile in tiles:
        for pers, sf in ((p, j) for p in modes for j in joined):
            c = dict(tile=list(tile), persistent=bool(pers), split_fwd=int(sf), batch=64)
            c["ms"] = round(_time(ds, xi, delta, targets, _settings(c), steps), 3)
            results.append(c)
    best = min(results, key=lambda r: r["ms"])
    for nb in batches:
        if nb == 64:
            continue
        c = dict(best, batch=int(nb))
        c["ms"] = round(_time(ds, xi, delta, targets, _settings(c), steps), 3)
        results.append(c)
    best = min(results, key=lambda r: r["ms"])
    report = dict(cached=False, key=key, best=best, candidates=results)
    if use_cache:
        cache[key] = best
        try:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            with open(CACHE, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return _settings(best), report
