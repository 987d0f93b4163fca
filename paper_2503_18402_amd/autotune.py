"""Autotuner for the blend kernels' tile size and LDS batch.

For a given set of views (a resolution mix) and scene size it times the
forward + backward of the hot path for every (tile, lds_batch) pair and keeps
the fastest.  The image does not depend on the choice (binning is
result-neutral; tile sizes differ only in the last-bit rounding of the mean
moved into each tile's frame), so the pick is purely a speed decision.
Results are cached in memory and, when ``path`` is given, in a JSON file
keyed by device, resolution mix and scene-size bucket.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import gsmi, raster

TILES = (8, 16, 32)
BATCHES = (128, 256, 512)
_cache: dict = {}


def _key(cams, n: int) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    mix = ",".join(f"{int(c.width)}x{int(c.height)}" for c in cams)
    return f"{dev}|{mix}|n2^{int(round(math.log2(max(n, 1))))}"


def _time_fwd_bwd(pipe: raster.Pipeline, reps: int) -> float:
    def once():
        pipe.forward()
        pipe.backward()
    once()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        once()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(params: dict, cams, targets: torch.Tensor, reps: int = 5, path: str | None = None,
         tiles=TILES, batches=BATCHES) -> dict:
    """Best {tile, lds_batch, ms} for these views; the full table under 'table'."""
    key = _key(cams, params["means"].shape[0])
    if key in _cache:
        return _cache[key]
    if path and os.path.exists(path):
        with open(path) as f:
            disk = json.load(f)
        if key in disk:
            _cache[key] = disk[key]
            return disk[key]
    table = []
    capacity = None
    for tile in tiles:
        for batch in batches:
            pipe = raster.Pipeline(params, cams, targets, tile=tile, lds_batch=batch,
                                   capacity=None if tile != 8 else capacity)
            ms = _time_fwd_bwd(pipe, reps)
            if pipe.overflowed():
                raise RuntimeError("autotune: pair capacity overflowed")
            table.append(dict(tile=tile, lds_batch=batch, ms=round(ms, 4)))
            del pipe
    best = min(table, key=lambda r: r["ms"])
    res = dict(tile=best["tile"], lds_batch=best["lds_batch"], ms=best["ms"], table=table)
    _cache[key] = res
    if path:
        disk = {}
        if os.path.exists(path):
            with open(path) as f:
                disk = json.load(f)
        disk[key] = res
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump(disk, f, indent=1)
    return res
