"""Autotuner for the uniform-grid cell size of the neighbour search.

The kNN result does not depend on the cell size (every candidate is compared
by exact integer distance and id), only its speed does.  The tuner times the
neighbour search for the default cell shift and its two neighbours on the
actual scene and keeps the fastest; results are cached per (vertex-count
bucket, k) in memory and, optionally, in a JSON file.
"""
from __future__ import annotations

import json
import math
import os

from . import DevicePaths, pg_default_cell_shift, pg_knn

_cache: dict = {}


def _key(n: int, k: int) -> str:
    b = int(round(math.log2(max(n, 1)) * 2))   # half-octave buckets of N
    return f"{b}:{k}"


def load(path: str) -> None:
    if path and os.path.exists(path):
        with open(path) as f:
            _cache.update(json.load(f))


def save(path: str) -> None:
    if path:
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump(_cache, f, indent=1, sort_keys=True)


def tune_cell_shift(paths: DevicePaths, k: int, reps: int = 2) -> int:
    """The fastest cell shift for this scene's neighbour search (cached)."""
    import torch

    n = paths.n_vertices
    key = _key(n, k)
    if key in _cache:
        return int(_cache[key])
    d = pg_default_cell_shift(n)
    cands = [s for s in (d - 1, d, d + 1) if 11 <= s <= 20]
    if n < 4096:
        _cache[key] = d
        return d
    best, best_t = d, float("inf")
    for s in cands:
        pg_knn(paths, k, s)            # warm-up (allocations, code load)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            pg_knn(paths, k, s)
        t1.record()
        t1.synchronize()
        t = t0.elapsed_time(t1) / reps
        if t < best_t:
            best, best_t = s, t
    _cache[key] = best
    return best
