"""Autotuner of the launch parameters that leave results unchanged.

* Grid cell size of the neighbour search (``cell_shift``): the kNN result
  does not depend on it (every candidate is compared by exact integer distance
  and id), only its speed does.  Timed with ``pg_knn`` on the actual scene for
  the default shift and its two neighbours.
* Edge tile of the propagation (``tile``: workgroup size of the aggregation
  and the shift; ``tile_group``: consecutive row tiles each XCD takes in turn
  in the aggregation): the same rows, slots and arithmetic in every launch
  shape, so images are bit-identical.  Timed as the summed ``spmv`` + ``shift``
  phase time of a short render (``probe_D`` iterations) with the library's
  phase profiler.

Results are cached per (vertex-count bucket, k) in memory and, optionally, in
a JSON file (``load`` / ``save``).
"""
from __future__ import annotations

import ctypes
import json
import math
import os

from . import DevicePaths, Renderer, lib, params, pg_default_cell_shift, pg_knn, _check

_cache: dict = {}

TILES = (128, 256, 512)
GROUPS = (1, 4, 16)


def _key(n: int, k: int, what: str = "cell") -> str:
    b = int(round(math.log2(max(n, 1)) * 2))   # half-octave buckets of N
    return f"{what}:{b}:{k}"


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


def _propagation_ms(render, image) -> float:
    """spmv + shift phase time of one render, from the phase profiler."""
    from . import ProfileEntry
    L = lib()
    _check(L.pg_profile_start())
    render(image)
    arr = (ProfileEntry * 64)()
    n = ctypes.c_int32()
    _check(L.pg_profile_stop(64, arr, ctypes.byref(n)))
    return sum(arr[i].total_ms for i in range(min(n.value, 64)) if arr[i].name in (b"spmv", b"shift"))


SCENE_DEFAULT = (512, 1)   # pg_render's launch shape when params.tile = 0
BATCH_DEFAULT = (256, 1)   # a batch's


def tune_tile(paths: DevicePaths, k: int, g: float = 0.5, probe_D: int = 16, cell_shift: int = 0,
              margin: float = 0.03, default: tuple = SCENE_DEFAULT) -> tuple[int, int]:
    """The fastest (tile, tile_group) for this scene's propagation (cached);
    `default` unless a candidate beats it by more than `margin` (the probe's
    noise is one to two percent)."""
    import torch

    n = paths.n_vertices
    default = tuple(default)
    key = _key(n, k, f"tile{default[0]}")
    if key in _cache:
        return tuple(_cache[key])
    if n < 65536:                      # a few waves per XCD: the launch shape hardly matters
        _cache[key] = default
        return default
    image = torch.empty(paths.height, paths.width, 3, device=paths.device)
    times = {}
    for t in TILES:
        for grp in GROUPS:
            r = Renderer(paths, params(k=k, D=probe_D, g=g, cell_shift=cell_shift, tile=t, tile_group=grp))
            r(image)                   # warm-up
            times[(t, grp)] = min(_propagation_ms(r, image) for _ in range(3))
            del r
    torch.cuda.empty_cache()
    best = min(times, key=times.get)
    if times[best] > (1.0 - margin) * times[default]:
        best = default
    _cache[key] = best
    return best


def tune(paths: DevicePaths, k: int, g: float = 0.5, probe_D: int = 16) -> dict:
    """cell_shift, tile and tile_group for this scene (each cached)."""
    s = tune_cell_shift(paths, k)
    t, grp = tune_tile(paths, k, g, probe_D, s)
    return {"cell_shift": s, "tile": t, "tile_group": grp}
