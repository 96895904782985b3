"""Tile-shape autotuning with a persistent cache.

``tune(handle, precision, ...)`` looks up the best smoother tile shapes for
the handle's grid, precision, sweep counts and batch size in a JSON cache
and applies them (lt_set_tiles); on a miss it runs lt_autotune on the GPU
and stores the result.  The cache file is ``$LT_TUNE_CACHE`` if set, else
``~/.cache/paper_1409_2556_amd/tiles.json``; entries are keyed by the
device name as well, so a cache copied between machines is not misapplied.
"""
from __future__ import annotations

import json
import os

from . import binding as lt


def cache_path() -> str:
    p = os.environ.get("LT_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1409_2556_amd", "tiles.json")


def _key(handle, precision, nu1, nu2, nvec):
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    g = handle.grid
    return f"{dev}|{g.ndim}|{g.n[0]}x{g.n[1]}x{g.n[2]}|p{int(precision)}|nu{int(nu1)}{int(nu2)}|r{int(nvec)}"


def _load(path):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def tune(handle, precision, nu1=2, nu2=2, nvec=8, path: str | None = None, force: bool = False):
    """Apply cached (or freshly measured) tile shapes; returns (tiles, us per step or None, from_cache)."""
    path = path or cache_path()
    key = _key(handle, precision, nu1, nu2, nvec)
    cache = _load(path)
    if not force and key in cache:
        tiles = [int(t) for t in cache[key]["tiles"]]
        lt.lt_set_tiles(handle, precision, tiles)
        return tiles, cache[key].get("us"), True
    tiles, us = lt.lt_autotune(handle, precision, nu1, nu2, nvec)
    cache = _load(path)  # re-read: another process may have written meanwhile
    cache[key] = {"tiles": tiles, "us": us, "shapes": [list(lt.lt_tile_shape(t)) for t in tiles]}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return tiles, us, False
