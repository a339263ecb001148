"""Autotuner of the type-1 spreading tile shape.

The spreading kernel sums each source's w x w kernel contributions per tile
of the fine grid in on-chip memory.  Small tiles give more workgroups but list
each source in more tiles (the support overlaps (T + w - 1)^2 / T^2 tiles);
large tiles amortise the list but leave fewer, longer workgroups.  Which wins
depends on the source density per tile and on the band size, so the tuner
times every shape on the plan itself (wfp2d_time_spread) and caches the
winner per size class in a JSON file.

Size class: (precision, kernel width w, padded band rounded up to a multiple
of 256, log2 of the sources per band cell rounded to a half).
"""
from __future__ import annotations

import json
import math
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "wfp2d", "spread_tiles.json")


def cache_path() -> str:
    return os.environ.get("WFP2D_TUNE_CACHE", DEFAULT_CACHE)


def size_class(info: dict) -> str:
    band = int(info["band"])
    density = info["M"] / float(max(band, 1) ** 2)
    d = round(2.0 * math.log2(max(density, 1e-12))) / 2.0
    prec = "mixed" if info["precision"] == 1 else "fp64"
    return f"{prec}_w{info['nufft_w']}_band{(band + 255) // 256 * 256}_dens2^{d:+.1f}"


def _load(path):
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path, data):
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_spread(plan, reps: int = 10, cache: str | None = None, retune: bool = False,
                codes=None) -> dict:
    """Select the fastest spreading tile shape for `plan` (cached per size class).

    Returns {"class", "code", "tile", "ms": {code: ms} or None when cached}.  `codes`
    defaults to every shape the plan offers."""
    codes = tuple(sorted(plan.SPREAD_TILES)) if codes is None else tuple(codes)
    path = cache_path() if cache is None else cache
    info = plan.info()
    key = size_class(info)
    data = _load(path) if path else {}
    hit = data.get(key)
    if hit is not None and not retune and int(hit.get("code", 0)) in codes:
        code = int(hit["code"])
        plan.set_spread_tile(code)
        return {"class": key, "code": code, "tile": plan.SPREAD_TILES[code], "ms": None}
    ms = {c: plan.time_spread(c, reps) for c in codes}
    code = min(ms, key=ms.get)
    plan.set_spread_tile(code)
    if path:
        data = _load(path)
        data[key] = {"code": code, "tile": list(plan.SPREAD_TILES[code]), "ms": {str(c): v for c, v in ms.items()}}
        _store(path, data)
    return {"class": key, "code": code, "tile": plan.SPREAD_TILES[code], "ms": ms}
