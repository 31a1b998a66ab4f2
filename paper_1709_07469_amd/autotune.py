"""Launch-setting autotuning with a persistent cache.

``tune(problem, kind)`` runs the library's sweep (``fk_autotune``: block
size, resident blocks per CU, queue-run length) on a reduced walk count of
the problem, installs the fastest setting for the problem's precision and
records it in a JSON cache keyed by device name, precision, kind and the
workload's shape (stations, walks per station, source kind, steps per walk
order of magnitude).  ``apply_cached(problem, kind)`` installs a cached
setting without timing anything.  The cache file is FKGRAV_TUNE_CACHE, or
~/.cache/fkgrav_tune.json.  Settings never change results, only time.
"""
from __future__ import annotations

import json
import math
import os

from . import fkgrav as F

CACHE = os.environ.get("FKGRAV_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "fkgrav_tune.json")


def _key(prob, kind) -> str:
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    src = "grid" if prob.rho is not None else ("bodies" if len(prob.prisms) + len(prob.spheres) else "none")
    extent = float(min(h - l for h, l in zip(prob.box_hi, prob.box_lo)))
    steps_order = int(round(math.log10(max(1.0, (extent / 2.0) ** 2 / prob.dt))))
    return f"{dev}|p{prob.precision}|k{kind}|S{prob.n_stations}|N{int(math.log10(prob.paths_per_station))}|{src}|s{steps_order}"


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict) -> None:
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def tune(prob, kind: int = 0, tuning_walks: int | None = None, force: bool = False) -> dict:
    """Tunes (or reuses the cached setting for) this workload; returns the
    installed setting with its tuning time."""
    cache = _load()
    key = _key(prob, kind)
    if key in cache and not force:
        s = cache[key]
        F.fk_set_launch(prob.precision, s["block"], s["blocks_per_cu"], s["grab"])
        return s
    n = tuning_walks or max(2, min(prob.paths_per_station, 2048))
    small = prob.replace(paths_per_station=n)
    P = F.Prepared(small)
    ws = F.alloc_workspace(F.fk_workspace_bytes(kind, small.n_stations, P.params))
    out = F.alloc_stats(small.n_stations)
    best, ms = F.fk_autotune(kind, P.stations, P.box, P.source, P.bc, P.params, out, ws)
    best["tune_ms"] = ms
    best["tuning_walks"] = n
    cache[key] = best
    _store(cache)
    return best


def apply_cached(prob, kind: int = 0) -> dict | None:
    s = _load().get(_key(prob, kind))
    if s:
        F.fk_set_launch(prob.precision, s["block"], s["blocks_per_cu"], s["grab"])
    return s
