"""Launch-setting autotuning with a persistent cache.

``tune(problem, kind)`` runs the library's sweep (``fk_autotune``: block
size, resident blocks per CU, queue-run length) on a reduced walk count of
the problem, installs the fastest setting for the problem's precision and
records it in a JSON cache keyed by device name, precision, kind and the
workload's shape (stations, walks per station, source kind, steps per walk
order of magnitude).  ``apply_cached(problem, kind)`` installs a cached
setting without timing anything.  ``tune_batch(problems, kinds)`` times the
same candidates on a scaled-down copy of a whole batch (every problem with a
fraction of its walks), so the choice reflects the batch's mix of problems.  The cache file is FKGRAV_TUNE_CACHE, or
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


BATCH_CANDIDATES = [(b, r, g) for b in (64, 128, 256) for r in (0, 2) for g in (16, 32, 64)]


def tune_batch(probs, kinds, walk_fraction: float = 0.05, min_walks: int = 64) -> dict:
    """Times every candidate launch setting (block size, resident blocks per
    CU -- 0 for the occupancy limit --, queue-run length) on the batch with
    each problem's walks cut to walk_fraction, installs the fastest for the
    batch's precision and returns it with its time.  Results never depend on
    the setting."""
    import torch
    small = [p.replace(paths_per_station=max(min_walks, int(p.paths_per_station * walk_fraction))) for p in probs]
    PB = F.PreparedBatch(small, kinds)
    ws = F.alloc_workspace(F.fk_batch_workspace_bytes(PB.problems))
    out = F.alloc_stats(PB.n_out)
    prec = probs[0].precision
    best = None
    for block, bpc, grab in BATCH_CANDIDATES:
        F.fk_set_launch(prec, block, bpc, grab)
        F.fk_solve_batch(PB.problems, out, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        F.fk_solve_batch(PB.problems, out, ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        if best is None or ms < best["tune_ms"]:
            best = {"block": block, "blocks_per_cu": bpc, "grab": grab, "tune_ms": ms}
    F.fk_set_launch(prec, best["block"], best["blocks_per_cu"], best["grab"])
    best["walk_fraction"] = walk_fraction
    del ws
    return best
