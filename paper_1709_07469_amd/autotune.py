"""Launch-setting autotuning with a persistent cache.

``tune(problem, kind)`` runs the library's sweep (``fk_autotune``: block
size, resident blocks per CU, queue-run length) on a reduced walk count of
the problem, installs the fastest setting for the problem's precision and
records it in a JSON cache keyed by device name, precision, kind and the
workload's shape (stations, walks per station, source kind, steps per walk
order of magnitude).  ``apply_cached(problem, kind)`` installs a cached
setting without timing anything.  ``tune_batch(problems, kinds)`` searches
all launch settings (block size, blocks per CU, queue-run length, queue
stripes, refill cost) one at a time on a scaled-down copy of a whole batch
(every problem with a fraction of its walks), so the choice reflects the
batch's mix of problems.  The cache file is FKGRAV_TUNE_CACHE, or
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
        F.fk_set_launch_dict(prob.precision, s)
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
        F.fk_set_launch_dict(prob.precision, s)
    return s


# Values tried for each launch setting of a batch (fk_launch), one setting at
# a time from the current one (coordinate search): block size, resident blocks
# per CU (0 = the occupancy limit), queue-run length, claim counters the queue
# is split into (0 = the library's default for the batch), and the refill
# rule's start-up cost (128 R; 0 = the default 64).
BATCH_KNOBS = {"block": (64, 128, 256), "blocks_per_cu": (0, 2), "grab": (16, 32, 64),
               "stripes": (0, 1, 4, 16), "refill_cost": (0, 16, 32, 128, 256)}


def tune_batch(probs, kinds, walk_fraction: float = 0.05, min_walks: int = 64, rounds: int = 1,
               repeats: int = 2) -> dict:
    """Tunes the launch settings of a batch by coordinate search: starting
    from the installed setting, each knob of BATCH_KNOBS in turn takes the
    value with the shortest time (the best of `repeats` solves) with the
    others fixed; `rounds` passes over the knobs.  Times are taken on the batch
    with each problem's walks cut to walk_fraction.  Installs the result for
    the batch's precision and returns it with its time and the default's.
    Results never depend on the setting."""
    import torch
    small = [p.replace(paths_per_station=max(min_walks, int(p.paths_per_station * walk_fraction))) for p in probs]
    PB = F.PreparedBatch(small, kinds)
    ws = F.alloc_workspace(F.fk_batch_workspace_bytes(PB.problems))
    out = F.alloc_stats(PB.n_out)
    prec = probs[0].precision

    def timed(setting):
        F.fk_set_launch_dict(prec, setting)
        F.fk_solve_batch(PB.problems, out, ws)
        torch.cuda.synchronize()
        best = None
        for _ in range(repeats):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            F.fk_solve_batch(PB.problems, out, ws)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        return best

    cur = F.fk_get_launch(prec)
    cur_ms = default_ms = timed(cur)
    trials = 1
    for _ in range(rounds):
        for knob, values in BATCH_KNOBS.items():
            for v in values:
                if v == cur[knob]:
                    continue
                cand = dict(cur, **{knob: v})
                ms = timed(cand)
                trials += 1
                if ms < cur_ms:
                    cur, cur_ms = cand, ms
    F.fk_set_launch_dict(prec, cur)
    del ws
    return dict(cur, tune_ms=cur_ms, default_ms=default_ms, walk_fraction=walk_fraction, trials=trials)
