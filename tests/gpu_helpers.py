"""Shared helpers of the GPU parity tests: run the HIP path through the C
interface and compare its per-walk samples with the CPU oracle's."""
import sys

import numpy as np

CAP = np.uint32(0x80000000)
MASK = np.uint32(0x7FFFFFFF)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_solve(prob, kind):
    from paper_1709_07469_amd import fkgrav as F
    stats, ws, P = F.solve(prob, kind)
    vals, steps = F.path_samples(ws, kind, len(P.stations_host), P.params)
    return stats, vals, steps


def compare_walks(g_vals, g_steps, o_vals, o_steps, scale, rel=1e-12):
    """Per-walk comparison.  Returns a dict with the number of walks, the
    step-count mismatches (a walk that left the box one step earlier or later
    on one side: a last-bit difference in a transcendental put a point on the
    other side of a face), the value mismatches among walks with equal step
    counts (a voxel or prism membership decided differently), and the largest
    relative difference of the matching walks."""
    shape = np.shape(g_vals)
    scale = np.broadcast_to(np.asarray(scale, dtype=np.float64), shape).ravel()
    g_vals = np.asarray(g_vals).ravel()
    o_vals = np.asarray(o_vals).ravel()
    g_steps = np.asarray(g_steps).ravel()
    o_steps = np.asarray(o_steps).ravel()
    same_steps = g_steps == o_steps
    capped = (o_steps & CAP) != 0
    ok = same_steps & ~capped
    diff = np.abs(g_vals[ok] - o_vals[ok])
    tol = rel * scale[ok]
    bad = diff > tol
    worst = float(np.max(diff / scale[ok])) if ok.any() else 0.0
    cap_ok = bool(np.all(np.isnan(g_vals[capped & same_steps])))
    return {"n": int(g_vals.size), "step_mismatch": int((~same_steps).sum()), "value_mismatch": int(bad.sum()),
            "worst_rel": worst, "capped_nan": cap_ok}
