#!/usr/bin/env python3
"""Benchmark of the Monte Carlo Feynman-Kac gravity solver on one MI355X.

One step is one pass of the hot path over the 32-model voxel batch: 32
independent density models (64^3 FP32 voxel grids of 1-8 voxel-aligned
prisms with contrasts in [50, 500], boxes of random aspect ratio 1-4), 8-256
stations each (3936 in all), 1e4-1e6 walks per station (1.2e9 walks,
6.3e11 Brownian steps of dt = 1e-3), exact prism data on the faces, the
potential at every station, in mixed precision (FP32 random stream and
stepping; FP64 path integrals, exit data and statistics): one persistent
batched walk launch with a work-stealing queue and the batched reduction,
captured once in a HIP graph and replayed.  Inputs are resident in device
memory before timing starts.

The JSON line reports Brownian steps per second of the whole pass (exact
in-kernel step counts over the event-timed replays), the walk kernel's
roofline (algorithmic FLOP per step over the kernel's own event-timed
duration against the vector peak of its precision, with the recorded VALU
counters and HBM bytes beside it), station estimates per second at a fixed
relative standard error, each result's error against the closed-form
solution, and further legs: the same batch in FP64 (the plain path at equal
walks, hence equal accuracy), the same batch in a bounded workspace, the
launch autotuner, the SI-prism workload (u and g_z) and the 128^3-grid
workload in both precisions, the paper's Table 1 workload, the adjoint, and
the CPU oracle timed on a prefix of the batch's walks (with a paired check of
the mixed kernel's walks against the oracle's FP32-stream mode).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs all|name,...]
                  [--cpu-seconds S] [--copy-bytes B]

Legs: headline f64 bounded tune cfg2 cfg3 table1 adjoint cpu.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Brownian steps/s and station estimates/s at fixed std error; % FP32/FP64 VALU peak"
LEGS = ("headline", "f64", "bounded", "tune", "cfg2", "cfg3", "table1", "adjoint", "cpu")

# MI355X vector peaks: FP64 78.6 TFLOP/s; FP32 157.3 TFLOP/s (the published
# figure, which counts packed FP32; the kernels are built without packed FP32,
# so 78.6 is their practical ceiling).  Full-rate VALU issue: 256 CUs x 4
# SIMDs x 16 lanes x 2.4 GHz lane-operations per second.
PEAK_F64_FLOPS = 78.6e12
PEAK_F32_FLOPS = 157.3e12
PEAK_LANE_OPS = 256 * 64 * 2.4e9

# Algorithmic floating-point work of one Euler-Maruyama step, independent of
# how a kernel does it (FMA = 2, a transcendental = 1):
#   3 normals = 1.5 Box-Muller pairs, each ln, sqrt, sin, cos (4) and the
#     products -2 ln u, 2 pi u, R cos, R sin (4): 12
#   position x + sqrt(dt) z, 3 FMA: 6
#   voxel index (x - o) / spacing per axis, 3 FMA: 6
#   trapezoid term rho_n + rho_{n+1} added to the sum: 2
ALGO_FLOP_PER_STEP = 26.0
# Algorithmic HBM bytes of a walk: its exit record (x, y, z, S: 32 B) and
# step count (4 B), written once; the density grids are read once per launch.
ALGO_BYTES_PER_WALK = 36

# Counter data of the kernels, recorded with rocprofv3 on the kernel sources
# hashed in "sources_sha256" (profiles/ hold the commands and summaries).
# VALU: SQ_INSTS_VALU per Brownian step in lane-instructions (x 64),
# SQ_ACTIVE_INST_VALU x 4 cycles over the SIMD-cycles the kernel ran
# (GRBM_GUI_ACTIVE x 4 SIMDs x 256 CUs / 8 XCDs summed; clamped at 1), and
# the FLOP counts (ADD + MUL + 2 FMA + TRANS, F64 and F32) per step, the L2
# hit rate (TCC_HIT / (TCC_HIT + TCC_MISS)).  Bytes:
# FETCH_SIZE and WRITE_SIZE per launch, each scaled by what the counter reads
# for a device copy of known size.  Figures are reported only while the
# sources still hash to the recorded value.
COUNTERS = {
    "sources_sha256": "c32df42d9cb8d2a74286ff80e714ef25820a8e3b38ced9b5f946827f59d3a723",
    "cfg4_mixed": {"valu_lane_instr_per_step": 103.1444, "valu_busy": 1.0913, "fp64_flop_per_step": 2.1044, "fp32_flop_per_step": 29.8313, "fetch_kib": 989051.3594, "write_kib": 80812283.2188, "fetch_scale": 1.999921, "write_scale": 1.0, "l2_hit": 0.9982},
    "cfg4_f64": {"valu_lane_instr_per_step": 257.1337, "valu_busy": 0.9469, "fp64_flop_per_step": 120.411, "fp32_flop_per_step": 0.0613, "fetch_kib": 799770.3594, "write_kib": 74725090.4297, "fetch_scale": 1.999921, "write_scale": 1.0, "l2_hit": 0.9987},
    "cfg2_f64": {"valu_lane_instr_per_step": 214.8479, "valu_busy": 0.967, "fp64_flop_per_step": 108.1473, "fp32_flop_per_step": 0.073, "fetch_kib": 168.7188, "write_kib": 879037.625, "fetch_scale": 1.999921, "write_scale": 1.0, "l2_hit": 0.8743},
    "cfg2_mixed": {"valu_lane_instr_per_step": 84.5602, "valu_busy": 1.0337, "fp64_flop_per_step": 2.1943, "fp32_flop_per_step": 23.5735, "fetch_kib": 7842.6875, "write_kib": 1169483.7031, "fetch_scale": 1.999921, "write_scale": 1.0, "l2_hit": 0.974},
    "cfg3_f64": {"valu_lane_instr_per_step": 263.2239, "valu_busy": 0.9743, "fp64_flop_per_step": 117.7145, "fp32_flop_per_step": 0.0941, "fetch_kib": 470147505.9792, "write_kib": 17541360.9792, "fetch_scale": 1.999921, "write_scale": 1.0, "l2_hit": 0.8799},
    "cfg3_mixed": {"valu_lane_instr_per_step": 106.8119, "valu_busy": 0.6596, "fp64_flop_per_step": 2.1656, "fp32_flop_per_step": 30.5892, "fetch_kib": 480741901.4792, "write_kib": 16468283.5312, "fetch_scale": 1.999921, "write_scale": 1.0, "l2_hit": 0.8767},
    "cfg3_f64_levels": {"valu_lane_instr_per_step": 266.0865, "valu_busy": 0.9891, "fp64_flop_per_step": 117.7144, "fp32_flop_per_step": 0.0941, "fetch_kib": 135953.8958, "write_kib": 31307932.0104, "fetch_scale": 1.999921, "write_scale": 1.0, "l2_hit": 0.9977},
    "cfg3_mixed_levels": {"valu_lane_instr_per_step": 111.1091, "valu_busy": 0.8127, "fp64_flop_per_step": 2.1655, "fp32_flop_per_step": 30.5884, "fetch_kib": 174965.0833, "write_kib": 31272405.9792, "fetch_scale": 1.999921, "write_scale": 1.0, "l2_hit": 0.9972},
}
TRAFFIC_SOURCES = ("paper_1709_07469_amd/csrc/fk_walk.hip", "paper_1709_07469_amd/csrc/fk_device.hpp",
                   "paper_1709_07469_amd/csrc/fk_internal.hpp", "paper_1709_07469_amd/csrc/fk_stats.hpp",
                   "paper_1709_07469_amd/csrc/fk_batch.hip", "paper_1709_07469_amd/csrc/fk_reduce.hip")
TARGETS = os.path.join(ROOT, "tests", "golden", "closed_form_targets.json")


def sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded(key: str):
    """The recorded counter data of one kernel, or None when it was taken on
    other kernel sources (or never)."""
    if not COUNTERS.get("sources_sha256") or COUNTERS["sources_sha256"] != sources_sha256():
        return None
    return COUNTERS.get(key)


def roofline(key, precision, steps_per_launch, kernel_ms, walks_per_launch, grid_bytes=0):
    """The walk kernel's roofline entry: ALGO_FLOP_PER_STEP x steps over the
    kernel's mean launch duration against the vector peak of its precision,
    and the recorded counters at the measured rate."""
    f64 = precision == "f64"
    peak = PEAK_F64_FLOPS if f64 else PEAK_F32_FLOPS
    rate = steps_per_launch / (kernel_ms * 1e-3)
    achieved = ALGO_FLOP_PER_STEP * rate
    algo_bytes = walks_per_launch * ALGO_BYTES_PER_WALK + grid_bytes
    rec = recorded(key)
    traffic = None
    counters = None
    if rec:
        if "fetch_kib" in rec:
            traffic = (rec["fetch_kib"] * rec.get("fetch_scale", 1.0) + rec["write_kib"] * rec.get("write_scale", 1.0)) * 1024
        if "valu_lane_instr_per_step" in rec:
            counters = {
                "valu_busy": min(1.0, rec["valu_busy"]),
                "valu_lane_instr_per_step": rec["valu_lane_instr_per_step"],
                "valu_issue_frac": rec["valu_lane_instr_per_step"] * rate / PEAK_LANE_OPS,
                "fp64_flop_per_step": rec["fp64_flop_per_step"], "fp32_flop_per_step": rec["fp32_flop_per_step"],
                "fp64_frac_of_peak": rec["fp64_flop_per_step"] * rate / PEAK_F64_FLOPS,
                "fp32_frac_of_peak": rec["fp32_flop_per_step"] * rate / PEAK_F32_FLOPS,
                "l2_hit": rec.get("l2_hit")}
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic,
            "kernel_avg_ms": kernel_ms, "steps_per_launch": steps_per_launch,
            "algo_flop_per_step": ALGO_FLOP_PER_STEP,
            "algorithmic_bytes_per_launch": algo_bytes,
            "traffic_over_algorithmic": None if traffic is None else traffic / algo_bytes,
            "frac_of_nonpacked_fp32_peak": None if f64 else achieved / PEAK_F64_FLOPS,
            "counters": counters}


def station_estimates_per_s(stats, steps_per_s, rel_se):
    """Stations per second at a target relative standard error: station s
    needs N_s = var_s / (rel_se |mean_s|)^2 samples of mean_steps_s steps."""
    work = 0.0
    for s in stats:
        if not (s["n"] > 1 and s["mean"] != 0):
            continue
        n_req = s["var"] / (rel_se * abs(s["mean"])) ** 2
        work += n_req * s["mean_steps"]
    return len(stats) / (work / steps_per_s) if work > 0 else None


def closed_form_error(mean, se, exact):
    """Station errors against the exact solution, in standard errors and
    relative to |exact|."""
    import numpy as np
    mean, se, exact = (np.asarray(a, dtype=np.float64) for a in (mean, se, exact))
    z = (mean - exact) / se
    rel = np.abs(mean - exact) / np.abs(exact)
    return {"stations": int(z.size), "max_abs_z": float(np.max(np.abs(z))), "rms_z": float(np.sqrt(np.mean(z * z))),
            "frac_within_4se": float(np.mean(np.abs(z) <= 4.0)), "max_rel_err": float(np.max(rel)),
            "median_rel_se": float(np.median(se / np.abs(exact)))}


_T0 = time.time()


def log(*a):
    """A progress line on stderr (the JSON line alone goes to stdout), with
    the seconds since the start."""
    print(f"bench: [{time.time() - _T0:.0f} s]", *a, file=sys.stderr, flush=True)


def load_targets():
    with open(TARGETS) as f:
        return json.load(f)


def rows(st):
    return [dict(zip(st.dtype.names, r)) for r in st.tolist()]


# ---------------------------------------------------------------------------
# GPU timing helpers.
# ---------------------------------------------------------------------------

def events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def capture(fn):
    """fn captured in a HIP graph (after one eager run on a side stream)."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def time_replays(g, K, Wm):
    """Wm untimed replays, then K replays between two events: seconds."""
    import torch
    for _ in range(Wm):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = events()
    e0.record()
    for _ in range(K):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def walk_kernel_ms(fn, reps):
    """Mean duration of the walk-kernel launches of `reps` eager calls of fn,
    from the library's event pairs recorded on the launch stream around each
    walk launch; also the calls' mean wall time on the stream."""
    import numpy as np
    import torch

    from paper_1709_07469_amd import fkgrav as F
    torch.cuda.synchronize()
    F.fk_timing_read()
    F.fk_timing_enable(True)
    e0, e1 = events()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    F.fk_timing_enable(False)
    ms = F.fk_timing_read()
    return float(np.sum(ms)) / reps, len(ms) // reps, e0.elapsed_time(e1) / reps


# ---------------------------------------------------------------------------
# Legs.
# ---------------------------------------------------------------------------

def batch_leg(precision, K, Wm, slice_walks=0, keep_walks=None, eager_reps=2):
    """The 32-model batch in one precision: graph-replay time of the whole
    pass, the walk kernel's time from eager passes, station statistics and
    their error against the closed forms.  keep_walks = (n_models, n_walks):
    per-walk samples of station 0 of the first models returned for the
    paired oracle check."""
    import numpy as np
    import torch

    from paper_1709_07469_amd import fkgrav as F
    from paper_1709_07469_amd import workloads as W

    probs = [p.replace(slice_walks=slice_walks) for p in W.cfg4(precision=precision)]
    kinds = [0] * len(probs)
    PB = F.PreparedBatch(probs, kinds)
    nbytes = F.fk_batch_workspace_bytes(PB.problems)
    ws = F.alloc_workspace(nbytes)
    out = F.alloc_stats(PB.n_out)

    def solve():
        F.fk_solve_batch(PB.problems, out, ws)

    g = capture(solve)
    seconds = time_replays(g, K, Wm)
    st = F.stats_to_numpy(out)[:PB.n_out]
    steps = int(st["sum_steps"].sum())
    kms, launches, eager_ms = walk_kernel_ms(solve, eager_reps)
    status, flags = F.fk_workspace_status(ws)
    walks = int(sum(p.n_stations * p.paths_per_station for p in probs))
    grid_bytes = int(sum(np.asarray(p.rho).nbytes for p in probs))
    t = load_targets()["cfg4"]["u"]
    exact = np.concatenate([np.asarray(u) for u in t])
    kept = None
    if keep_walks:
        # the first walks of station 0 of the first models: the leading
        # entries of each model's per-walk arrays
        nm, nw = keep_walks
        kept = []
        for m in range(nm):
            v_off, s_off = F.fk_batch_layout(PB.problems, m)
            v = ws[v_off:v_off + 8 * nw].view(torch.float64).cpu().numpy()
            s = ws[s_off:s_off + 4 * nw].view(torch.int32).cpu().numpy().view(np.uint32)
            kept.append((v.copy(), s.copy()))
    del g, ws
    torch.cuda.empty_cache()
    prec = "f64" if precision == W.PREC_F64 else "mixed"
    res = {"value": steps * K / seconds, "unit": "Brownian steps/s", "seconds_per_pass": seconds / K,
           "eager_seconds_per_pass": eager_ms / 1e3, "steps_per_pass": steps, "walks": walks,
           "workspace_bytes": nbytes, "status": status, "status_flags": flags,
           "roofline": roofline("cfg4_" + prec + ("_bounded" if slice_walks else ""), prec, steps / launches,
                                kms, walks / launches, grid_bytes),
           "walk_launches_per_pass": launches,
           "walk_kernel_share_of_pass": kms * launches / eager_ms,
           "station_estimates_per_s": {"u_rel_se_1e-3": station_estimates_per_s(rows(st), steps * K / seconds, 1e-3)},
           "vs_closed_form": closed_form_error(st["mean"], st["se"], exact)}
    return res, st, kept


def cfg2_leg(reps=3):
    """The SI-prism workload (64 stations x 1e5 walks, u and g_z in one
    batched launch) in FP64 and in mixed precision."""
    import numpy as np
    import torch

    from paper_1709_07469_amd import fkgrav as F
    from paper_1709_07469_amd import workloads as W
    tg = load_targets()["cfg2"]
    out = {"workload": "SI prism 300 kg/m^3 in box [0,1000]^2x[-500,100] m, 8x8 stations at z=0, 1e5 walks/station, "
                       "sqrt(dt)=2 m, exact prism data, u + g_z (CRN, h=2 m), one batched launch"}
    for name, prec in (("f64", W.PREC_F64), ("mixed", W.PREC_MIXED_F64ACC)):
        prob = W.cfg2(precision=prec)
        S = prob.n_stations
        PB = F.PreparedBatch([prob, prob], [0, 1])
        ws = F.alloc_workspace(F.fk_batch_workspace_bytes(PB.problems))
        o = F.alloc_stats(PB.n_out)

        def solve():
            F.fk_solve_batch(PB.problems, o, ws)
        solve()
        kms, launches, ems = walk_kernel_ms(solve, reps)
        st = F.stats_to_numpy(o)
        su, sg = st[:S], st[S:2 * S]
        steps = int(su["sum_steps"].sum() + sg["sum_steps"].sum())
        rate = steps / (ems * 1e-3)
        out[name] = {"value": rate, "unit": "Brownian steps/s", "seconds_per_pass": ems / 1e3,
                     "roofline": roofline("cfg2_" + name, name, steps / launches, kms, 3 * S * prob.paths_per_station),
                     "station_estimates_per_s": {"u_rel_se_1e-3": station_estimates_per_s(rows(su), rate, 1e-3),
                                                 "gz_rel_se_1e-2": station_estimates_per_s(rows(sg), rate, 1e-2)},
                     "u_vs_closed_form": closed_form_error(su["mean"], su["se"], tg["u"]),
                     "gz_vs_closed_form_difference_at_h": closed_form_error(sg["mean"], sg["se"], tg["gz_fd_h"])}
        del ws
        torch.cuda.empty_cache()
    out["mixed_speedup"] = out["mixed"]["value"] / out["f64"]["value"]
    return out


def cfg3_leg(reps=2):
    """The 128^3-grid workload (5 random prisms, 256 stations x 1e6 walks,
    potential) in FP64 and in mixed precision, one solve each."""
    import torch

    from paper_1709_07469_amd import fkgrav as F
    from paper_1709_07469_amd import workloads as W
    tg = load_targets()["cfg3"]
    out = {"workload": "[-1,1]^3, 128^3 FP32 grid of 5 prisms (log-normal contrasts), exact prism data, "
                       "16x16 stations at z = 0.5, 1e6 walks/station, dt = 1e-3, potential; *_levels: the same "
                       "grid given by levels (a byte per voxel and its 6 densities)"}
    stats = {}
    for name, prec, levels in (("f64", W.PREC_F64, False), ("mixed", W.PREC_MIXED_F64ACC, False),
                               ("f64_levels", W.PREC_F64, True), ("mixed_levels", W.PREC_MIXED_F64ACC, True)):
        prob = W.cfg3(precision=prec).replace(grid_levels=levels)
        P = F.Prepared(prob)
        ws = F.alloc_workspace(F.fk_workspace_bytes(0, prob.n_stations, P.params))
        o = F.alloc_stats(prob.n_stations)

        def solve():
            F.fk_solve_potential(P.stations, P.box, P.source, P.bc, P.params, o, ws)
        solve()
        kms, launches, ems = walk_kernel_ms(solve, reps)
        st = F.stats_to_numpy(o)[:prob.n_stations]
        stats[name] = st
        steps = int(st["sum_steps"].sum())
        prec_name = name.split("_")[0]
        grid_bytes = prob.rho.size * (1 if levels else 4)
        out[name] = {"value": steps / (ems * 1e-3), "unit": "Brownian steps/s", "seconds_per_solve": ems / 1e3,
                     "walk_kernel_share": kms * launches / ems,
                     "roofline": roofline("cfg3_" + name, prec_name, steps / launches, kms,
                                          prob.n_stations * prob.paths_per_station, grid_bytes),
                     "vs_closed_form": closed_form_error(st["mean"], st["se"], tg["u"])}
        if levels:
            out[name]["bitwise_equal_to_fp32_grid"] = stats[prec_name].tobytes() == st.tobytes()
        del ws
        torch.cuda.empty_cache()
    out["mixed_speedup"] = out["mixed"]["value"] / out["f64"]["value"]
    out["levels_speedup"] = {p: out[p + "_levels"]["value"] / out[p]["value"] for p in ("f64", "mixed")}
    return out


def tune_leg(reps=3):
    """Default launch setting against the autotuner's pick (timed on the
    batch at 5 % of its walks) on the mixed 32-model batch: the best of
    `reps` graph replays each."""
    import torch

    from paper_1709_07469_amd import autotune
    from paper_1709_07469_amd import fkgrav as F
    from paper_1709_07469_amd import workloads as W

    probs = W.cfg4()
    kinds = [0] * len(probs)
    PB = F.PreparedBatch(probs, kinds)
    ws = F.alloc_workspace(F.fk_batch_workspace_bytes(PB.problems))
    out = F.alloc_stats(PB.n_out)

    def best():
        g = capture(lambda: F.fk_solve_batch(PB.problems, out, ws))
        g.replay()
        t = min(time_replays(g, 1, 0) for _ in range(reps))
        del g
        return t

    keep = F.fk_get_launch(W.PREC_MIXED_F64ACC)
    t_default = best()
    tuned = autotune.tune_batch(probs, kinds, walk_fraction=0.05)
    t_tuned = best()
    F.fk_set_launch_dict(W.PREC_MIXED_F64ACC, keep)
    del ws
    torch.cuda.empty_cache()
    return {"default": {"seconds": t_default, "launch": keep},
            "tuned": {"seconds": t_tuned, "launch": {k: tuned[k] for k in F.LAUNCH_KEYS},
                      "search": {k: tuned[k] for k in ("tune_ms", "default_ms", "walk_fraction", "trials")}},
            "tuned_over_default_time": t_tuned / t_default, "replays_each": reps}


def paper_table1_reference():
    n, rows_ = None, {}
    with open(os.path.join(ROOT, "tests", "golden", "paper_experiments.txt")) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "table1_N":
                n = tuple(int(v) for v in w[1:])
            elif w[0] == "table1":
                rows_[float(w[1])] = tuple(float(v) for v in w[2:])
    return n, rows_


def paper_table1():
    """Experiment 1 of the paper (ball of radius 10 km, zero data, 100 m cube,
    31 stations) at every cell of Table 1, FP64: seconds per solve on this
    GPU (event-timed, median of 3, inputs resident) next to the K20Xm's
    (the paper's Table 1).  Lengths are read as km."""
    import numpy as np
    import torch

    from paper_1709_07469_amd import fkgrav as F
    from paper_1709_07469_amd import workloads as W

    table_n, table_s = paper_table1_reference()
    rows_, ours_total, paper_total, steps_total = [], 0.0, 0.0, 0
    for dtp, paper_s in table_s.items():
        row = []
        for N, ps in zip(table_n, paper_s):
            prob = W.paper_ball(dt_paper=dtp, paths_per_station=N)
            P = F.Prepared(prob)
            ws = F.alloc_workspace(F.fk_workspace_bytes(0, prob.n_stations, P.params))
            o = F.alloc_stats(prob.n_stations)
            F.fk_solve_potential(P.stations, P.box, P.source, P.bc, P.params, o, ws)
            times = []
            for _ in range(3):
                e0, e1 = events()
                e0.record()
                F.fk_solve_potential(P.stations, P.box, P.source, P.bc, P.params, o, ws)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1) / 1e3)
            t = float(np.median(times))
            st = F.stats_to_numpy(o)[: prob.n_stations]
            steps_total += int(st["sum_steps"].sum())
            ours_total += t
            paper_total += ps
            row.append(round(t, 5))
        rows_.append({"dt_paper": dtp, "seconds": row, "paper_k20xm_seconds": list(paper_s)})
    return {"workload": "paper experiment 1: ball R = 10 km (lengths in km), zero data, cube [0,100 m]^3 of "
                        "2000 kg/m^3, 31 stations y = 50 m, z = 200 m, x = -100..200 m; potential, FP64",
            "N": list(table_n), "rows": rows_, "total_seconds": ours_total, "paper_total_seconds": paper_total,
            "speedup_vs_paper_total": paper_total / ours_total, "steps": steps_total,
            "steps_per_s": steps_total / ours_total}


def adjoint_leg(reps=2):
    """d g_z / d rho on the voxel workload (32^3 FP32 grid of 5 prisms, 32
    stations, 1e6 common-random-number walk pairs, zero data, FP64): the
    forward g_z solve and the adjoint replay of the same walks, each timed
    with events over `reps` runs after one warm-up."""
    import numpy as np
    import torch

    from paper_1709_07469_amd import fkgrav as F
    from paper_1709_07469_amd import workloads as W

    pr = W.cfg5()
    P = F.Prepared(pr)
    S = pr.n_stations
    ws = F.alloc_workspace(F.fk_workspace_bytes(1, S, P.params))
    out = F.alloc_stats(S)
    g = torch.full((S,), 1.0 / S, dtype=torch.float64, device=P.stations.device)
    grad = torch.empty(int(np.asarray(pr.rho).size), dtype=torch.float64, device=P.stations.device)
    aws = F.alloc_workspace(F.fk_adjoint_workspace_bytes(S, P.source))

    def forward():
        F.fk_solve_gz(P.stations, P.box, P.source, P.bc, P.params, out, ws)

    def backward():
        F.fk_gz_adjoint(P.stations, P.box, P.source, P.bc, P.params, out, ws, g, grad, aws)

    def seconds(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = events()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    t_fwd = seconds(forward)
    steps = int(F.stats_to_numpy(out)[:S]["sum_steps"].sum())
    t_adj = seconds(backward)
    del ws, aws
    torch.cuda.empty_cache()
    return {"workload": "d(mean g_z)/d rho: 32^3 FP32 grid of 5 prisms, 32 stations, 1e6 CRN walk pairs, zero data, "
                        "FP64; the adjoint replays the forward walks and scatters their trapezoid weights per voxel",
            "voxels": int(np.asarray(pr.rho).size), "steps": steps,
            "forward_seconds": t_fwd, "forward_steps_per_s": steps / t_fwd,
            "adjoint_seconds": t_adj, "adjoint_steps_per_s": steps / t_adj, "adjoint_over_forward": t_adj / t_fwd}


def host_cpu():
    """The host CPU's model, physical cores and hardware threads."""
    model, cores, threads = "unknown", set(), 0
    try:
        phys = None
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model == "unknown":
                    model = v
                elif k == "processor":
                    threads += 1
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    cores.add((phys, v))
    except OSError:
        pass
    return {"model": model, "physical_cores": len(cores) or None, "hardware_threads": threads or None,
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def cpu_baseline(seconds, kept=None):
    """The oracle (plain FP64 C, OpenMP over walks) on the host: every
    station of every model of the 32-model batch, its first n walks, n grown
    until about `seconds` of work; and, with the mixed kernel's per-walk
    samples of station 0 of the first models (kept), the same walks by the
    oracle's FP32-stream mode (the mixed kernel's uniforms, FP64 arithmetic)
    for a paired comparison."""
    import numpy as np

    import oracle
    from paper_1709_07469_amd import workloads as W

    probs = W.cfg4(precision=W.PREC_F64)
    n, steps, elapsed = 1, 0, 0.0
    while True:
        t0 = time.perf_counter()
        tot = 0
        for p in probs:
            S = p.n_stations
            items = np.stack([np.repeat(np.arange(S), n), np.tile(np.arange(n), S)], axis=1)
            _, st = oracle.run_paths(p, 0, items)
            tot += int((st & np.uint32(0x7FFFFFFF)).astype(np.int64).sum())
        elapsed = time.perf_counter() - t0
        steps = tot
        if elapsed >= 0.5 * seconds:
            break
        n = max(n + 1, int(n * min(8.0, 1.1 * seconds / max(elapsed, 1e-3))))
    threads = oracle.max_threads()
    cpu = host_cpu()
    res = {"value": steps / elapsed, "unit": "Brownian steps/s", "cores": threads, "kind": "oracle",
           "threads_used": threads, "cpu": cpu,
           "per_thread_steps_per_s": steps / elapsed / threads,
           "per_physical_core_steps_per_s": (steps / elapsed / min(threads, cpu["physical_cores"]))
           if cpu["physical_cores"] else None,
           "sample": f"the 32-model batch's 3936 stations x first {n} walks each (FP64 oracle): "
                     f"{steps} steps in {elapsed:.1f} s"}
    if kept:
        mixed = [p.replace(precision=W.PREC_MIXED_F64ACC) for p in probs]
        mism, rels, zs = 0, [], []
        total = 0
        for m, (gv, gs) in enumerate(kept):
            nw = len(gv)
            items = np.stack([np.zeros(nw, dtype=np.int64), np.arange(nw)], axis=1)
            ou, ost = oracle.run_paths(mixed[m], 0, items, stream=oracle.STREAM_F32)
            same = gs == ost
            mism += int((~same).sum())
            total += nw
            rels.append(np.abs(gv - ou)[same] / np.abs(ou)[same])
            zs.append(float(np.mean(gv - ou) / (np.std(ou, ddof=1) / math.sqrt(nw))))
        rel = np.concatenate(rels)
        res["paired_mixed_vs_oracle_fp32_stream"] = {
            "walks": total, "models": len(kept),
            "step_count_mismatch_frac": mism / total,
            "median_rel_diff_matching_walks": float(np.median(rel)),
            "q999_rel_diff_matching_walks": float(np.quantile(rel, 0.999)),
            "max_abs_mean_diff_in_se": float(np.max(np.abs(zs)))}
    return res


def run(a):
    import numpy as np

    from paper_1709_07469_amd import workloads as W

    legs = set(LEGS) if a.legs == "all" else set(a.legs.split(","))
    unknown = legs - set(LEGS)
    if unknown:
        raise SystemExit(f"bench.py: unknown legs {sorted(unknown)}")
    K, Wm = max(1, a.steps), max(0, a.warmup)
    result = {"metric": METRIC, "value": None, "unit": "Brownian steps/s", "n_gpus": 1, "steps": K, "warmup": Wm,
              "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "f32/f64-acc", "data": "synthetic",
              "config": {"workload": "32 voxel models (64^3 FP32 grids of 1-8 prisms, boxes of aspect 1-4), "
                                     "8-256 stations each, 1e4-1e6 walks/station, dt = 1e-3, exact prism data, "
                                     "potential; mixed precision; one persistent batched launch replayed from a "
                                     "HIP graph"}}
    kept = None
    if "headline" in legs:
        h, st, kept = batch_leg(W.PREC_MIXED_F64ACC, K, Wm, keep_walks=(8, 256) if "cpu" in legs else None)
        result["value"] = h["value"]
        result["ms_per_step"] = h["seconds_per_pass"] * 1e3
        result["config"].update({"models": 32, "stations": int(len(st)), "walks": h["walks"],
                                 "steps_per_pass": h["steps_per_pass"], "precision": "mixed", "dt": 1e-3,
                                 "workspace": "record mode (every walk's record kept)"})
        result["roofline"] = h.pop("roofline")
        result["station_estimates_per_s"] = h.pop("station_estimates_per_s")
        result["vs_closed_form"] = h.pop("vs_closed_form")
        result["headline_detail"] = h
        log("headline", result["value"])
    if "f64" in legs:
        f, _, _ = batch_leg(W.PREC_F64, min(K, 2), 1, eager_reps=1)
        result["f64"] = f
        log("f64", f["value"])
        if result["value"]:
            m_est = result["station_estimates_per_s"]["u_rel_se_1e-3"]
            f_est = f["station_estimates_per_s"]["u_rel_se_1e-3"]
            result["mixed_vs_f64"] = {
                "speedup_steps_per_s": result["value"] / f["value"],
                "speedup_at_equal_se": m_est / f_est,
                "note": "same walks and stream definition in both legs; each agrees with the closed form within "
                        "its standard errors (vs_closed_form), so equal walk counts give equal accuracy"}
    if "bounded" in legs:
        b, _, _ = batch_leg(W.PREC_MIXED_F64ACC, 1, 1, slice_walks=40_000_000, eager_reps=1)
        result["bounded_workspace"] = {k: b[k] for k in ("value", "seconds_per_pass", "workspace_bytes",
                                                         "walk_launches_per_pass", "status")}
        result["bounded_workspace"]["slice_walks"] = 40_000_000
        log("bounded", b["value"])
    for name, key, fn in (("tune", "autotune", tune_leg), ("cfg2", "si_prism", cfg2_leg),
                          ("cfg3", "grid128", cfg3_leg), ("table1", "paper_table1", paper_table1),
                          ("adjoint", "adjoint", adjoint_leg)):
        if name in legs:
            result[key] = fn()
            log(name, "done")
    if "cpu" in legs:
        result["cpu_baseline"] = cpu_baseline(a.cpu_seconds, kept)
        log("cpu", result["cpu_baseline"]["value"])
    return result


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--legs", default="all", help="comma-separated legs to run (default: all): " + " ".join(LEGS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one device-to-device copy of this many bytes (calibrates HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 (running on several GPUs -- path ranges "
              "per GPU merged by an all-gather of per-station statistics -- is not implemented)", file=sys.stderr,
              flush=True)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr, flush=True)
        sys.exit(1)
    torch.cuda.set_device(0)
    res = run(a)
    if a.copy_bytes > 0:
        src = torch.ones(a.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = int(src.numel() * 4)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
