#!/usr/bin/env python3
"""Benchmark of the Monte Carlo Feynman-Kac gravity solver on one MI355X.

One step is one pass of the hot path over the benchmark problem: the
potential u and the vertical acceleration g_z (common-random-number central
difference) at all 64 stations of the SI-prism workload -- box
[0,1000]^2 x [-500,100] m, one prism [400,600]x[450,550]x[-300,-150] m of
300 kg/m^3, exact prism data on the faces, 1e5 walks per station,
sqrt(dt) = 2 m, FP64 -- by default as one persistent launch over both
(--launch separate: two launches).  Inputs live in device memory before
timing starts.

Prints one JSON line: Brownian steps per second of the whole job (exact
in-kernel step counts over the event-timed region), the ALU roofline of the
walk kernel, station estimates per second at fixed relative standard error,
the mixed-precision kernel on the same workload, the paper's Table 1
workload (its experiment 1 at every time step and walk count, next to the
K20Xm times it reports), the 32-model batched workload in one graph-captured
launch (default and autotuned launch settings), the adjoint d g_z / d rho on
a voxel workload next to its forward solve, and the CPU oracle timed on a
bounded sample on the host.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision f64|mixed]
                  [--launch batched|separate] [--no-cpu-baseline] [--cpu-seconds S]
                  [--no-paper-table] [--no-batched-models] [--no-adjoint]
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

# Peak full-rate VALU issue of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# lane-operations per second (the same count that gives 78.6 TFLOP/s of FP64
# FMA at 2 FLOP per lane-op).  One "lane-slot" is one such operation.
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# MI355X's published vector peaks: FP64 78.6 TFLOP/s; FP32 157.3 TFLOP/s
# (packed FP32, which these kernels do not use; 78.6 without it).
PEAK_F64_FLOPS = 78.6e12
PEAK_F32_FLOPS = 157.3e12

# Issue cost, in lane-slots, of the parts one Euler-Maruyama step is made of,
# each measured alone on MI355X by paper_1709_07469_amd/fk_issue_probe (eight
# dependent chains per lane, so nothing folds or stalls on latency):
#   philox_block          one Philox4x32-10 block (10 rounds)
#   box_muller_pair_*     uniform bits -> two normals (FP64: software log,
#                         sqrt and sincos; FP32: the hardware units)
#   step_*                position update, density of one analytic prism,
#                         trapezoid sum and exit test (FP64; FP32 with an
#                         FP64 sum)
ISSUE_COST = {"philox_block": 60.82, "box_muller_pair_f64": 79.46, "box_muller_pair_f32": 20.31,
              "step_f64": 29.54, "step_f32_f64sum": 25.01}

# HBM bytes of the walk kernels on this workload, from two rocprofv3 --pmc
# runs of this script (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch averaged
# over the launches of each form), each scaled by what the same counter reads for
# a 1 GiB device-to-device copy.  They describe the kernel sources hashed in
# "sources_sha256" only; for any other source the traffic is reported as null.
PMC_BYTES = {
    "sources_sha256": "7e95cd34b6c3e8ae15958d54f1bd9b4bda9fb76400ceb974b20135f0f609960d",
    "fetch_scale": 1.9998796058653638, "write_scale": 1.0,
    "f64_batched": {"fetch_kib": 153.75, "write_kib": 868267.125},
    "f64_separate": {"fetch_kib": 1894.25, "write_kib": 444061.8828125},
    "mixed_batched": {"fetch_kib": 151.84375, "write_kib": 914944.671875},
    "mixed_separate": {"fetch_kib": 14555.109375, "write_kib": 491642.7890625},
}
# VALU counters of the walk kernels per Brownian step (rocprofv3 --pmc
# SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, GRBM_GUI_ACTIVE and the
# SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F{64,32} counts, FLOP = ADD + MUL + 2 FMA +
# TRANS, each times 64 lanes), recorded like PMC_BYTES for the sources hashed
# in "sources_sha256"; with the measured steps/s they give the fractions of
# the FP64 and FP32 vector peaks.
VALU_COUNTERS = {
    "sources_sha256": "7e95cd34b6c3e8ae15958d54f1bd9b4bda9fb76400ceb974b20135f0f609960d",
    "f64_batched": {"valu_lane_instr_per_step": 250.3, "valu_busy": 0.968, "fp64_flop_per_step": 108.15, "fp32_flop_per_step": 0.07},
    "f64_separate": {"valu_lane_instr_per_step": 252.2, "valu_busy": 0.9492, "fp64_flop_per_step": 109.15, "fp32_flop_per_step": 0.13},
    "mixed_batched": {"valu_lane_instr_per_step": 105.7, "valu_busy": 1.0852, "fp64_flop_per_step": 2.2, "fp32_flop_per_step": 20.55},
    "mixed_separate": {"valu_lane_instr_per_step": 105.3, "valu_busy": 1.0382, "fp64_flop_per_step": 2.5, "fp32_flop_per_step": 21.56},
}
TRAFFIC_SOURCES = ("paper_1709_07469_amd/csrc/fk_walk.hip", "paper_1709_07469_amd/csrc/fk_device.hpp",
                   "paper_1709_07469_amd/csrc/fk_internal.hpp")


def algorithmic_ops_per_step(precision: str) -> float:
    """Lane-slots one step of the benchmark problem needs: 1.5 Philox blocks
    and 1.5 Box-Muller pairs (FP64 stream: one pair per block) or 0.75 blocks
    and 1.5 pairs (FP32 stream: two pairs per block) for the 3 normals, plus
    the step itself."""
    c = ISSUE_COST
    if precision == "f64":
        return 1.5 * c["philox_block"] + 1.5 * c["box_muller_pair_f64"] + c["step_f64"]
    return 0.75 * c["philox_block"] + 1.5 * c["box_muller_pair_f32"] + c["step_f32_f64sum"]


def sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(precision: str, mode: str):
    """HBM bytes per walk-kernel launch from the recorded counters, or None
    when they were taken on other kernel sources or another launch form."""
    key = precision + "_" + mode
    if not PMC_BYTES or PMC_BYTES.get("sources_sha256") != sources_sha256() or key not in PMC_BYTES:
        return None
    r = PMC_BYTES[key]
    return r["fetch_kib"] * 1024 * PMC_BYTES["fetch_scale"] + r["write_kib"] * 1024 * PMC_BYTES["write_scale"]


def valu_counters(precision: str, mode: str, kernel_steps_per_s: float):
    """The walk kernel's counters per Brownian step and the FLOP rates they
    give at the kernel's measured steps/s, or None when they were taken on
    other kernel sources or another launch form."""
    key = precision + "_" + mode
    if not VALU_COUNTERS or VALU_COUNTERS.get("sources_sha256") != sources_sha256() or key not in VALU_COUNTERS:
        return None
    c = VALU_COUNTERS[key]
    f64 = c["fp64_flop_per_step"] * kernel_steps_per_s
    f32 = c["fp32_flop_per_step"] * kernel_steps_per_s
    return {"valu_busy": c["valu_busy"], "valu_lane_instr_per_step": c["valu_lane_instr_per_step"],
            "fp64_flop_per_step": c["fp64_flop_per_step"], "fp32_flop_per_step": c["fp32_flop_per_step"],
            "fp64_tflops": f64 / 1e12, "fp64_frac_of_peak": f64 / PEAK_F64_FLOPS,
            "fp32_tflops": f32 / 1e12, "fp32_frac_of_peak": f32 / PEAK_F32_FLOPS}


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


def cpu_baseline(prob, seconds):
    """The oracle on the host cores: the first n walks of every station, u
    and g_z, n grown until about `seconds` of work."""
    import numpy as np

    import oracle
    S = prob.n_stations
    n, elapsed, steps = 2, 0.0, 0
    while True:
        t0 = time.perf_counter()
        tot = 0
        for kind in (0, 1):
            items = np.stack([np.repeat(np.arange(S), n), np.tile(np.arange(n), S)], axis=1)
            _, st = oracle.run_paths(prob, kind, items)
            tot += int((st & np.uint32(0x7FFFFFFF)).astype(np.int64).sum())
        elapsed = time.perf_counter() - t0
        steps = tot
        if elapsed >= 0.6 * seconds or n >= prob.paths_per_station:
            break
        n = min(prob.paths_per_station, max(n + 1, int(n * min(8.0, 1.1 * seconds / max(elapsed, 1e-3)))))
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": steps / elapsed, "unit": "Brownian steps/s", "cores": oracle.max_threads(), "kind": "oracle",
            "cpu": cpu,
            "sample": f"all {S} stations x first {n} walks, u and g_z (FP64): {steps} steps in {elapsed:.1f} s"}


# The paper's Table 1: seconds on one Tesla K20Xm for experiment 1 (31
# stations, potential) at its time steps Delta t and walk counts N, read from
# tests/golden/paper_experiments.txt.  Lengths are read as km (the only unit
# that makes these times consistent with the expected exit time of the 10 km
# ball).
def paper_table1_reference():
    n, rows = None, {}
    with open(os.path.join(ROOT, "tests", "golden", "paper_experiments.txt")) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] == "table1_N":
                n = tuple(int(v) for v in w[1:])
            elif w[0] == "table1":
                rows[float(w[1])] = tuple(float(v) for v in w[2:])
    return n, rows


def paper_table1(precision_name):
    """Experiment 1 of the paper (ball of radius 10 km, zero data, 100 m cube,
    31 stations) at every cell of Table 1: seconds per solve on this GPU
    (event-timed, median of 3, inputs resident) next to the K20Xm's."""
    import numpy as np
    import torch

    from paper_1709_07469_amd import fkgrav as F
    from paper_1709_07469_amd import workloads as W

    prec = W.PREC_F64 if precision_name == "f64" else W.PREC_MIXED_F64ACC
    table_n, table_s = paper_table1_reference()
    rows, ours_total, paper_total, steps_total = [], 0.0, 0.0, 0
    for dtp, paper_s in table_s.items():
        row = []
        for N, ps in zip(table_n, paper_s):
            prob = W.paper_ball(dt_paper=dtp, paths_per_station=N, precision=prec)
            P = F.Prepared(prob)
            ws = F.alloc_workspace(F.fk_workspace_bytes(0, prob.n_stations, P.params))
            out = F.alloc_stats(prob.n_stations)
            F.fk_solve_potential(P.stations, P.box, P.source, P.bc, P.params, out, ws)
            times = []
            for _ in range(3):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                F.fk_solve_potential(P.stations, P.box, P.source, P.bc, P.params, out, ws)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1) / 1e3)
            t = float(np.median(times))
            st = F.stats_to_numpy(out)[: prob.n_stations]
            steps_total += int(st["sum_steps"].sum())
            ours_total += t
            paper_total += ps
            row.append(round(t, 5))
        rows.append({"dt_paper": dtp, "seconds": row, "paper_k20xm_seconds": list(paper_s)})
    return {"workload": "paper experiment 1: ball R = 10 km (lengths in km), zero data, cube [0,100 m]^3 of "
                        "2000 kg/m^3, 31 stations y = 50 m, z = 200 m, x = -100..200 m; potential",
            "precision": precision_name, "N": list(table_n), "rows": rows,
            "total_seconds": ours_total, "paper_total_seconds": paper_total,
            "speedup_vs_paper_total": paper_total / ours_total, "steps": steps_total,
            "steps_per_s": steps_total / ours_total}


def make_stepper(prob, mode):
    """One pass of the hot path over the benchmark problem: u and g_z at all
    stations, either as two launches (mode "separate") or as one persistent
    launch over both (mode "batched").  Returns (step, stats) where stats()
    gives the u and g_z station statistics of the last pass."""
    from paper_1709_07469_amd import fkgrav as F

    S = prob.n_stations
    if mode == "batched":
        PB = F.PreparedBatch([prob, prob], [0, 1])
        ws = F.alloc_workspace(F.fk_batch_workspace_bytes(PB.problems))
        out = F.alloc_stats(PB.n_out)

        def step():
            F.fk_solve_batch(PB.problems, out, ws)

        def stats():
            st = F.stats_to_numpy(out)
            return st[:S], st[S:2 * S]
        return step, stats
    P = F.Prepared(prob)
    ws_u = F.alloc_workspace(F.fk_workspace_bytes(0, S, P.params))
    ws_g = F.alloc_workspace(F.fk_workspace_bytes(1, S, P.params))
    out_u, out_g = F.alloc_stats(S), F.alloc_stats(S)

    def step():
        F.fk_solve_potential(P.stations, P.box, P.source, P.bc, P.params, out_u, ws_u)
        F.fk_solve_gz(P.stations, P.box, P.source, P.bc, P.params, out_g, ws_g)

    def stats():
        return F.stats_to_numpy(out_u)[:S], F.stats_to_numpy(out_g)[:S]
    return step, stats


def timed(step, K, Wm, walk_timing=False):
    """Wm untimed passes, then K passes between two events; returns seconds
    and (optionally) the walk kernels' own event times in ms."""
    import torch

    from paper_1709_07469_amd import fkgrav as F
    for _ in range(Wm):
        step()
    torch.cuda.synchronize()
    if walk_timing:
        F.fk_timing_read()
        F.fk_timing_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(K):
        step()
    e1.record()
    torch.cuda.synchronize()
    walk_ms = None
    if walk_timing:
        F.fk_timing_enable(False)
        walk_ms = F.fk_timing_read()
    return e0.elapsed_time(e1) / 1e3, walk_ms


def batched_models():
    """The uneven batched workload: 32 random 64^3 voxel models (1-8 prisms
    each, 8-256 stations, 1e4-1e6 walks per station), mixed precision, in one
    persistent launch captured in a HIP graph; timed with the default launch
    setting and with the one the autotuner picks on the same batch at 5 % of
    its walks."""
    import torch

    from paper_1709_07469_amd import autotune
    from paper_1709_07469_amd import fkgrav as F
    from paper_1709_07469_amd import workloads as W

    probs = W.cfg4()
    kinds = [0] * len(probs)
    PB = F.PreparedBatch(probs, kinds)
    ws = F.alloc_workspace(F.fk_batch_workspace_bytes(PB.problems))
    out = F.alloc_stats(PB.n_out)

    def graph_seconds():
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            F.fk_solve_batch(PB.problems, out, ws)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            F.fk_solve_batch(PB.problems, out, ws)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    keep = F.fk_get_launch(W.PREC_MIXED_F64ACC)
    t_default = graph_seconds()
    steps = int(F.stats_to_numpy(out)[:PB.n_out]["sum_steps"].sum())
    tuned = autotune.tune_batch(probs, kinds, walk_fraction=0.05)
    t_tuned = graph_seconds()
    F.fk_set_launch(W.PREC_MIXED_F64ACC, keep["block"], keep["blocks_per_cu"], keep["grab"])
    del ws
    torch.cuda.empty_cache()
    return {"workload": "32 voxel models (64^3 FP32 grids, 1-8 prisms), 8-256 stations, 1e4-1e6 walks/station, "
                        "mixed precision, one graph-captured persistent launch",
            "models": len(probs), "stations": PB.n_out,
            "walks": int(sum(p.n_stations * p.paths_per_station for p in probs)), "steps": steps,
            "default": {"seconds": t_default, "steps_per_s": steps / t_default, "launch": keep},
            "tuned": {"seconds": t_tuned, "steps_per_s": steps / t_tuned,
                      "launch": {k: tuned[k] for k in ("block", "blocks_per_cu", "grab")}}}


def adjoint_leg(reps=2):
    """d g_z / d rho on the voxel workload (32^3 FP32 grid of 5 prisms, 32
    stations, 1e6 common-random-number walk pairs, zero data, FP64): the
    forward g_z solve and the adjoint replay of the same walks (occupation
    counts and their combination into one gradient), each timed with events
    over `reps` runs after one warm-up."""
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
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
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


def run(precision_name, K, Wm, cpu_seconds, want_cpu, want_paper=True, mode="batched", want_models=True,
        want_adjoint=True):
    import numpy as np

    from paper_1709_07469_amd import workloads as W

    prec = W.PREC_F64 if precision_name == "f64" else W.PREC_MIXED_F64ACC
    prob = W.cfg2(precision=prec)
    S = prob.n_stations
    step, stats = make_stepper(prob, mode)
    elapsed, walk_ms = timed(step, K, Wm, walk_timing=True)
    su, sg = stats()
    steps_per_pass = int(su["sum_steps"].sum()) + int(sg["sum_steps"].sum())
    value = steps_per_pass * K / elapsed

    ops = algorithmic_ops_per_step(precision_name)
    achieved = steps_per_pass * K * ops / (sum(walk_ms) * 1e-3) / 1e12
    peak = PEAK_LANE_OPS / 1e12
    launches_per_pass = len(walk_ms) // K
    walks_per_launch = 3 * S * prob.paths_per_station / launches_per_pass   # u: S*N walks, g_z: 2*S*N
    algo_bytes = walks_per_launch * (32 + 4)                     # exit record + step count per walk
    traffic = measured_traffic(precision_name, mode)
    kname = "walk_kernel" if mode == "separate" else "batch_walk_kernel"
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "T lane-slots/s", "frac": achieved / peak,
            "traffic": traffic,
            "kernel": kname + ("<F64>" if precision_name == "f64" else "<F32, F64 sum>"),
            "ops_per_step": ops, "steps_per_launch": steps_per_pass / launches_per_pass,
            "kernel_avg_ms": float(np.mean(walk_ms)), "launches": len(walk_ms),
            "kernel_share_of_step": sum(walk_ms) / (elapsed * 1e3),
            "algorithmic_bytes_per_launch": algo_bytes,
            "traffic_over_algorithmic": None if traffic is None else traffic / algo_bytes,
            "counters": valu_counters(precision_name, mode, steps_per_pass * K / (sum(walk_ms) * 1e-3))}

    rows_u = [dict(zip(su.dtype.names, r)) for r in su.tolist()]
    rows_g = [dict(zip(sg.dtype.names, r)) for r in sg.tolist()]
    est = {"u_rel_se_1e-3": station_estimates_per_s(rows_u, value, 1e-3),
           "gz_rel_se_1e-2": station_estimates_per_s(rows_g, value, 1e-2)}

    result = {
        "metric": METRIC, "value": value, "unit": "Brownian steps/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": elapsed * 1e3 / K, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if precision_name == "f64" else "f32-step/f64-acc", "data": "synthetic",
        "config": {"workload": "SI prism 300 kg/m^3 in box [0,1000]^2x[-500,100] m, 8x8 stations at z=0, "
                               "1e5 walks/station, sqrt(dt)=2 m, exact prism data, u + g_z (CRN, h=2 m)",
                   "stations": S, "paths_per_station": prob.paths_per_station, "dt": prob.dt,
                   "precision": precision_name, "launch": mode, "steps_per_pass": steps_per_pass},
        "roofline": roof,
        "station_estimates_per_s": est,
    }

    if precision_name == "f64":
        # the same pass in the other launch form, and the mixed-precision
        # kernel in both forms -- outside the timed region
        other = "separate" if mode == "batched" else "batched"
        ostep, ostats = make_stepper(prob, other)
        oel, _ = timed(ostep, K, 1)
        result["f64_" + other] = {"value": steps_per_pass * K / oel, "unit": "Brownian steps/s"}
        pmix = prob.replace(precision=W.PREC_MIXED_F64ACC)
        mstep, mstats = make_stepper(pmix, "batched")
        mel, mwalk_ms = timed(mstep, K, 1, walk_timing=True)
        mu, mg = mstats()
        msteps = int(mu["sum_steps"].sum()) + int(mg["sum_steps"].sum())
        mval = msteps * K / mel
        sstep, _ = make_stepper(pmix, "separate")
        sel, _ = timed(sstep, K, 1)
        # the two kernels turn the same Philox words into different normals
        # (FP32 and FP64 streams), so their estimates are neither equal nor
        # independent: differences are scaled by sqrt(se_a^2 + se_b^2), the
        # standard error of the difference of independent estimates, as a
        # rough scale only
        zu = (mu["mean"] - su["mean"]) / np.hypot(mu["se"], su["se"])
        zg = (mg["mean"] - sg["mean"]) / np.hypot(mg["se"], sg["se"])
        du, dg = float(np.max(np.abs(zu))), float(np.max(np.abs(zg)))
        mach = msteps * K * algorithmic_ops_per_step("mixed") / (sum(mwalk_ms) * 1e-3) / 1e12
        result["mixed"] = {"value": mval, "unit": "Brownian steps/s", "launch": "batched",
                           "speedup_vs_f64": mval / value,
                           "roofline": {"bound": "alu", "achieved": mach, "peak": peak, "unit": "T lane-slots/s",
                                        "frac": mach / peak, "traffic": measured_traffic("mixed", "batched"),
                                        "kernel": "batch_walk_kernel<F32, F64 sum>",
                                        "ops_per_step": algorithmic_ops_per_step("mixed"),
                                        "kernel_avg_ms": float(np.mean(mwalk_ms)),
                                        "counters": valu_counters("mixed", "batched",
                                                                  msteps * K / (sum(mwalk_ms) * 1e-3))},
                           "separate_value": msteps * K / sel,
                           "station_estimates_per_s": {
                               "u_rel_se_1e-3": station_estimates_per_s(
                                   [dict(zip(mu.dtype.names, r)) for r in mu.tolist()], mval, 1e-3),
                               "gz_rel_se_1e-2": station_estimates_per_s(
                                   [dict(zip(mg.dtype.names, r)) for r in mg.tolist()], mval, 1e-2)},
                           "max_abs_diff_vs_f64_in_combined_se": {"u": du, "g_z": dg},
                           # over the 64 stations (about 1 for independent estimates)
                           "rms_diff_vs_f64_in_combined_se": {"u": float(np.sqrt(np.mean(zu * zu))),
                                                              "g_z": float(np.sqrt(np.mean(zg * zg)))}}

    if want_paper:
        result["paper_table1"] = paper_table1(precision_name)
    if want_adjoint and precision_name == "f64":
        result["adjoint"] = adjoint_leg()
    if want_models and precision_name == "f64":
        result["batched_models"] = batched_models()
    if want_cpu:
        result["cpu_baseline"] = cpu_baseline(prob, cpu_seconds)
    return result


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["f64", "mixed"], default="f64")
    ap.add_argument("--launch", choices=["batched", "separate"], default="batched",
                    help="u and g_z in one persistent launch (default) or in two")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper-table", action="store_true", help="skip the paper's Table 1 workload")
    ap.add_argument("--no-batched-models", action="store_true", help="skip the 32-model batched workload")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint workload")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="also run one device-to-device copy of this many bytes (calibrates HBM byte counters)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 (running on several GPUs -- path ranges "
              "per GPU merged by an all-gather of per-station statistics -- is not implemented)", file=sys.stderr, flush=True)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr, flush=True)
        sys.exit(1)
    torch.cuda.set_device(0)
    res = run(a.precision, max(1, a.steps), max(0, a.warmup), a.cpu_seconds, not a.no_cpu_baseline,
              not a.no_paper_table, a.launch, not a.no_batched_models, not a.no_adjoint)
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
