"""Host logic of bench.py (no GPU): the derived metrics and the rules that
attach recorded counter data to the bench line only for the kernel sources
they were taken on."""
import subprocess
import sys

import pytest

import bench


def test_station_estimates_per_s_hand_example():
    # two stations: N_s = var / (rel_se * |mean|)^2 walks of mean_steps each
    st = [{"n": 100, "mean": 2.0, "var": 4.0, "mean_steps": 10.0},
          {"n": 100, "mean": -1.0, "var": 9.0, "mean_steps": 20.0}]
    rel = 0.1
    work = 4.0 / (0.1 * 2.0) ** 2 * 10.0 + 9.0 / (0.1 * 1.0) ** 2 * 20.0   # steps for both stations
    assert bench.station_estimates_per_s(st, 1e6, rel) == pytest.approx(2 / (work / 1e6), rel=1e-15)
    # a station without a usable variance or with a zero mean is left out
    st2 = st + [{"n": 1, "mean": 5.0, "var": 0.0, "mean_steps": 1.0}, {"n": 50, "mean": 0.0, "var": 1.0,
                                                                       "mean_steps": 1.0}]
    assert bench.station_estimates_per_s(st2, 1e6, rel) == pytest.approx(4 / (work / 1e6), rel=1e-15)
    assert bench.station_estimates_per_s([], 1e6, rel) is None


def test_algorithmic_ops_are_the_sum_of_the_parts():
    c = bench.ISSUE_COST
    assert bench.algorithmic_ops_per_step("f64") == pytest.approx(
        1.5 * c["philox_block"] + 1.5 * c["box_muller_pair_f64"] + c["step_f64"])
    assert bench.algorithmic_ops_per_step("mixed") == pytest.approx(
        0.75 * c["philox_block"] + 1.5 * c["box_muller_pair_f32"] + c["step_f32_f64sum"])
    assert bench.PEAK_LANE_OPS == 256 * 4 * 16 * 2.4e9


def test_recorded_counters_apply_only_to_their_sources(monkeypatch):
    monkeypatch.setattr(bench, "PMC_BYTES", {"sources_sha256": "abc", "fetch_scale": 2.0, "write_scale": 1.0,
                                             "f64_batched": {"fetch_kib": 1.0, "write_kib": 3.0}})
    monkeypatch.setattr(bench, "VALU_COUNTERS", {"sources_sha256": "abc", "f64_batched": {
        "valu_lane_instr_per_step": 250.0, "valu_busy": 0.97, "fp64_flop_per_step": 100.0,
        "fp32_flop_per_step": 2.0}})
    monkeypatch.setattr(bench, "sources_sha256", lambda: "abc")
    assert bench.measured_traffic("f64", "batched") == 1024 * (2.0 * 1.0 + 3.0)
    c = bench.valu_counters("f64", "batched", 1e11)
    assert c["fp64_tflops"] == pytest.approx(10.0)
    assert c["fp64_frac_of_peak"] == pytest.approx(1e13 / 78.6e12)
    assert c["fp32_frac_of_peak"] == pytest.approx(2e11 / 157.3e12)
    # another launch form, or the sources changed since: no figure at all
    assert bench.measured_traffic("f64", "separate") is None
    assert bench.valu_counters("mixed", "batched", 1e11) is None
    monkeypatch.setattr(bench, "sources_sha256", lambda: "changed")
    assert bench.measured_traffic("f64", "batched") is None
    assert bench.valu_counters("f64", "batched", 1e11) is None


def test_sources_hash_covers_the_walk_kernel_sources():
    h = bench.sources_sha256()
    assert len(h) == 64 and int(h, 16) >= 0
    assert any(p.endswith("fk_walk.hip") for p in bench.TRAFFIC_SOURCES)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
