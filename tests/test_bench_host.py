"""Host logic of bench.py (no GPU): the derived metrics, the roofline entry
and the rule that attaches recorded counter data to the bench line only for
the kernel sources it was taken on."""
import subprocess
import sys

import numpy as np
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


def test_algorithmic_flop_count():
    # 1.5 Box-Muller pairs of 8, three position FMAs, three index FMAs and
    # the trapezoid term's two additions
    assert bench.ALGO_FLOP_PER_STEP == 1.5 * 8 + 3 * 2 + 3 * 2 + 2
    assert bench.PEAK_LANE_OPS == 256 * 4 * 16 * 2.4e9


def test_roofline_entry_follows_the_algorithmic_work(monkeypatch):
    monkeypatch.setattr(bench, "COUNTERS", {})
    r = bench.roofline("x", "mixed", 6e11, 2000.0, 1.2e9, grid_bytes=32 << 20)
    rate = 6e11 / 2.0
    assert r["achieved"] == pytest.approx(26 * rate / 1e12)
    assert r["peak"] == pytest.approx(157.3) and r["unit"] == "TFLOP/s" and r["bound"] == "alu"
    assert r["frac"] == pytest.approx(26 * rate / 157.3e12)
    assert r["algorithmic_bytes_per_launch"] == 1.2e9 * 36 + (32 << 20)
    assert r["traffic"] is None and r["counters"] is None
    r64 = bench.roofline("x", "f64", 6e11, 2000.0, 1.2e9)
    assert r64["peak"] == pytest.approx(78.6) and r64["frac"] == pytest.approx(26 * rate / 78.6e12)


def test_recorded_counters_apply_only_to_their_sources(monkeypatch):
    monkeypatch.setattr(bench, "COUNTERS", {"sources_sha256": "abc", "k": {
        "fetch_kib": 1.0, "write_kib": 3.0, "fetch_scale": 2.0, "write_scale": 1.0,
        "valu_lane_instr_per_step": 100.0, "valu_busy": 1.08, "fp64_flop_per_step": 2.0,
        "fp32_flop_per_step": 20.0}})
    monkeypatch.setattr(bench, "sources_sha256", lambda: "abc")
    r = bench.roofline("k", "mixed", 1e11, 1000.0, 1e6)
    assert r["traffic"] == 1024 * (2.0 * 1.0 + 3.0)
    c = r["counters"]
    assert c["valu_busy"] == 1.0                       # clamped
    assert c["valu_issue_frac"] == pytest.approx(100.0 * 1e11 / bench.PEAK_LANE_OPS)
    assert c["fp32_frac_of_peak"] == pytest.approx(20.0 * 1e11 / 157.3e12)
    assert c["fp64_frac_of_peak"] == pytest.approx(2.0 * 1e11 / 78.6e12)
    # another kernel, or the sources changed since: no figure at all
    assert bench.roofline("other", "mixed", 1e11, 1000.0, 1e6)["counters"] is None
    monkeypatch.setattr(bench, "sources_sha256", lambda: "changed")
    r = bench.roofline("k", "mixed", 1e11, 1000.0, 1e6)
    assert r["traffic"] is None and r["counters"] is None


def test_closed_form_error():
    e = bench.closed_form_error([1.0, 2.2, -3.0], [0.1, 0.1, 0.5], [1.1, 2.0, -3.0])
    assert e["stations"] == 3
    assert e["max_abs_z"] == pytest.approx(2.0)
    assert e["rms_z"] == pytest.approx(np.sqrt((1.0 + 4.0 + 0.0) / 3))
    assert e["frac_within_4se"] == 1.0
    assert e["max_rel_err"] == pytest.approx(0.1)


def test_host_cpu_description():
    c = bench.host_cpu()
    assert c["model"] and c["hardware_threads"] and c["hardware_threads"] >= 1
    assert c["physical_cores"] is None or 1 <= c["physical_cores"] <= c["hardware_threads"]


def test_sources_hash_covers_the_kernel_sources():
    h = bench.sources_sha256()
    assert len(h) == 64 and int(h, 16) >= 0
    for name in ("fk_walk.hip", "fk_device.hpp", "fk_batch.hip", "fk_stats.hpp"):
        assert any(p.endswith(name) for p in bench.TRAFFIC_SOURCES)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
