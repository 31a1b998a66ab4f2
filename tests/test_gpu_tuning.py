"""GPU: launch settings change time only.  Results under different block
sizes, residency and queue-run lengths must be identical bit for bit (walk
records are stored by walk index and reduced in a fixed order), and the
autotuner must install and cache one of the candidate settings."""
import json
import os

import numpy as np
import pytest

from paper_1709_07469_amd import workloads as W
from gpu_helpers import gpu_solve, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision", [W.PREC_F64, W.PREC_MIXED_F64ACC])
def test_results_do_not_depend_on_launch_settings(precision):
    from paper_1709_07469_amd import fkgrav as F
    keep = F.fk_get_launch(precision)
    pr = W.cfg1(3000, precision=precision)
    ref = None
    try:
        for block, bpc, grab in ((256, 0, 32), (64, 1, 1), (128, 3, 64), (256, 1, 7)):
            F.fk_set_launch(precision, block, bpc, grab)
            for kind in (0, 1):
                st, v, s = gpu_solve(pr, kind)
                key = (st.tobytes(), v.tobytes(), s.tobytes())
                if ref is None or len(ref) < 2:
                    ref = (ref or []) + [key]
                else:
                    assert key == ref[kind], (block, bpc, grab, kind)
    finally:
        F.fk_set_launch_dict(precision, keep)


def test_autotuner_installs_and_caches_a_setting(tmp_path, monkeypatch):
    from paper_1709_07469_amd import fkgrav as F
    monkeypatch.setenv("FKGRAV_TUNE_CACHE", str(tmp_path / "tune.json"))
    import importlib

    from paper_1709_07469_amd import autotune
    importlib.reload(autotune)
    keep = F.fk_get_launch(W.PREC_MIXED_F64ACC)
    try:
        pr = W.cfg2(precision=W.PREC_MIXED_F64ACC)
        best = autotune.tune(pr, 0, tuning_walks=256)
        say("tuned", best)
        assert best["block"] in (64, 128, 256) and best["grab"] in (16, 32, 64) and best["tune_ms"] > 0
        got = F.fk_get_launch(W.PREC_MIXED_F64ACC)
        assert {k: got[k] for k in ("block", "blocks_per_cu", "grab")} == {k: best[k] for k in ("block", "blocks_per_cu", "grab")}
        cache = json.load(open(tmp_path / "tune.json"))
        assert len(cache) == 1
        F.fk_set_launch(W.PREC_MIXED_F64ACC, 64, 1, 1)
        again = autotune.apply_cached(pr, 0)
        assert again is not None and F.fk_get_launch(W.PREC_MIXED_F64ACC)["block"] == best["block"]
    finally:
        F.fk_set_launch_dict(W.PREC_MIXED_F64ACC, keep)


def test_batch_autotuner_picks_a_candidate_and_keeps_results():
    from paper_1709_07469_amd import autotune
    from paper_1709_07469_amd import fkgrav as F
    prec = W.PREC_MIXED_F64ACC
    keep = F.fk_get_launch(prec)
    probs = [m.replace(paths_per_station=400) for m in W.cfg4(n_models=3, precision=prec, n=32)]
    kinds = [0, 1, 0]
    try:
        before, _, _, _ = F.solve_batch(probs, kinds)
        best = autotune.tune_batch(probs, kinds, walk_fraction=0.25)
        say("  batch tuning picked", best)
        for knob, values in autotune.BATCH_KNOBS.items():
            assert best[knob] in values or best[knob] == keep[knob], knob
        assert best["tune_ms"] <= best["default_ms"]
        got = F.fk_get_launch(prec)
        assert all(got[k] == best[k] for k in F.LAUNCH_KEYS)
        after, _, _, _ = F.solve_batch(probs, kinds)
        for a, b in zip(before, after):
            assert a.tobytes() == b.tobytes()
    finally:
        F.fk_set_launch_dict(prec, keep)
