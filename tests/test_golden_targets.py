"""The stored closed-form targets the benchmark reads
(tests/golden/closed_form_targets.json, written by make_targets.py from the
oracle's closed forms) agree with the oracle as it stands, and the layout
matches the workload generators."""
import importlib.util
import json
import os

import numpy as np

from paper_1709_07469_amd import workloads as W

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _stored():
    with open(os.path.join(HERE, "closed_form_targets.json")) as f:
        return json.load(f)


def test_targets_match_the_oracle():
    spec = importlib.util.spec_from_file_location("make_targets", os.path.join(HERE, "make_targets.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    fresh = mod.targets()
    stored = _stored()
    np.testing.assert_allclose(stored["cfg2"]["u"], fresh["cfg2"]["u"], rtol=1e-15, atol=0)
    np.testing.assert_allclose(stored["cfg2"]["gz"], fresh["cfg2"]["gz"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(stored["cfg2"]["gz_fd_h"], fresh["cfg2"]["gz_fd_h"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(stored["cfg3"]["u"], fresh["cfg3"]["u"], rtol=1e-15, atol=0)
    for a, b in zip(stored["cfg4"]["u"], fresh["cfg4"]["u"]):
        np.testing.assert_allclose(a, b, rtol=1e-15, atol=0)


def test_targets_layout_and_physics():
    t = _stored()
    assert len(t["cfg2"]["u"]) == 64 and len(t["cfg3"]["u"]) == 256
    models = W.cfg4()
    assert [len(u) for u in t["cfg4"]["u"]] == [m.n_stations for m in models]
    # positive masses: negative potential, downward pull (g_z > 0 with z up)
    assert all(v < 0 for v in t["cfg2"]["u"]) and all(v > 0 for v in t["cfg2"]["gz"])
    # the central difference at h = 2 m is within 1e-3 of the analytic g_z here
    np.testing.assert_allclose(t["cfg2"]["gz_fd_h"], t["cfg2"]["gz"], rtol=1e-3)
    assert all(v < 0 for u in t["cfg4"]["u"] for v in u)
