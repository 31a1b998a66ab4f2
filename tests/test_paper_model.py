"""The paper's own model and experiments (section 3) as the workload
generators build them, against the values the paper prints
(tests/golden/paper_experiments.txt): ball radius, cube, density, the
stations of experiments 1 and 2, and the shape of Table 1 that the
benchmark times."""
import os

import numpy as np
import pytest

from paper_1709_07469_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_experiments.txt")


def _golden():
    g = {}
    for line in open(GOLDEN):
        w = line.split()
        if not w or w[0].startswith("#"):
            continue
        g.setdefault(w[0], []).append(w[1:])
    return g


def test_model_matches_the_paper():
    g = _golden()
    m = {r[0]: [float(v) for v in r[1:]] for r in g["model"]}
    pr = W.paper_ball(dt_paper=0.1, paths_per_station=2)
    km = 1000.0
    assert pr.domain == W.DOMAIN_BALL
    assert np.allclose(0.5 * (pr.box_hi - pr.box_lo) * km, m["ball_radius_m"][0])
    assert np.allclose(0.5 * (pr.box_hi + pr.box_lo), 0.0)
    assert np.allclose(pr.prisms[0, :3] * km, m["cube_lo_m"]) and np.allclose(pr.prisms[0, 3:6] * km, m["cube_hi_m"])
    # density x G is unit-free: 2000 kg/m^3 x 6.674e-11 m^3 kg^-1 s^-2
    assert pr.prisms[0, 6] * pr.G == pytest.approx(m["density_kg_m3"][0] * W.G_SI, rel=1e-12)
    assert pr.bc_kind == W.BC_ZERO


def test_experiment_stations_match_the_paper():
    g = _golden()
    e1 = {r[0]: float(r[1]) for r in g["exp1"]}
    e2 = {r[0]: float(r[1]) for r in g["exp2"]}
    s1 = W.paper_exp1_stations() * 1000.0
    x = np.arange(e1["x_first_m"], e1["x_last_m"] + 0.5, e1["x_step_m"])
    assert s1.shape == (len(x), 3) and len(x) == 31
    assert np.allclose(s1[:, 0], x) and np.allclose(s1[:, 1], e1["y_m"]) and np.allclose(s1[:, 2], e1["z_m"])
    s2 = W.paper_exp2_stations() * 1000.0
    z = np.arange(e2["z_first_m"], e2["z_last_m"] + 0.5, e2["z_step_m"])
    assert np.allclose(s2[:, 2], z) and np.allclose(s2[:, 0], e2["x_m"]) and np.allclose(s2[:, 1], e2["y_m"])


def test_table1_shape_and_time_step_reading():
    g = _golden()
    n = [int(v) for v in g["table1_N"][0]]
    rows = {float(r[0]): [float(v) for v in r[1:]] for r in g["table1"]}
    assert len(n) == 8 and sorted(rows) == [0.001, 0.005, 0.01, 0.05, 0.1]
    assert all(len(v) == 8 for v in rows.values())
    # times grow with N and shrink with Delta t, as the paper's table does
    for dt, v in rows.items():
        assert all(b >= a for a, b in zip(v, v[1:]))
    # the paper's walk sqrt(2) W with step sqrt(2 Delta t) is standard
    # Brownian motion with dt = 2 Delta t
    assert W.paper_ball(dt_paper=0.01, paths_per_station=2).dt == pytest.approx(0.02)


def test_discrete_walk_expectation_pins():
    """The discrete walk's expectation for the paper's model (used by the GPU
    experiment tests) tends to the Green solution as dt -> 0, and at the
    paper's Delta t = 0.1 the oracle's own walks agree with it (and so show
    the same two-thirds deficit against the Green solution)."""
    import oracle
    from paper_expectation import discrete_potential, green_potential
    pr = W.paper_ball(dt_paper=1e-4)
    x0 = W.paper_exp1_stations()[15]
    assert abs(discrete_potential(pr, x0) / green_potential(pr, x0) - 1.0) < 2e-3
    pr = W.paper_ball(dt_paper=0.1, paths_per_station=4000, stations=W.paper_exp1_stations()[::5])
    stats, _, _ = oracle.solve(pr, 0)
    for s, x in enumerate(pr.stations):
        pred = discrete_potential(pr, x)
        assert abs(stats[s]["mean"] - pred) < 4.0 * stats[s]["se"] + 1e-3 * abs(pred)
    assert 0.6 < 1.0 - discrete_potential(pr, pr.stations[3]) / green_potential(pr, pr.stations[3]) < 0.72
