"""GPU: the paper's experiments on its own model (section 3: a ball of radius
10 km with zero data around a 100 m cube of 2000 kg/m^3; lengths in km, the
paper's walk sqrt(2) W with step sqrt(2 Delta t) being standard Brownian motion
with dt = 2 Delta t).

Each estimate is checked against the exact expectation of the discrete walk.
The ball is far away (10 km against a cube 100-300 m from the stations), so
the walk's expected trapezoid sum is that of the unbounded Gaussian walk,
    dt [ 1/2 1(x0 in cube) + sum_{n >= 1} P(x0 + sqrt(n dt) Z in cube) ],
each probability a product of three normal-CDF differences (the sum's tail
beyond n = 20000 taken from its n^(-3/2) asymptote), minus the occupation
after the walk has left the ball, which is the continuous walk's to well
below the standard errors: the Kelvin-image term G rho (V/R + x0.m1/R^3).
Replacing the sum by its continuous limit gives the Green's-function solution
(the cube's potential plus the image term); the gap between the two is the
time-step bias, which at the paper's Delta t = 0.1 is large because a step
(0.45 km) is longer than the distance to the cube.

  * experiment 1 (the line y = 50 m, z = 200 m): the estimate equals the
    discrete expectation at Delta t = 0.1 and 0.01, and the bias against the
    Green solution is what that expectation predicts;
  * experiment 2 (the vertical line x = y = 50 m through the cube);
  * experiment 3 (section 4.2): g_z on the 21 x 11 grid by central
    differences over Delta z = 1 m between independent stations, raw and after
    the moving average of section 4.1, at N = 65536 and 4194304 walks;
  * experiment 4 (section 4.4): g_z along the vertical line crossing the cube,
    where the source jumps.
The RMS errors against the analytic g_z, which the paper reports, are printed
next to their bias and noise parts."""
import math

import numpy as np
import pytest
from paper_1709_07469_amd import workloads as W
from gpu_helpers import say
from paper_expectation import discrete_potential, green_gz, green_potential

pytestmark = pytest.mark.gpu

MGAL_PER_KM_S2 = 1e8        # 1 km/s^2 = 1e3 m/s^2 = 1e8 mGal


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _event(pr):
    """The change of a common-random-number pair's sample when one point of
    one walk lies in the cube and its partner's does not: 2 w rho / (2 h)
    (w = 2 pi G dt / 2, a point counting in two trapezoid terms)."""
    return 2.0 * math.pi * pr.G * 0.5 * pr.dt * pr.prisms[0][6] / pr.h


def _z_pairs(st, pred, pr):
    """Standardised gaps of CRN pair means from their expectation.  The pair
    differences come from rare events of size _event / N, so the sample
    standard error is floored at one event (a station may see none)."""
    floor = _event(pr) / pr.paths_per_station
    return (st["mean"] - pred) / np.sqrt(st["se"] ** 2 + floor ** 2 + (1e-3 * pred / 4.0) ** 2)


def _solve(pr, kind):
    from paper_1709_07469_amd import fkgrav as F
    stats, ws, _ = F.solve(pr.replace(slice_walks=100_000_000), kind)
    del ws
    return stats


@pytest.mark.parametrize("dt_paper,deficit", [(0.1, (0.60, 0.72)), (0.01, (0.10, 0.22))])
def test_experiment1_time_step_bias(dt_paper, deficit):
    """At the paper's Delta t = 0.1 the method underestimates the potential
    100 m above the cube by about two thirds against the Green solution, and
    by about a sixth at 0.01: the estimates equal the discrete walk's
    expectation, and that expectation has this bias."""
    pr = W.paper_ball(dt_paper=dt_paper, paths_per_station=51200)
    st = _solve(pr, 0)
    pred = np.array([discrete_potential(pr, x) for x in pr.stations])
    green = np.array([green_potential(pr, x) for x in pr.stations])
    z = (st["mean"] - pred) / np.hypot(st["se"], 1e-3 * np.abs(pred) / 4.0)
    bias = 1.0 - st["mean"] / green
    say(f"exp1 dt_paper {dt_paper}: z vs discrete expectation max {np.max(np.abs(z)):.2f} rms "
        f"{np.sqrt(np.mean(z * z)):.2f}; deficit vs Green: measured {bias.min():.3f}..{bias.max():.3f} "
        f"(above the cube {bias[15]:.3f}), predicted {(1 - pred / green)[15]:.3f}; RMS rel error vs Green "
        f"{np.sqrt(np.mean(bias ** 2)):.3f}")
    assert np.all(np.abs(z) < 4.0)
    lo, hi = deficit
    assert lo < bias[15] < hi and lo < 1.0 - pred[15] / green[15] < hi


@pytest.mark.parametrize("dt_paper", [0.1, 0.01])
def test_experiment2_vertical_line(dt_paper):
    """The potential along the vertical line x = y = 50 m, z = -100 m ..
    200 m, through the cube (section 3.4; the paper: RMS 0.7 % at Delta t =
    0.01, about 7 % at 0.1)."""
    pr = W.paper_ball(dt_paper=dt_paper, paths_per_station=51200, stations=W.paper_exp2_stations())
    st = _solve(pr, 0)
    pred = np.array([discrete_potential(pr, x) for x in pr.stations])
    green = np.array([green_potential(pr, x) for x in pr.stations])
    z = (st["mean"] - pred) / np.hypot(st["se"], 1e-3 * np.abs(pred) / 4.0)
    rel = (st["mean"] - green) / np.abs(green)
    say(f"exp2 dt_paper {dt_paper}: z vs discrete expectation max {np.max(np.abs(z)):.2f}; RMS rel error vs "
        f"Green {np.sqrt(np.mean(rel ** 2)):.4f} (max {np.max(np.abs(rel)):.4f} at z = "
        f"{pr.stations[np.argmax(np.abs(rel)), 2] * 1e3:.0f} m), median rel se {np.median(st['se'] / np.abs(green)):.4f}")
    assert np.all(np.abs(z) < 4.0)


def _smooth_weights(n, k, span=5):
    """Weights of the centred moving average (shrinking at the ends) that
    gives the smoothed value k of a profile of n points."""
    r = min(span // 2, k, n - 1 - k)
    w = np.zeros(n)
    w[k - r:k + r + 1] = 1.0 / (2 * r + 1)
    return w


@pytest.mark.parametrize("N", [65536, 4194304])
def test_experiment3_gz_by_differences_and_smoothing(N):
    """Experiment 3: the potential on the 21 x 11 grid (z = 195 .. 205 m every
    metre, independent stations), g_z at z = 200 m by the central difference
    over Delta z = 1 m, raw and with each vertical profile smoothed by the
    library's moving average (span 5) first; Delta t = 0.1.  Both agree with
    the discrete expectation within their propagated standard errors, the
    smoothing cuts the standard error by (sqrt(2) / 2) / (sqrt(4) / 10) =
    3.5, and the RMS against the analytic g_z is printed beside the paper's
    (0.21 -> 0.06 at N = 65536, 0.02 -> 0.009 at N = 4194304)."""
    from paper_1709_07469_amd import fkgrav as F
    pr = W.paper_ball(dt_paper=0.1, paths_per_station=N, stations=W.paper_exp3_stations())
    st = _solve(pr, 0)
    nz = 11
    u = st["mean"].reshape(21, nz)
    se = st["se"].reshape(21, nz)
    pred = np.array([discrete_potential(pr, x) for x in pr.stations]).reshape(21, nz)
    dz = 0.001
    k0 = 5                                      # z = 200 m
    line = pr.stations.reshape(21, nz, 3)[:, k0]
    exact = np.array([green_gz(pr, x) for x in line])
    out = {}
    for name in ("raw", "smoothed"):
        if name == "raw":
            wd = np.zeros(nz)
            wd[k0 + 1], wd[k0 - 1] = 1.0, -1.0
            vals = u
        else:
            wd = _smooth_weights(nz, k0 + 1) - _smooth_weights(nz, k0 - 1)
            vals = np.empty_like(u)
            for i in range(21):
                vals[i], _ = F.fk_moving_average(u[i], se[i], span=5)
        g = (vals[:, k0 + 1] - vals[:, k0 - 1]) / (2 * dz)
        g_se = np.sqrt((se ** 2) @ (wd ** 2)) / (2 * dz)
        g_pred = (pred @ wd) / (2 * dz)
        z = (g - g_pred) / np.hypot(g_se, 1e-3 * np.abs(g_pred) / 4.0)
        rms = math.sqrt(float(np.mean((g - exact) ** 2))) * MGAL_PER_KM_S2
        bias = math.sqrt(float(np.mean((g_pred - exact) ** 2))) * MGAL_PER_KM_S2
        noise = float(np.median(g_se)) * MGAL_PER_KM_S2
        out[name] = (g_se, z)
        say(f"exp3 N {N} {name}: RMS vs analytic g_z {rms:.4f} mGal ({rms / (np.sqrt(np.mean(exact ** 2)) * MGAL_PER_KM_S2):.3f} "
            f"of the RMS g_z {np.sqrt(np.mean(exact ** 2)) * MGAL_PER_KM_S2:.3f} mGal); bias part {bias:.4f} mGal, "
            f"median se {noise:.4f} mGal; z vs discrete expectation max {np.max(np.abs(z)):.2f}")
        assert np.all(np.abs(z) < 4.0)
    ratio = float(np.median(out["raw"][0] / out["smoothed"][0]))
    say(f"exp3 N {N}: smoothing divides the standard error by {ratio:.2f}")
    assert 3.0 < ratio < 4.2


def test_experiment3_common_random_numbers():
    """The same g_z line by common-random-number pairs (fk_solve_gz, h = 1 m)
    instead of independent stations: the same expectation, a far smaller
    standard error at the same N.  At Delta t = 0.1 a pair's two walks differ
    only when one of their points falls within 2 m of a face of the cube,
    events that nearly cancel between the faces: N = 4194304 gives each
    station hundreds of them."""
    pr = W.paper_ball(dt_paper=0.1, paths_per_station=4194304,
                      stations=W.paper_exp3_stations().reshape(21, 11, 3)[:, 5]).replace(h=0.001)
    st = _solve(pr, 1)
    g_pred = np.array([(discrete_potential(pr, x + [0, 0, 0.001]) - discrete_potential(pr, x - [0, 0, 0.001])) / 0.002
                       for x in pr.stations])
    exact = np.array([green_gz(pr, x) for x in pr.stations])
    z = _z_pairs(st, g_pred, pr)
    rms = math.sqrt(float(np.mean((st["mean"] - exact) ** 2))) * MGAL_PER_KM_S2
    say(f"exp3 CRN N 4194304: RMS vs analytic g_z {rms:.4f} mGal, median se "
        f"{np.median(st['se']) * MGAL_PER_KM_S2:.5f} mGal; z vs discrete expectation max {np.max(np.abs(z)):.2f}")
    assert np.all(np.abs(z) < 4.0)


@pytest.mark.parametrize("dt_paper,N", [(0.1, 4194304), (0.01, 4194304)])
def test_experiment4_gz_across_the_source_jump(dt_paper, N):
    """Experiment 4: g_z along the vertical line x = y = 50 m through the cube
    (common-random-number pairs, h = 1 m), against the discrete expectation;
    the largest error against the difference of the exact potential (the
    paper's comparison curve) lies at a face of the cube, where the source
    jumps: a pair straddling the face differs in its start point, whose
    trapezoid weight dt/2 is large at these time steps.  (The paper's left
    panel used N = 65536 at Delta t = 0.1; more walks make the rare pair
    differences numerous enough for a standard-error test.)"""
    pr = W.paper_ball(dt_paper=dt_paper, paths_per_station=N, stations=W.paper_exp2_stations()).replace(h=0.001)
    st = _solve(pr, 1)
    e = np.array([0.0, 0.0, 0.001])
    g_pred = np.array([(discrete_potential(pr, x + e) - discrete_potential(pr, x - e)) / 0.002 for x in pr.stations])
    g_fd = np.array([(green_potential(pr, x + e) - green_potential(pr, x - e)) / 0.002 for x in pr.stations])
    z = _z_pairs(st, g_pred, pr)
    err = st["mean"] - g_fd
    worst = int(np.argmax(np.abs(err)))
    zs = pr.stations[:, 2]
    say(f"exp4 dt_paper {dt_paper} N {N}: z vs discrete expectation max {np.max(np.abs(z)):.2f}; largest error vs the "
        f"exact difference {err[worst] * MGAL_PER_KM_S2:.4f} mGal at z = {zs[worst] * 1e3:.0f} m; RMS "
        f"{np.sqrt(np.mean(err ** 2)) * MGAL_PER_KM_S2:.4f} mGal of RMS g_z "
        f"{np.sqrt(np.mean(g_fd ** 2)) * MGAL_PER_KM_S2:.4f} mGal")
    assert np.all(np.abs(z) < 4.0)
    assert min(abs(zs[worst] - 0.0), abs(zs[worst] - 0.1)) <= 0.0201
