"""Pins for the oracle's ball domain (the paper's Omega, section 3: a ball of
radius 10 km with zero data), against facts fixed by the mathematics rather
than by the oracle's own code:

* the Dirichlet solution for a uniform ball source inside a ball domain with
  zero data is the source's potential minus its Kelvin image (the Green's
  function of the ball); given that solution's exterior continuation as data,
  the overshoot estimator is unbiased up to the O(dt) trapezoid error;
* constant density with the quadratic data (2/3) pi G rho |x - c|^2 + h
  (h harmonic), and zero density with harmonic data: exact at any dt,
  because |X_n - c|^2 - 3 n dt is a martingale and harmonic quadratics have
  the Gaussian mean-value property;
* a Gaussian random walk overshoots a smooth boundary by beta sqrt(dt) on
  average, beta = -zeta(1/2) / sqrt(2 pi) = 0.5826 (Siegmund's constant),
  which pins the exit test's centre, radius and direction;
* the INTERSECT rule puts every exit point on the sphere.
"""
import numpy as np
import pytest

import oracle
from paper_1709_07469_amd import workloads as W

C0 = np.array([0.3, -0.2, 0.1])        # ball centre (box [C0 - 1, C0 + 1])
R = 1.0
STATIONS = np.array([C0 + [0.0, 0.0, 0.5], C0 + [0.4, -0.3, 0.2], C0 + [-0.2, 0.1, 0.0]])


def _ball(**kw):
    base = dict(box_lo=C0 - R, box_hi=C0 + R, stations=STATIONS, G=1.0, domain=W.DOMAIN_BALL)
    base.update(kw)
    return W.Problem(**base)


def test_kelvin_image_solution():
    # uniform ball source (radius a, centre y0) in the ball domain, zero data:
    # u = Phi_source + G M (R/|d|) / |x - y*|,  d = y0 - c,  y* = c + R^2 d / |d|^2.
    # The data is that solution continued outside: point masses M at y0 and
    # -M R/|d| at y*, which vanishes on the sphere.
    y0, a, rho, G = C0 + np.array([0.15, 0.1, -0.35]), 0.2, 1.0, 1.0
    M = 4.0 / 3.0 * np.pi * a ** 3 * rho
    d = y0 - C0
    ys = C0 + R * R * d / np.dot(d, d)
    mi = -M * R / np.linalg.norm(d)
    for sp in (C0 + [R, 0, 0], C0 + np.array([0.6, -0.48, 0.64])):      # on the sphere
        g = -G * (M / np.linalg.norm(sp - y0) + mi / np.linalg.norm(sp - ys))
        assert abs(g) < 1e-14
    pr = _ball(dt=4e-3, paths_per_station=100000, spheres=np.array([[*y0, a, rho]]),
               bc_kind=W.BC_POINT_MASSES, bc_data=np.array([*y0, M, *ys, mi]))
    stats, _, _ = oracle.solve(pr, 0)
    for s, x in zip(stats, STATIONS):
        exact = oracle.sphere_potential(y0, a, rho, G, x) - G * mi / np.linalg.norm(x - ys)
        assert abs(s["mean"] - exact) < 4.0 * s["se"], (x, s["mean"], exact, s["se"])


def test_constant_density_quadratic_data_is_exact():
    # rho = rho0 on every point a walk can reach (a source ball far larger than
    # the domain), data (2/3) pi G rho0 |x - c|^2 + 1 + 0.3 x - 0.2 z + x y
    G, rho0, dt = 1.3, 0.7, 4e-3
    k = 2.0 / 3.0 * np.pi * G * rho0
    c = C0
    b = np.array([0.3, 0.0, -0.2]) - 2.0 * k * c
    q = np.array([1.0 + k * np.dot(c, c), *b, k, 0.5, 0.0, k, 0.0, k])
    pr = _ball(dt=dt, paths_per_station=40000, G=G, spheres=np.array([[*c, 3.0 * R, rho0]]),
               bc_kind=W.BC_QUADRATIC, bc_data=q)
    stats, _, _ = oracle.solve(pr, 0)
    for s, x in zip(stats, STATIONS):
        target = k * np.dot(x - c, x - c) + 1.0 + 0.3 * x[0] - 0.2 * x[2] + x[0] * x[1]
        assert abs(s["mean"] - target) < 4.0 * s["se"], (x, s["mean"], target, s["se"])


def test_harmonic_data_mean_value_property():
    # rho = 0, data x^2 - y^2 + 2 y z + 0.5 x: E[u_p] = h(x0) for any dt
    q = np.array([0.0, 0.5, 0.0, 0.0, 1.0, 0.0, 0.0, -1.0, 1.0, 0.0])
    pr = _ball(dt=4e-3, paths_per_station=40000, bc_kind=W.BC_QUADRATIC, bc_data=q)
    stats, _, _ = oracle.solve(pr, 0)
    for s, x in zip(stats, STATIONS):
        h = x[0] ** 2 - x[1] ** 2 + 2 * x[1] * x[2] + 0.5 * x[0]
        assert abs(s["mean"] - h) < 4.0 * s["se"], (x, s["mean"], h, s["se"])


def test_overshoot_constant_and_exit_time_identity():
    dt, n = 1e-4, 2000
    pr = _ball(dt=dt, paths_per_station=n, stations=STATIONS[:1])
    items = np.stack([np.zeros(n, np.int64), np.arange(n)], 1)
    _, steps, _, xe = oracle.run_paths(pr, 0, items, want_exit=True)
    r = np.linalg.norm(xe - C0, axis=1)
    assert r.min() >= R
    ov = (r - R) / np.sqrt(dt)
    beta = 0.5826
    assert abs(ov.mean() - beta) < 4.0 * ov.std() / np.sqrt(n) + 0.02
    # optional stopping of |X_n - c|^2 - 3 n dt
    D = np.sum((xe - C0) ** 2, axis=1) - np.sum((STATIONS[0] - C0) ** 2) - 3.0 * dt * steps.astype(np.float64)
    assert abs(D.mean()) < 4.0 * D.std() / np.sqrt(n)


def test_intersect_exit_points_lie_on_the_sphere():
    n = 3000
    pr = _ball(dt=4e-3, paths_per_station=n, stations=STATIONS[:1])
    items = np.stack([np.zeros(n, np.int64), np.arange(n)], 1)
    _, so, _, xo = oracle.run_paths(pr, 0, items, want_exit=True)
    _, si, _, xi = oracle.run_paths(pr, 0, items, want_exit=True, exit_rule=W.EXIT_INTERSECT)
    assert np.array_equal(so, si)                                   # same walks, same exit step
    assert np.max(np.abs(np.sum((xi - C0) ** 2, axis=1) - R * R)) < 1e-13
    # the intersection lies before the overshoot point, within one step of it
    assert np.all(np.linalg.norm(xo - C0, axis=1) >= np.linalg.norm(xi - C0, axis=1) - 1e-15)
    assert np.max(np.linalg.norm(xo - xi, axis=1)) < 7.0 * np.sqrt(3 * 4e-3)


def test_paper_model_geometry():
    # the paper's model in km: ball of radius 10 about the origin, the cube
    # [0, 0.1]^3 of 2000 kg/m^3, experiment-1 stations 100 m above the cube
    pr = W.paper_ball(dt_paper=0.1, paths_per_station=2)
    assert pr.domain == W.DOMAIN_BALL and np.allclose(pr.box_hi - pr.box_lo, 20.0)
    assert pr.stations.shape == (31, 3) and np.allclose(pr.stations[:, 2], 0.2)
    assert pr.dt == pytest.approx(0.2)
    # G rho is the same in any length unit: 6.674e-11 * 2000 s^-2
    assert pr.G * pr.prisms[0, 6] == pytest.approx(6.674e-11 * 2000.0, rel=1e-12)
