"""Pins for the oracle's Brownian-bridge exit test (the paper's remark on
estimating the exit time within a step, after Gobet 2000):

* its uniforms are the documented Philox blocks (checked against the raw
  words);
* on a slab, the probability of leaving through the top is x0 / L for
  Brownian motion; stopping only when a step lands outside overestimates it
  by the overshoot (an O(sqrt(dt)) error of many standard errors), while
  the bridge test brings the estimate within noise;
* in the ball with zero data (the paper's model), the exact Kelvin-image
  solution is recovered at a time step where the overshoot rule misses it.
"""
import numpy as np
import pytest

import oracle
from paper_1709_07469_amd import workloads as W


def test_bridge_uniform_layout():
    seed = (3 << 32) | 17
    for stream, q in ((oracle.STREAM_F64, 2), (oracle.STREAM_F32, 4)):
        for n in (0, 1, 5, 1234567):
            w = oracle.philox4x32_10([0x80000000 + n // q, 11, 2, 1], [17, 3]).astype(np.uint64)
            j = n % q
            if stream == oracle.STREAM_F64:
                ref = ((int(w[2 * j + 1]) << 21 | int(w[2 * j]) >> 11) + 1) * 2.0 ** -53
            else:
                ref = ((int(w[j]) >> 8) + 1) * 2.0 ** -24
            assert oracle.bridge_uniform(stream, seed, 1, 2, 11, n) == ref


def _slab(rule, dt, N=100000):
    # z in [0, 1], x and y bounds far away; data 1 on the top face, 0 on the bottom
    fn = np.array([[2, 2]] * 6, dtype=np.int32)
    vals = np.concatenate([np.full(16, 0.5), np.zeros(4), np.ones(4)])
    st = np.array([[0.0, 0.0, 0.3], [0.0, 0.0, 0.7], [0.0, 0.0, 0.05]])
    pr = W.Problem(box_lo=np.array([-1e3, -1e3, 0.0]), box_hi=np.array([1e3, 1e3, 1.0]), stations=st, dt=dt,
                   paths_per_station=N, bc_kind=W.BC_FACE_GRID, bc_data=vals, face_n=fn, exit_rule=rule)
    stats, _, _ = oracle.solve(pr, 0)
    return [(s["mean"] - x[2]) / s["se"] for s, x in zip(stats, st)]


def test_slab_harmonic_measure():
    z_int = _slab(W.EXIT_INTERSECT, 1e-2)
    z_br = _slab(W.EXIT_BRIDGE, 1e-2)
    assert min(abs(z) for z in z_int) > 8.0          # the step-end test misses exits
    assert max(abs(z) for z in z_br) < 4.0


def test_ball_zero_data_recovers_green_solution():
    C0 = np.array([0.3, -0.2, 0.1])
    R = 1.0
    y0, a = C0 + np.array([0.15, 0.1, -0.35]), 0.2
    M = 4.0 / 3.0 * np.pi * a ** 3
    d = y0 - C0
    ys = C0 + R * R * d / np.dot(d, d)
    mi = -M * R / np.linalg.norm(d)
    st = np.array([C0 + [0.0, 0.0, 0.5], C0 + [0.0, 0.0, 0.9]])
    exact = [oracle.sphere_potential(y0, a, 1.0, 1.0, x) - mi / np.linalg.norm(x - ys) for x in st]
    zs = {}
    for rule in (W.EXIT_OVERSHOOT, W.EXIT_BRIDGE):
        pr = W.Problem(box_lo=C0 - R, box_hi=C0 + R, stations=st, dt=4e-3, paths_per_station=200000, G=1.0,
                       spheres=np.array([[*y0, a, 1.0]]), bc_kind=W.BC_ZERO, domain=W.DOMAIN_BALL, exit_rule=rule)
        stats, _, _ = oracle.solve(pr, 0)
        zs[rule] = [(s["mean"] - e) / s["se"] for s, e in zip(stats, exact)]
    assert zs[W.EXIT_OVERSHOOT][1] < -5.0
    assert max(abs(z) for z in zs[W.EXIT_BRIDGE]) < 4.0


def test_bridge_only_stops_walks_earlier():
    # the bridge test adds stops between step ends; it never delays an exit
    pr = W.cfg1(300)
    items = np.array([[0, i] for i in range(300)])
    _, so = oracle.run_paths(pr, 0, items, exit_rule=W.EXIT_INTERSECT)
    _, sb = oracle.run_paths(pr, 0, items, exit_rule=W.EXIT_BRIDGE)
    assert np.all(sb <= so)
    assert np.mean(sb < so) > 0.05
