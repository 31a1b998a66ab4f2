"""Moving-average smoothing of station profiles (paper section 4.1), host
side: the library against the oracle, and the oracle against what the
definition fixes -- a hand-worked example with shrinking end windows, exact
reproduction of linear profiles, and the 1/span variance reduction of
independent noise."""
import numpy as np
import pytest

import oracle
from paper_1709_07469_amd import fkgrav as F


def test_oracle_hand_example_with_shrinking_ends():
    v = np.array([1.0, 2.0, 4.0, 8.0, 16.0, 32.0, 64.0])
    out, _ = oracle.moving_average(v, span=5)
    ref = [1.0, 7.0 / 3.0, 31.0 / 5.0, 62.0 / 5.0, 124.0 / 5.0, 112.0 / 3.0, 64.0]
    assert np.allclose(out, ref, rtol=1e-15)
    out1, _ = oracle.moving_average(v, span=1)
    assert np.array_equal(out1, v)


def test_oracle_reproduces_linear_profiles_and_reduces_variance():
    x = np.linspace(-3.0, 5.0, 41)
    lin = 0.7 - 2.5 * x
    out, _ = oracle.moving_average(lin, span=7)
    assert np.allclose(out, lin, rtol=0, atol=1e-13)
    rng = np.random.Generator(np.random.PCG64(0))
    noise = rng.normal(size=(4000, 41))
    sm = np.array([oracle.moving_average(r, span=5)[0] for r in noise])
    var = sm[:, 10:31].var(axis=0).mean()
    assert var == pytest.approx(1.0 / 5.0, rel=0.05)
    _, se = oracle.moving_average(np.zeros(41), np.full(41, 1.0), span=5)
    assert se[20] == pytest.approx(1.0 / np.sqrt(5.0), rel=1e-15) and se[0] == 1.0


def test_library_matches_oracle():
    rng = np.random.Generator(np.random.PCG64(1))
    for n in (1, 2, 5, 31):
        v = rng.normal(size=n)
        e = rng.uniform(0.1, 1.0, size=n)
        for span in (1, 3, 5, 9):
            a, ae = F.fk_moving_average(v, e, span)
            b, be = oracle.moving_average(v, e, span)
            assert np.allclose(a, b, rtol=1e-15, atol=1e-15) and np.allclose(ae, be, rtol=1e-15)
    with pytest.raises(F.FkError):
        F.fk_moving_average(np.zeros(3), None, 4)
