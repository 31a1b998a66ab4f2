"""Merging per-station results of disjoint walk ranges (fk_merge_stats, the
statistics step of running a station's walks in several parts, e.g. on
several GPUs): checked on the host against the oracle's two-pass statistics
of the concatenated samples, the plain definition of eq. 11's mean and the
unbiased variance."""
import numpy as np
import pytest

import oracle
from paper_1709_07469_amd import fkgrav as F

CAP = np.uint32(0x80000000)


def _stat(u, steps):
    o = oracle.station_stats(u, steps)
    r = np.zeros(1, dtype=F.STAT_DTYPE)
    for k in ("mean", "var", "se", "n", "mean_steps", "max_steps", "n_trunc"):
        r[k] = o[k]
    r["sum_steps"] = int((steps & ~CAP).astype(np.int64).sum())
    return r


@pytest.mark.parametrize("split", [1, 2, 17, 5000, 9998])
def test_merge_equals_statistics_of_the_union(split):
    rng = np.random.Generator(np.random.PCG64(split))
    n = 10000
    u = rng.normal(3.0, 2.0, n) ** 3
    steps = rng.integers(1, 5000, n).astype(np.uint32)
    trunc = rng.random(n) < 0.01
    steps[trunc] |= CAP
    u[trunc] = np.nan
    a, b = _stat(u[:split], steps[:split]), _stat(u[split:], steps[split:])
    whole = _stat(u, steps)
    m = F.fk_merge_stats(a, b)
    for k in ("n", "n_trunc", "sum_steps", "max_steps"):
        assert m[k][0] == whole[k][0], k
    assert m["mean"][0] == pytest.approx(whole["mean"][0], rel=1e-13)
    assert m["var"][0] == pytest.approx(whole["var"][0], rel=1e-12)
    assert m["se"][0] == pytest.approx(whole["se"][0], rel=1e-12)
    assert m["mean_steps"][0] == pytest.approx(whole["mean_steps"][0], rel=1e-15)


def test_merge_with_empty_and_single_sample_parts():
    u = np.array([1.0, 2.0, 4.0])
    st = np.array([3, 4, 5], dtype=np.uint32)
    empty = np.zeros(1, dtype=F.STAT_DTYPE)
    empty["mean"] = empty["var"] = empty["se"] = np.nan
    whole = _stat(u, st)
    m = F.fk_merge_stats(empty, whole)
    assert m["mean"][0] == whole["mean"][0] and m["var"][0] == whole["var"][0] and m["n"][0] == 3
    one, rest = _stat(u[:1], st[:1]), _stat(u[1:], st[1:])
    m = F.fk_merge_stats(one, rest)
    assert m["mean"][0] == pytest.approx(7.0 / 3.0, rel=1e-15)
    assert m["var"][0] == pytest.approx(np.var(u, ddof=1), rel=1e-15)
    both_empty = F.fk_merge_stats(empty, empty)
    assert both_empty["n"][0] == 0 and np.isnan(both_empty["mean"][0])
