"""GPU: voxel grids given by levels (a byte index grid and 256 densities)
against the same grids given as FP32 densities.  The densities are the same,
so every walk's record and every station's statistics must come out bit for
bit the same: in FP64 and both mixed modes, for the potential and g_z, in
the box, ball and Brownian-bridge loops, in batches (one source, separate
sources) and in the adjoint.  One case goes walk by walk against the oracle
(which sees the FP32 grid)."""
import numpy as np
import pytest

import oracle
from paper_1709_07469_amd import workloads as W
from gpu_helpers import CAP, compare_walks, gpu_solve, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _small(prec=W.PREC_F64, n_walks=3000, model_seed=3, **kw):
    """The 128^3-grid workload's generator at 32^3 (6 distinct densities), 16
    of its stations, a few thousand walks each."""
    pr = W.cfg3(n=32, paths_per_station=n_walks, precision=prec, model_seed=model_seed)
    return pr.replace(stations=pr.stations[::16].copy(), **kw)


def _same(a, b):
    return np.asarray(a).tobytes() == np.asarray(b).tobytes()


@pytest.mark.parametrize("prec", [W.PREC_F64, W.PREC_MIXED_F64ACC, W.PREC_MIXED_KAHAN])
@pytest.mark.parametrize("kind", [0, 1])
def test_levels_equal_fp32_grid_bitwise(prec, kind):
    pr = _small(prec)
    say("case levels prec", prec, "kind", kind)
    st, vals, steps = gpu_solve(pr, kind)
    stl, valsl, stepsl = gpu_solve(pr.replace(grid_levels=True), kind)
    assert _same(steps, stepsl) and _same(vals, valsl)
    assert _same(st, stl)
    assert np.all(st["n"] > 0)


@pytest.mark.parametrize("prec", [W.PREC_F64, W.PREC_MIXED_F64ACC])
@pytest.mark.parametrize("loop", ["ball", "bridge"])
def test_levels_in_ball_and_bridge_loops(prec, loop):
    pr = _small(prec)
    if loop == "ball":
        inside = np.linalg.norm(pr.stations, axis=1) < 0.9
        pr = pr.replace(domain=W.DOMAIN_BALL, stations=pr.stations[inside].copy())
    else:
        pr = pr.replace(exit_rule=W.EXIT_BRIDGE)
    say("case levels", loop, "prec", prec, "stations", pr.n_stations)
    st, vals, steps = gpu_solve(pr, 0)
    stl, valsl, stepsl = gpu_solve(pr.replace(grid_levels=True), 0)
    assert _same(steps, stepsl) and _same(vals, valsl) and _same(st, stl)


def test_levels_batch_equals_fp32_standalone():
    from paper_1709_07469_amd import fkgrav as F
    for prec in (W.PREC_F64, W.PREC_MIXED_F64ACC):
        # one source for both problems (u and g_z of one model), then two
        # models with their own sources
        for probs, kinds in (([_small(prec)] * 2, [0, 1]),
                             ([_small(prec), _small(prec, model_seed=4, problem_id=1)], [0, 0])):
            say("case levels batch prec", prec, "kinds", kinds)
            res, _, _, _ = F.solve_batch([p.replace(grid_levels=True) for p in probs], kinds)
            for m, (p, k) in enumerate(zip(probs, kinds)):
                alone, _, _ = F.solve(p, k)
                assert _same(res[m], alone), (prec, kinds, m)


def test_levels_adjoint_equals_fp32():
    from paper_1709_07469_amd import fkgrav as F
    pr = _small(W.PREC_F64, n_walks=2000)
    g = np.linspace(1.0, 2.0, pr.n_stations)
    say("case levels adjoint")
    st, grad = F.adjoint(pr, 1, g)
    stl, gradl = F.adjoint(pr.replace(grid_levels=True), 1, g)
    assert _same(st, stl) and _same(grad, gradl)
    assert np.any(grad != 0.0)


def test_levels_walks_against_the_oracle():
    pr = _small(W.PREC_F64, n_walks=400).replace(grid_levels=True)
    say("case levels vs oracle")
    stats, gv, gs = gpu_solve(pr, 0)
    ost, ou, osteps = oracle.solve(pr, 0)
    ok = (osteps & CAP) == 0
    scale = np.nanmean(np.where(ok, np.abs(ou), np.nan), axis=1)
    r = compare_walks(gv, gs, ou, osteps, scale[:, None] * np.ones_like(ou))
    say("  walks", r)
    assert r["step_mismatch"] == 0 and r["value_mismatch"] == 0 and r["capped_nan"]
    for s in range(len(stats)):
        assert stats["n"][s] == ost[s]["n"]
        assert abs(stats["mean"][s] - ost[s]["mean"]) <= 1e-12 * max(abs(ost[s]["mean"]), scale[s])
