"""GPU: the library's documented limits, at their edges -- the last path
indices of the 32-bit counter word, the largest batch, the largest analytic
source and boundary-data tables, and a walk count that leaves a one-walk
tail in the reduction's last 8192-walk chunk -- each against the CPU oracle
(walk by walk) or against the same problems solved alone (bit for bit)."""
import numpy as np
import pytest

import oracle
from paper_1709_07469_amd import workloads as W
from gpu_helpers import compare_walks, gpu_solve, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _parity(pr, kind=0):
    stats, gv, gs = gpu_solve(pr, kind)
    ost, ou, osteps = oracle.solve(pr, kind)
    if kind == 1:
        gv = (gv[..., 0] - gv[..., 1]) / (2.0 * (pr.h if pr.h > 0 else np.sqrt(pr.dt)))
        gs = ((gs[..., 0] & 0x7FFFFFFF) + (gs[..., 1] & 0x7FFFFFFF)).astype(np.uint32)
    scale = np.nanmean(np.abs(ou), axis=1)[:, None]
    r = compare_walks(gv, gs, ou, osteps, scale)
    say("  walks", r)
    assert r["step_mismatch"] == 0 and r["value_mismatch"] == 0
    for s in range(pr.n_stations):
        assert abs(stats["mean"][s] - ost[s]["mean"]) <= 1e-12 * max(abs(ost[s]["mean"]), scale[s, 0])
        assert stats["n"][s] == ost[s]["n"]
    return stats, ost


def test_last_path_indices_of_the_counter_word():
    N = 700
    _parity(W.cfg1(N).replace(path_offset=(1 << 32) - N, problem_id=0xFFFFFFFF, seed=(1 << 64) - 1))


def test_one_walk_tail_in_the_last_reduction_chunk():
    pr = W.cfg1(8193).replace(stations=W.cfg1().stations[::3])
    stats, ost = _parity(pr)
    assert np.all(stats["n"] == 8193)


def test_largest_analytic_source_and_boundary_tables():
    rng = np.random.Generator(np.random.PCG64(16))
    lo = rng.uniform(-0.9, 0.3, size=(16, 3))
    prisms = np.concatenate([lo, lo + rng.uniform(0.05, 0.5, size=(16, 3)), rng.uniform(0.5, 2.0, (16, 1))], axis=1)
    spheres = np.concatenate([rng.uniform(-0.7, 0.7, (16, 3)), rng.uniform(0.05, 0.2, (16, 1)),
                              rng.uniform(0.5, 2.0, (16, 1))], axis=1)
    bc = prisms.copy()                      # 16 rows of prism boundary data
    st = np.array([[0.1, 0.2, 0.8], [-0.3, 0.4, 0.75], [0.5, -0.5, 0.85]])
    pr = W.Problem(box_lo=-np.ones(3), box_hi=np.ones(3), stations=st, dt=2e-3, paths_per_station=1500, G=1.0,
                   prisms=prisms, spheres=spheres, bc_kind=W.BC_PRISMS, bc_data=bc.ravel().copy(),
                   name="16-prisms-16-balls")
    for kind in (0, 1):
        _parity(pr, kind)


def test_largest_batch_equals_standalone():
    from paper_1709_07469_amd import fkgrav as F
    base = W.cfg1(64)
    rng = np.random.Generator(np.random.PCG64(256))
    probs, kinds = [], []
    for m in range(F.FK_MAX_BATCH):
        ns = int(rng.integers(1, 9))
        probs.append(base.replace(stations=base.stations[:ns], paths_per_station=int(rng.integers(2, 200)),
                                  problem_id=m, seed=int(rng.integers(0, 1 << 62))))
        kinds.append(int(rng.integers(0, 2)))
    res, _, _, _ = F.solve_batch(probs, kinds)
    say("  batch of", len(probs), "problems,", sum(p.n_stations for p in probs), "stations")
    for m in range(0, F.FK_MAX_BATCH, 5):
        alone, _, _ = F.solve(probs[m], kinds[m])
        assert res[m].tobytes() == alone.tobytes(), m
    with pytest.raises(F.FkError):
        F.solve_batch(probs + [probs[0]], kinds + [0])
