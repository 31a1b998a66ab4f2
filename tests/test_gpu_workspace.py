"""GPU: the bounded workspace and the status word.

A solve with slice_walks > 0 runs its walks in slices of whole (station,
8192-path chunk) pairs and reduces each slice before the next; it keeps no
per-walk record, only every pair's partial statistics, and must give the
station results of the record-mode solve bit for bit (the same partials,
merged in the same order).  Budgets are chosen to exercise both ways of
cutting: whole stations per slice, and runs of chunks of one station, with
ragged last chunks and slices that cross problem boundaries in a batch.

The status word of a workspace collects anomaly bits on the device: capped
walks (reported as FK_ETRUNC by a strict solve) and non-finite samples (a NaN
voxel).  Truncation is forced from the host with max_steps = 1, so every
kernel ends normally.
"""
import numpy as np
import pytest

from paper_1709_07469_amd import workloads as W
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1709_07469_amd import fkgrav as F
    F.lib()


def _bits(a):
    return np.ascontiguousarray(a).tobytes()


@pytest.mark.parametrize("precision", [W.PREC_F64, W.PREC_MIXED_F64ACC])
@pytest.mark.parametrize("kind", [0, 1])
def test_slices_equal_record_mode_bitwise(precision, kind):
    from paper_1709_07469_amd import fkgrav as F
    # 8 stations x 20000 walks: 3 chunks per station, the last one ragged
    pr = W.cfg1(20000, precision=precision)
    ref, _, _ = F.solve(pr, kind)
    npair = 2 if kind else 1
    per_station = 20000 * npair
    budgets = [8192 * npair,                  # one chunk per slice
               3 * 8192 * npair + 100,        # a station's 3 chunks (ragged budget)
               per_station,                   # one station per slice
               int(2.5 * per_station),        # two stations, then a remainder
               10 * per_station]              # everything in one slice
    for b in budgets:
        say("slice budget", b, "kind", kind, "precision", precision)
        got, ws, P = F.solve(pr.replace(slice_walks=b), kind)
        assert ws.numel() < F.fk_workspace_bytes(kind, pr.n_stations, F.make_params(pr))
        assert _bits(got) == _bits(ref), (b, got["mean"], ref["mean"])


def test_batch_slices_equal_record_mode_bitwise():
    from paper_1709_07469_amd import fkgrav as F
    models = W.cfg4(n_models=3, precision=W.PREC_MIXED_F64ACC, n=32)
    probs = [m.replace(paths_per_station=[17000, 3000, 9000][i], stations=m.stations[: [5, 11, 3][i]])
             for i, m in enumerate(models)]
    probs.append(W.cfg1(12000, precision=W.PREC_MIXED_F64ACC).replace(problem_id=40))
    kinds = [0, 1, 0, 1]
    ref, _, _, _ = F.solve_batch(probs, kinds)
    for b in (16384, 16384 * 3 + 7, 100000, 400000):
        say("batch slice budget", b)
        sl = [p.replace(slice_walks=b) for p in probs]
        got, ws, PB, _ = F.solve_batch(sl, kinds)
        for m in range(len(probs)):
            assert _bits(got[m]) == _bits(ref[m]), (b, m)


def test_full_32_model_batch_in_under_2_gb():
    """The whole 32-model voxel batch (1.2e9 walks; 53 GB of records in
    record mode) in a bounded workspace of under 2 GB, equal bit for bit to
    the record-mode solve."""
    import torch

    from paper_1709_07469_amd import fkgrav as F
    probs = W.cfg4()
    kinds = [0] * len(probs)
    slice_walks = 40_000_000
    sl = [p.replace(slice_walks=slice_walks) for p in probs]
    PBs = F.PreparedBatch(sl, kinds)
    nb = F.fk_batch_workspace_bytes(PBs.problems)
    say("bounded batch workspace bytes", nb)
    assert 0 < nb < 2 * 1024 ** 3
    got, ws, _, _ = F.solve_batch(sl, kinds, prepared=PBs)
    del ws
    torch.cuda.empty_cache()
    ref, ws, _, _ = F.solve_batch(probs, kinds)
    say("record-mode workspace bytes", ws.numel())
    del ws
    torch.cuda.empty_cache()
    for m in range(len(probs)):
        assert _bits(got[m]) == _bits(ref[m]), m


def test_strict_truncation_reported():
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg1(300)
    stats, ws, _ = F.solve(pr, 0)
    st, flags = F.fk_workspace_status(ws)
    assert st == F.FK_OK and flags == 0
    # every walk capped after one step: counted, excluded, flagged
    stats, ws, _ = F.solve(pr.replace(max_steps=1), 0)
    assert np.all(stats["n_trunc"] == 300) and np.all(stats["n"] == 0)
    st, flags = F.fk_workspace_status(ws)
    assert st == F.FK_OK and flags == F.FK_FLAG_TRUNCATED
    stats, ws, _ = F.solve(pr.replace(max_steps=1, strict=1), 1)
    st, flags = F.fk_workspace_status(ws)
    assert st == F.FK_ETRUNC and flags == F.FK_FLAG_TRUNCATED | F.FK_FLAG_STRICT
    # strict without truncation is fine; the same through the bounded workspace
    stats, ws, _ = F.solve(pr.replace(strict=1, slice_walks=8192), 0)
    st, flags = F.fk_workspace_status(ws)
    assert st == F.FK_OK and flags == F.FK_FLAG_STRICT
    # a batch: one strict problem with capped walks makes the batch report it
    res, ws, _, _ = F.solve_batch([pr, pr.replace(max_steps=1, strict=1, problem_id=3)], [0, 0])
    st, flags = F.fk_workspace_status(ws)
    assert st == F.FK_ETRUNC and flags & F.FK_FLAG_TRUNCATED
    assert np.all(res[0]["n_trunc"] == 0) and np.all(res[1]["n_trunc"] == 300)


@pytest.mark.parametrize("precision", [W.PREC_F64, W.PREC_MIXED_F64ACC])
def test_nan_voxel_flagged(precision):
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg3(500, precision=precision, n=32).replace(stations=W.cfg3(n=32).stations[:4])
    stats, ws, _ = F.solve(pr, 0)
    st, flags = F.fk_workspace_status(ws)
    assert st == F.FK_OK and flags == 0 and np.all(np.isfinite(stats["mean"]))
    rho = np.array(pr.rho, copy=True)
    # the voxel under the first station (x = y = -0.75, z = 0.5), where every walk starts
    i = int((-0.75 + 1.0) * 16)
    k = int((0.5 + 1.0) * 16)
    rho[k, i, i] = np.nan
    bad = pr.replace(rho=rho)
    stats, ws, _ = F.solve(bad, 0)
    st, flags = F.fk_workspace_status(ws)
    say("nan voxel", st, flags, stats["mean"])
    assert st == F.FK_ENONFINITE and flags & F.FK_FLAG_NONFINITE
    assert np.isnan(stats["mean"][0])
