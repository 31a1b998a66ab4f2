"""GPU: the entry point that allocates nothing (fk_solve_static), called
through the C interface, against the workspace solves fk_solve_potential and
fk_solve_gz: equal results bit for bit on two calls in a row, the second with
a smaller input, so the second call runs on the scratch the first one left
behind.  A solve too large for the scratch is refused on the host before
anything is launched."""
import ctypes as C

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


def _static(pr, kind):
    import torch

    from paper_1709_07469_amd import fkgrav as F
    P = F.Prepared(pr)
    out = F.alloc_stats(pr.n_stations)
    F.fk_solve_static(kind, P.stations, P.box, P.source, P.bc, P.params, out)
    torch.cuda.synchronize()
    return F.stats_to_numpy(out)[: pr.n_stations]


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("precision", [W.PREC_F64, W.PREC_MIXED_F64ACC])
def test_static_equals_workspace_solve_twice(kind, precision):
    from paper_1709_07469_amd import fkgrav as F
    # first call: 64 stations x 100000 walks of the SI-prism workload (g_z:
    # 12.8e6 walks, several slices of the 64 MiB scratch); second call: a
    # smaller input (8 stations x 20000 walks of the sphere workload)
    big = W.cfg2(100_000, precision=precision)
    small = W.cfg1(20_000, precision=precision)
    for pr in (big, small):
        say("static solve", pr.name, "kind", kind, "precision", precision)
        ref, _, _ = F.solve(pr, kind)
        got = _static(pr, kind)
        assert got.tobytes() == ref.tobytes(), (pr.name, got["mean"], ref["mean"])


def test_static_with_a_slice_bound_and_a_grid():
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg3(30_000, n=32).replace(stations=W.cfg3(n=32).stations[:40])
    ref, _, _ = F.solve(pr, 0)
    got = _static(pr.replace(slice_walks=3 * 8192 + 5), 0)
    assert got.tobytes() == ref.tobytes()
    # the same grid given by levels (a byte per voxel and its densities)
    got = _static(pr.replace(slice_walks=3 * 8192 + 5, grid_levels=True), 0)
    assert got.tobytes() == ref.tobytes()


def test_static_refuses_what_does_not_fit():
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg1(100).replace(paths_per_station=1 << 31)     # 262144 pairs per station, 8 stations
    P = F.Prepared(pr)
    out = F.alloc_stats(pr.n_stations)
    with pytest.raises(F.FkError) as e:
        F.fk_solve_static(0, P.stations, P.box, P.source, P.bc, P.params, out)
    assert e.value.status == F.FK_EUNSUPPORTED
    assert "scratch" in str(e.value)
    with pytest.raises(F.FkError) as e:
        F.fk_solve_static(2, P.stations, P.box, P.source, P.bc, P.params, out)
    assert e.value.status == F.FK_EINVAL
