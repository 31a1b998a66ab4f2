"""GPU: a station's walks run in disjoint parts (path_offset ranges -- one
part per GPU when the path is sharded) and merged with fk_merge_stats give
the single run's statistics: the counter-based streams make the parts' walks
exactly the single run's walks, and the merge is the same Chan update the
reduction applies, in a different association."""
import numpy as np
import pytest

from paper_1709_07469_amd import workloads as W
from gpu_helpers import gpu_solve, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("precision", [W.PREC_F64, W.PREC_MIXED_F64ACC])
@pytest.mark.parametrize("kind", [0, 1])
def test_parts_merge_to_the_single_run(kind, precision):
    from paper_1709_07469_amd import fkgrav as F
    N = 40000
    whole, _, _ = gpu_solve(W.cfg1(N, precision=precision), kind)
    merged = None
    for lo, hi in ((0, 8192), (8192, 21000), (21000, N)):          # 8192-aligned and ragged cuts
        part, _, _ = gpu_solve(W.cfg1(hi - lo, precision=precision).replace(path_offset=lo), kind)
        merged = part if merged is None else F.fk_merge_stats(merged, part)
    for k in ("n", "n_trunc", "sum_steps", "max_steps"):
        assert np.array_equal(merged[k], whole[k]), k
    rel = np.abs(merged["mean"] - whole["mean"]) / np.abs(whole["mean"])
    say("  kind", kind, "precision", precision, "largest relative mean difference", rel.max())
    assert np.all(rel < 1e-13)
    assert np.allclose(merged["var"], whole["var"], rtol=1e-12)
    assert np.allclose(merged["se"], whole["se"], rtol=1e-12)
