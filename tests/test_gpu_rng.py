"""GPU: the walk kernels' random stream against the CPU oracle's.  Philox
words must be identical; FP64-stream normals (the library's own log, sqrt
and sincos) must agree with the oracle's glibc-based ones to a few ulp; the
mixed-precision stream's normals (hardware FP32 log2, sqrt, sin, cos) to
FP32 accuracy."""
import numpy as np
import pytest

import oracle
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _counters(n=4096, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    c[:64, 0] = np.arange(64)            # consecutive blocks of one walk
    c[:64, 1:] = [12345, 7, 3]
    c[64] = [0, 0, 0, 0]
    c[65] = [0xFFFFFFFF] * 4
    return c


@pytest.mark.parametrize("seed", [0, (5 << 32) | 9, 0xFFFFFFFFFFFFFFFF])
def test_philox_words_and_normals_match_oracle(seed):
    import torch
    from paper_1709_07469_amd import fkgrav as F
    c = _counters(seed=seed & 0xFFFF)
    n = len(c)
    ct = torch.from_numpy(c.view(np.int32)).cuda()
    words = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    z64 = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    z32 = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    F.fk_stream_blocks(ct, seed, words, z64, z32)
    torch.cuda.synchronize()
    w = words.cpu().numpy().view(np.uint32)
    g64 = z64.cpu().numpy()
    g32 = z32.cpu().numpy().astype(np.float64)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    worst64 = worst32 = 0.0
    for i in range(n):
        ref = oracle.philox4x32_10(c[i], key)
        assert np.array_equal(w[i], ref), (i, w[i], ref)
        k, p, s, m = (int(v) for v in c[i])
        for j in range(2):
            o = oracle.normal(oracle.STREAM_F64, seed, m, s, p, 2 * k + j)
            worst64 = max(worst64, abs(g64[i, j] - o) / max(1.0, abs(o)))
        for j in range(4):
            o = oracle.normal(oracle.STREAM_F32, seed, m, s, p, 4 * k + j)
            worst32 = max(worst32, abs(g32[i, j] - o) / max(1.0, abs(o)))
    say("worst FP64 normal error", worst64, "worst FP32 normal error", worst32)
    # the oracle evaluates cos(2 pi U) with 2 pi U rounded to FP64 (up to
    # 4.4e-16 absolute in the angle), so with R up to 8.6 its own error
    # reaches ~4e-15 of max(1, |z|)
    assert worst64 < 1e-14
    assert worst32 < 2e-6
