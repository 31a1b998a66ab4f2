"""GPU: the mixed-precision voxel workload at full size -- a 128^3 FP32
density grid of 5 random prisms, 256 stations x 1e6 walks -- with FP32
stepping (FP64 and Kahan-compensated FP32 sums) and with FP64 stepping:
sampled walks against the oracle one by one, every station against the
prisms' closed-form potential, and the mixed kernels against the FP64 one at
equal walk counts (accuracy stated in standard errors)."""
import time

import numpy as np
import pytest

import oracle
from paper_1709_07469_amd import workloads as W
from gpu_helpers import CAP, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _exact(pr):
    return np.array([sum(oracle.prism_potential(q[:3], q[3:6], q[6], pr.G, x) for q in pr.model_prisms)
                     for x in pr.stations])


def _solve_and_sample(pr, items):
    import torch
    from paper_1709_07469_amd import fkgrav as F
    P = F.Prepared(pr)
    S, N = pr.n_stations, pr.paths_per_station
    ws = F.alloc_workspace(F.fk_workspace_bytes(0, S, P.params))
    out = F.alloc_stats(S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F.fk_solve_potential(P.stations, P.box, P.source, P.bc, P.params, out, ws)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    v_off, s_off, _ = F.fk_workspace_layout(0, S, P.params)
    T = S * N
    idx = torch.as_tensor(items[:, 0] * N + items[:, 1], device="cuda")
    vals = ws[v_off:v_off + 8 * T].view(torch.float64)[idx].cpu().numpy()
    steps = ws[s_off:s_off + 4 * T].view(torch.int32)[idx].cpu().numpy().view(np.uint32)
    st = F.stats_to_numpy(out)[:S]
    del ws
    torch.cuda.empty_cache()
    return st, vals, steps, secs


def test_cfg3_full_size_mixed_and_f64():
    base = W.cfg3()
    exact = _exact(base)
    rng = np.random.Generator(np.random.PCG64(33))
    items = np.stack([rng.integers(0, base.n_stations, 48), rng.integers(0, base.paths_per_station, 48)], axis=1)
    res = {}
    for prec, stream in ((W.PREC_F64, oracle.STREAM_F64), (W.PREC_MIXED_F64ACC, oracle.STREAM_F32),
                         (W.PREC_MIXED_KAHAN, oracle.STREAM_F32)):
        pr = base.replace(precision=prec)
        st, gv, gs, secs = _solve_and_sample(pr, items)
        steps = int(st["sum_steps"].sum())
        ou, osteps = oracle.run_paths(pr, 0, items, stream=stream)
        same = gs == osteps
        if prec == W.PREC_F64:
            assert np.all(same)
            assert np.all(np.abs(gv - ou) <= 1e-12 * np.abs(ou).mean())
        else:
            assert np.mean(same) >= 0.9
            assert np.all(np.abs(gv[same] - ou[same]) <= 1e-4 * np.abs(ou).mean())
        z = (st["mean"] - exact) / st["se"]
        say(f"  precision {prec}: {steps:.4g} steps in {secs:.3f} s ({steps / secs:.3e} steps/s), "
            f"closed-form |z| max {np.abs(z).max():.2f}, mean z {z.mean():+.3f}, "
            f"sampled step mismatches {int((~same).sum())}/{len(items)}")
        assert np.all(st["n"] == pr.paths_per_station) and np.all(st["n_trunc"] == 0)
        assert np.abs(z).max() < 5.0
        res[prec] = st
    for prec in (W.PREC_MIXED_F64ACC, W.PREC_MIXED_KAHAN):
        d = (res[prec]["mean"] - res[W.PREC_F64]["mean"]) / np.hypot(res[prec]["se"], res[W.PREC_F64]["se"])
        say(f"  precision {prec} vs FP64: |diff| max {np.abs(d).max():.2f} combined SE, mean {d.mean():+.3f}")
        assert np.abs(d).max() < 5.0 and abs(d.mean()) < 4.0 / np.sqrt(len(d))
