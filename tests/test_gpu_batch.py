"""GPU: the batched persistent launch.  Every problem of a batch must give the
same bits as the same problem solved alone (same streams, same arithmetic,
results stored by walk index), FP64 batches must match the CPU oracle walk by
walk, and a HIP-graph capture of a batch must replay to the eager result."""
import numpy as np
import pytest

import oracle
from paper_1709_07469_amd import workloads as W
from gpu_helpers import compare_walks, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _small_mix(precision):
    models = W.cfg4(n_models=3, precision=precision, n=32)
    probs = [m.replace(paths_per_station=[700, 300, 1100][i], stations=m.stations[: [9, 20, 5][i]])
             for i, m in enumerate(models)]
    probs.append(W.cfg1(900, precision=precision).replace(problem_id=40))
    c2 = W.cfg2(40, precision=precision)
    probs.append(c2.replace(stations=c2.stations[::9], problem_id=41))
    kinds = [0, 1, 0, 1, 0]
    return probs, kinds


@pytest.mark.parametrize("precision", [W.PREC_F64, W.PREC_MIXED_F64ACC, W.PREC_MIXED_KAHAN])
@pytest.mark.parametrize("seeds", ["one", "per_problem"])
def test_batch_equals_standalone_bitwise(precision, seeds):
    """One seed for the whole batch (mixed batches then hold the generator key
    in scalar registers) and a seed per problem (each lane its own key)."""
    from paper_1709_07469_amd import fkgrav as F
    probs, kinds = _small_mix(precision)
    if seeds == "per_problem":
        probs = [p.replace(seed=(0x9E3779B97F4A7C15 * (m + 1)) % (1 << 64)) for m, p in enumerate(probs)]
    say("batch of", len(probs), "precision", precision, "seeds", seeds)
    res, ws, PB, _ = F.solve_batch(probs, kinds)
    for m, (p, k) in enumerate(zip(probs, kinds)):
        alone, ws1, P1 = F.solve(p, k)
        assert res[m].tobytes() == alone.tobytes(), (m, res[m], alone)
        bv, bs = F.batch_path_samples(ws, PB, m)
        av, as_ = F.path_samples(ws1, k, p.n_stations, P1.params)
        assert np.array_equal(bv.view(np.uint64), av.view(np.uint64)) and np.array_equal(bs, as_)


@pytest.mark.parametrize("precision", [W.PREC_F64, W.PREC_MIXED_F64ACC, W.PREC_MIXED_KAHAN])
def test_shared_source_batch_equals_standalone_bitwise(precision):
    """u and g_z of one SI-prism model in one batch: the two problems share
    the source and the seed, so every precision runs the kernel that holds
    the source and the generator key in scalar registers."""
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg2(60, precision=precision)
    pr = pr.replace(stations=pr.stations[::5])
    say("shared-source batch precision", precision)
    res, ws, PB, _ = F.solve_batch([pr, pr], [0, 1])
    for m, k in enumerate((0, 1)):
        alone, _, _ = F.solve(pr, k)
        assert res[m].tobytes() == alone.tobytes(), (precision, m)


@pytest.mark.parametrize("walks", [(2, 3), (2, 5, 4), (7, 2, 3, 9)])
def test_tiny_batches_of_separate_sources_equal_standalone(walks):
    """Batches of problems with their own sources split the queue into
    stripes; with fewer walks than stripes most stripes are empty or hold one
    walk, and every walk must still run exactly once."""
    from paper_1709_07469_amd import fkgrav as F
    c1 = W.cfg1(2)
    models = W.cfg4(n_models=len(walks), n=16)
    probs, kinds = [], []
    for j, n in enumerate(walks):
        base = c1 if j == 0 else models[j].replace(precision=W.PREC_F64)
        probs.append(base.replace(paths_per_station=max(n, 2), stations=base.stations[:1], problem_id=60 + j))
        kinds.append(j % 2)
    say("tiny batch walks", walks)
    res, ws, PB, _ = F.solve_batch(probs, kinds)
    for m, (p, k) in enumerate(zip(probs, kinds)):
        alone, _, _ = F.solve(p, k)
        assert res[m].tobytes() == alone.tobytes(), (m, res[m], alone)
        assert res[m]["n"][0] + res[m]["n_trunc"][0] == p.paths_per_station


def test_batch_f64_matches_oracle_walk_by_walk():
    from paper_1709_07469_amd import fkgrav as F
    probs, kinds = _small_mix(W.PREC_F64)
    res, ws, PB, _ = F.solve_batch(probs, [0] * len(probs))
    for m, p in enumerate(probs):
        gv, gs = F.batch_path_samples(ws, PB, m)
        ost, ou, osteps = oracle.solve(p, 0)
        scale = np.nanmean(np.abs(ou), axis=1)[:, None]
        r = compare_walks(gv, gs, ou, osteps, scale)
        say("  problem", m, p.name, r)
        assert r["step_mismatch"] == 0 and r["value_mismatch"] == 0
        for s in range(p.n_stations):
            assert abs(res[m]["mean"][s] - ost[s]["mean"]) <= 1e-12 * max(abs(ost[s]["mean"]), scale[s, 0])


def test_batch_graph_capture_replays_the_eager_result():
    import torch
    from paper_1709_07469_amd import fkgrav as F
    probs, kinds = _small_mix(W.PREC_MIXED_F64ACC)
    PB = F.PreparedBatch(probs, kinds)
    nb = F.fk_batch_workspace_bytes(PB.problems)
    ws = F.alloc_workspace(nb)
    out = F.alloc_stats(PB.n_out)
    F.fk_solve_batch(PB.problems, out, ws)
    torch.cuda.synchronize()
    eager = out.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        F.fk_solve_batch(PB.problems, out, ws)            # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        F.fk_solve_batch(PB.problems, out, ws)
    other = W.cfg1(500)
    for r in range(3):
        out.zero_()
        ws.fill_(0xAB)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {r}"
        F.solve(other, 0)                                  # eager work between replays
        torch.cuda.synchronize()


def test_cfg4_full_batch_against_closed_forms():
    """The batched workload: 32 random voxel models, 8-256 stations each,
    1e4-1e6 walks per station, mixed precision, in one launch."""
    import torch
    from paper_1709_07469_amd import fkgrav as F
    probs = W.cfg4()
    n_walks = sum(p.n_stations * p.paths_per_station for p in probs)
    say("cfg4:", len(probs), "models,", sum(p.n_stations for p in probs), "stations,", n_walks, "walks")
    res, ws, PB, _ = F.solve_batch(probs, [0] * len(probs))
    steps = sum(int(r["sum_steps"].sum()) for r in res)
    say("  steps", steps)
    worst = 0.0
    for m, p in enumerate(probs):
        assert np.all(res[m]["n_trunc"] == 0) and np.all(res[m]["n"] == p.paths_per_station)
        for s in np.linspace(0, p.n_stations - 1, 3).astype(int):
            ex = sum(oracle.prism_potential(q[:3], q[3:6], q[6], p.G, p.stations[s]) for q in p.model_prisms)
            z = (res[m]["mean"][s] - ex) / res[m]["se"][s]
            worst = max(worst, abs(z))
    say("  worst closed-form |z| over 96 stations", worst)
    assert worst < 5.0
    # sampled walks of a few problems against the oracle's FP32-stream mode
    for m in (0, 13, 31):
        gv, gs = F.batch_path_samples(ws, PB, m)
        p = probs[m]
        rng = np.random.Generator(np.random.PCG64(m))
        items = np.stack([rng.integers(0, p.n_stations, 24), rng.integers(0, p.paths_per_station, 24)], axis=1)
        ou, osteps = oracle.run_paths(p, 0, items, stream=oracle.STREAM_F32)
        g = gv[items[:, 0], items[:, 1]]
        gst = gs[items[:, 0], items[:, 1]]
        same = gst == osteps
        say("  model", m, "sampled walks with equal step counts", int(same.sum()), "of", len(same))
        assert same.mean() > 0.8
        assert np.all(np.abs(g[same] - ou[same]) <= 1e-3 * np.abs(ou[same]) + 1e-9)
    del ws
    torch.cuda.empty_cache()
