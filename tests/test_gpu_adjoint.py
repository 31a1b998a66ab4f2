"""GPU: the adjoint (d mean / d rho through fk_potential_adjoint /
fk_gz_adjoint and the torch.autograd.Function).

For fixed random streams a station mean is an affine function of the voxel
densities, so the adjoint is checked against
  * the oracle's occupation counts (integer, walk by walk: must be equal),
  * central finite differences with the same seed (equal to rounding),
  * the linearity identity sum_s g_s mean_s = sum_v rho_v grad_v when the
    data is zero and the grid is the only source.
Both LDS gathering schemes of the adjoint are run (launch setting
adjoint_table: 0 = dense per-station tables where the grid has at most 32768
voxels, 1 = the hashed block table), each at the limits where weights bypass
the table."""
import math

import numpy as np
import pytest

import oracle
from paper_1709_07469_amd import workloads as W
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _counts_from_workspace(aws, S, nvox):
    import torch
    return aws[: 8 * S * nvox].view(torch.int64).cpu().numpy().reshape(S, nvox)


class _table:
    """Runs the block with the adjoint's LDS table scheme set, then restores
    the launch setting."""

    def __init__(self, precision, table):
        self.precision, self.table = precision, table

    def __enter__(self):
        from paper_1709_07469_amd import fkgrav as F
        self.keep = F.fk_get_launch(self.precision)
        k = self.keep
        F.fk_set_launch_dict(self.precision, dict(k, adjoint_table=self.table))

    def __exit__(self, *exc):
        from paper_1709_07469_amd import fkgrav as F
        k = self.keep
        F.fk_set_launch_dict(self.precision, k)


@pytest.mark.parametrize("table", [0, 1])
@pytest.mark.parametrize("kind", [0, 1])
def test_adjoint_counts_equal_oracle_occupation(kind, table):
    pr = W.cfg5(300)
    with _table(pr.precision, table):
        _check_counts(pr.replace(stations=pr.stations[::6]), kind)


def _coarse_grid(n, dt, paths, n_stations):
    """Zero data, an n^3 grid of random densities over [-1, 1]^3."""
    rng = np.random.Generator(np.random.PCG64(n))
    st = np.stack([rng.uniform(-0.6, 0.6, n_stations), rng.uniform(-0.6, 0.6, n_stations),
                   rng.uniform(-0.6, 0.6, n_stations)], axis=1)
    o = np.full(3, -1.0)
    return W.Problem(box_lo=o.copy(), box_hi=-o, stations=st, dt=dt, paths_per_station=paths, seed=3,
                     rho=rng.uniform(0.5, 2.0, size=(n, n, n)), grid_origin=o, grid_spacing=np.full(3, 2.0 / n),
                     name=f"grid{n}")


@pytest.mark.parametrize("table", [0, 1])
@pytest.mark.parametrize("case", ["long-runs", "wide-index"])
@pytest.mark.parametrize("kind", [0, 1])
def test_adjoint_counts_at_the_table_limits(kind, case, table):
    """The hashed LDS table holds 11-bit counts under 21-bit keys and passes
    the rest to the global counts: a 2^3 grid at dt = 1e-4 gives runs of
    hundreds of steps in one voxel (weights past the count range) and slots
    that overflow; a 64^3 grid with 9 stations puts station x voxel indices
    past 2^21 (too many voxels for the dense tables, so hashed either way)."""
    pr = _coarse_grid(2, 1e-4, 60, 2) if case == "long-runs" else _coarse_grid(64, 1e-3, 24, 9)
    with _table(pr.precision, table):
        _check_counts(pr, kind)


@pytest.mark.parametrize("case", ["direct", "exchange"])
def test_dense_table_limits(case):
    """A one-voxel grid covering the whole box: every step of every walk
    lands in voxel 0, so its count is the sum over walks of (2 steps - 1)
    (the start point once, each later point inside twice, the exit point
    outside).  dt = 2e-7 gives walks of ~2e6 steps whose run-length weights
    exceed 2^19 and go straight to the global counts; dt = 4e-6 with 1.3e6
    walks of ~1e5 steps drives each block's dense count past 2^30, where it
    is exchanged out of the table."""
    import torch
    from paper_1709_07469_amd import fkgrav as F
    dt, N = (2e-7, 512) if case == "direct" else (4e-6, 1_300_000)
    o = np.full(3, -1.0)
    pr = W.Problem(box_lo=o.copy(), box_hi=-o, stations=np.zeros((1, 3)), dt=dt, paths_per_station=N, seed=9,
                   rho=np.ones((1, 1, 1), dtype=np.float32), grid_origin=o, grid_spacing=np.full(3, 2.0),
                   name="one-voxel")
    say("dense table limit case", case, "dt", dt, "walks", N)
    stats, ws, P = F.solve(pr, 0)
    _, steps = F.path_samples(ws, 0, 1, P.params)
    assert not np.any(steps & np.uint32(0x80000000))
    expect = int((2 * steps.astype(np.int64) - 1).sum())
    out = F.stats_to_device(stats)
    aws = F.alloc_workspace(F.fk_adjoint_workspace_bytes(1, P.source))
    grad = torch.empty(1, dtype=torch.float64, device="cuda")
    F.fk_potential_adjoint(P.stations, P.box, P.source, P.bc, P.params, out, ws,
                           torch.ones(1, dtype=torch.float64, device="cuda"), grad, aws)
    torch.cuda.synchronize()
    counts = _counts_from_workspace(aws, 1, 1)
    say("  count", int(counts[0, 0]), "expected", expect, "longest walk", int(steps.max()))
    assert int(counts[0, 0]) == expect
    if case == "direct":
        assert 2 * int(steps.max()) - 1 >= (1 << 19)
    else:
        assert expect >= 256 * (1 << 30)     # past 2^30 per block, on average, of the 256 that share the station


def _check_counts(pr, kind):
    import torch
    from paper_1709_07469_amd import fkgrav as F
    S = pr.n_stations
    nvox = pr.rho.size
    rng = np.random.Generator(np.random.PCG64(1))
    g = rng.normal(size=S)
    P = F.Prepared(pr)
    stats, ws, P = F.solve(pr, kind, prepared=P)
    out = F.stats_to_device(stats)
    aws = F.alloc_workspace(F.fk_adjoint_workspace_bytes(S, P.source))
    grad = torch.empty(nvox, dtype=torch.float64, device="cuda")
    fn = F.fk_gz_adjoint if kind == 1 else F.fk_potential_adjoint
    fn(P.stations, P.box, P.source, P.bc, P.params, out, ws, torch.as_tensor(g, device="cuda"), grad, aws)
    torch.cuda.synchronize()
    counts = _counts_from_workspace(aws, S, nvox)
    cp, cm = oracle.occupation(pr, kind, 0, pr.paths_per_station)
    ref = cp.astype(np.int64) - (cm.astype(np.int64) if cm is not None else 0)
    say("kind", kind, "visits", int(np.abs(ref).sum()), "mismatching voxels", int((counts != ref).sum()))
    assert np.array_equal(counts, ref)
    w = 2 * math.pi * pr.G * (0.5 * pr.dt)
    h = math.sqrt(pr.dt)
    scale = -w / (2 * h if kind == 1 else 1.0)
    expect = sum(g[s] * scale / stats["n"][s] * ref[s].astype(np.float64) for s in range(S))
    got = grad.cpu().numpy()
    assert np.allclose(got, expect, rtol=1e-12, atol=1e-300)


def test_adjoint_matches_central_differences_f64():
    import torch
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg5(2000)
    pr = pr.replace(stations=pr.stations[::4])
    S = pr.n_stations
    rng = np.random.Generator(np.random.PCG64(2))
    g = rng.normal(size=S)
    stats, grad = F.adjoint(pr, 1, g)
    grad = grad.ravel()
    voxels = W.cfg5_fd_voxels(pr.rho.size, 16)
    hot = np.argsort(-np.abs(grad))[:16]               # plus the most sensitive voxels
    eps = 0.01 * float(pr.rho.max())
    worst = 0.0
    for v in np.concatenate([voxels, hot]):
        r_p = pr.rho.copy().ravel()
        r_m = pr.rho.copy().ravel()
        r_p[v] += eps
        r_m[v] -= eps
        sp, _, _ = F.solve(pr.replace(rho=r_p.reshape(pr.rho.shape)), 1)
        sm, _, _ = F.solve(pr.replace(rho=r_m.reshape(pr.rho.shape)), 1)
        # the grid is FP32: the step actually taken is the rounded difference
        step = float(np.float32(r_p[v])) - float(np.float32(r_m[v]))
        fd = float(np.dot(g, sp["mean"] - sm["mean"])) / step
        scale = float(np.abs(g) @ np.abs(stats["mean"])) / eps * 1e-12
        err = abs(fd - grad[v])
        worst = max(worst, err / (abs(grad[v]) + scale))
        assert err <= 1e-7 * abs(grad[v]) + scale, (v, fd, grad[v])
    say("worst relative FD gap", worst)


@pytest.mark.parametrize("precision", [W.PREC_F64, W.PREC_MIXED_F64ACC])
def test_linearity_identity(precision):
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg5(3000, precision=precision)
    S = pr.n_stations
    rng = np.random.Generator(np.random.PCG64(3))
    g = rng.normal(size=S)
    for kind in (0, 1):
        stats, grad = F.adjoint(pr, kind, g)
        lhs = float(np.dot(g, stats["mean"]))
        rhs = float(np.dot(pr.rho.ravel().astype(np.float64), grad.ravel()))
        say("precision", precision, "kind", kind, "sum g mean", lhs, "sum rho grad", rhs)
        assert rhs == pytest.approx(lhs, rel=1e-9, abs=1e-12 * float(np.abs(g) @ np.abs(stats["mean"])))


def test_autograd_function_matches_adjoint():
    import torch
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg5(1500)
    pr = pr.replace(stations=pr.stations[:8])
    P = F.Prepared(pr)
    rho = torch.tensor(pr.rho, device="cuda", requires_grad=True)
    fn = F.gz_function()
    means = fn.apply(rho, P, 1)
    stats, _, _ = F.solve(pr, 1)
    assert np.array_equal(means.detach().cpu().numpy(), stats["mean"])
    g = torch.linspace(-1.0, 1.0, means.numel(), dtype=torch.float64, device="cuda")
    (grad,) = torch.autograd.grad(means, rho, grad_outputs=g)
    _, ref = F.adjoint(pr, 1, g.cpu().numpy())
    assert np.allclose(grad.cpu().numpy(), ref.astype(np.float32), rtol=1e-6, atol=0)


def test_cfg5_full_size_adjoint():
    """32 stations x 1e6 CRN pairs on the 32^3 grid: forward, adjoint, the
    linearity identity and central differences on all 64 voxels the cfg5
    recipe draws (128 perturbed full-size solves, 16 per batched launch in a
    bounded workspace)."""
    import time

    import torch
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg5()
    S = pr.n_stations
    rng = np.random.Generator(np.random.PCG64(5))
    g = rng.normal(size=S)
    t0 = time.perf_counter()
    stats, grad = F.adjoint(pr, 1, g)
    say("cfg5 forward + adjoint", round(time.perf_counter() - t0, 2), "s; steps", int(stats["sum_steps"].sum()))
    lhs = float(np.dot(g, stats["mean"]))
    rhs = float(np.dot(pr.rho.ravel().astype(np.float64), grad.ravel()))
    assert rhs == pytest.approx(lhs, rel=1e-9)
    eps = 0.01 * float(pr.rho.max())
    flat = grad.ravel()
    voxels = W.cfg5_fd_voxels(pr.rho.size, 64)
    assert len(voxels) == 64
    tol0 = 1e-12 * float(np.abs(g) @ np.abs(stats["mean"])) / eps
    worst = 0.0
    for k in range(0, 64, 8):
        group = voxels[k:k + 8]
        probs = []
        for v in group:
            for sign in (1.0, -1.0):
                r = pr.rho.copy().ravel()
                r[v] += sign * eps
                probs.append(pr.replace(rho=r.reshape(pr.rho.shape), slice_walks=100_000_000))
        res, ws, _, _ = F.solve_batch(probs, [1] * len(probs))
        del ws
        for j, v in enumerate(group):
            sp, sm = res[2 * j], res[2 * j + 1]
            step = float(np.float32(pr.rho.ravel()[v] + eps)) - float(np.float32(pr.rho.ravel()[v] - eps))
            fd = float(np.dot(g, sp["mean"] - sm["mean"])) / step
            err = abs(fd - flat[v])
            worst = max(worst, err / (abs(flat[v]) + tol0))
            assert err <= 1e-7 * abs(flat[v]) + tol0, (v, fd, flat[v])
        say("  voxels", k, "..", k + 7, "checked")
    say("worst FD gap relative to (|grad| + rounding scale)", worst)
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", [0, 1])
def test_mixed_adjoint_counts_against_oracle_fp32_stream(kind):
    """The mixed-precision adjoint (FP32 stream and stepping) against the
    oracle's FP32-stream occupation (the same uniforms, FP64 stepping): FP32
    rounding moves a point across a voxel face, or a walk's exit by a step,
    now and then, so the counts agree closely but not exactly; the gradient
    they give agrees to well below the statistical error of the means."""
    import torch
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg5(2000, precision=W.PREC_MIXED_F64ACC)
    pr = pr.replace(stations=pr.stations[::4])
    S = pr.n_stations
    nvox = pr.rho.size
    stats, ws, P = F.solve(pr, kind)
    out = F.stats_to_device(stats)
    aws = F.alloc_workspace(F.fk_adjoint_workspace_bytes(S, P.source))
    grad = torch.empty(nvox, dtype=torch.float64, device="cuda")
    fn = F.fk_gz_adjoint if kind == 1 else F.fk_potential_adjoint
    fn(P.stations, P.box, P.source, P.bc, P.params, out, ws, torch.ones(S, dtype=torch.float64, device="cuda"),
       grad, aws)
    torch.cuda.synchronize()
    counts = _counts_from_workspace(aws, S, nvox)
    cp, cm = oracle.occupation(pr, kind, 0, pr.paths_per_station, stream=oracle.STREAM_F32)
    ref = cp.astype(np.int64) - (cm.astype(np.int64) if cm is not None else 0)
    moved = int(np.abs(counts - ref).sum())
    total = int(np.abs(ref).sum())
    say("mixed adjoint kind", kind, "weights", total, "moved", moved, "fraction", moved / total)
    assert moved <= 2e-3 * total
    # per station: the count-weighted sum equals within the same fraction
    for s in range(S):
        a, b = counts[s].astype(np.float64), ref[s].astype(np.float64)
        assert abs(a.sum() - b.sum()) <= 2e-3 * np.abs(b).sum() + 4
