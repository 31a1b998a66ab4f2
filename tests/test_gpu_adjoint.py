"""GPU: the adjoint (d mean / d rho through fk_potential_adjoint /
fk_gz_adjoint and the torch.autograd.Function).

For fixed random streams a station mean is an affine function of the voxel
densities, so the adjoint is checked against
  * the oracle's occupation counts (integer, walk by walk: must be equal),
  * central finite differences with the same seed (equal to rounding),
  * the linearity identity sum_s g_s mean_s = sum_v rho_v grad_v when the
    data is zero and the grid is the only source."""
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


@pytest.mark.parametrize("kind", [0, 1])
def test_adjoint_counts_equal_oracle_occupation(kind):
    pr = W.cfg5(300)
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


@pytest.mark.parametrize("case", ["long-runs", "wide-index"])
@pytest.mark.parametrize("kind", [0, 1])
def test_adjoint_counts_at_the_table_limits(kind, case):
    """The LDS table holds 11-bit counts under 21-bit keys and passes the rest
    to the global counts: a 2^3 grid at dt = 1e-4 gives runs of hundreds of
    steps in one voxel (weights past the count range) and slots that overflow;
    a 64^3 grid with 9 stations puts station x voxel indices past 2^21."""
    pr = _coarse_grid(2, 1e-4, 60, 2) if case == "long-runs" else _coarse_grid(64, 1e-3, 24, 9)
    _check_counts(pr, kind)


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
    linearity identity and central differences on 8 of the cfg5 voxels."""
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
    for v in W.cfg5_fd_voxels(pr.rho.size, 64)[:8]:
        r_p = pr.rho.copy().ravel()
        r_m = pr.rho.copy().ravel()
        r_p[v] += eps
        r_m[v] -= eps
        sp, _, _ = F.solve(pr.replace(rho=r_p.reshape(pr.rho.shape)), 1)
        sm, _, _ = F.solve(pr.replace(rho=r_m.reshape(pr.rho.shape)), 1)
        step = float(np.float32(r_p[v])) - float(np.float32(r_m[v]))
        fd = float(np.dot(g, sp["mean"] - sm["mean"])) / step
        tol = 1e-7 * abs(flat[v]) + 1e-12 * float(np.abs(g) @ np.abs(stats["mean"])) / eps
        assert abs(fd - flat[v]) <= tol, (v, fd, flat[v])
    torch.cuda.empty_cache()
