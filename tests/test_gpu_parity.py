"""GPU parity: the HIP walk kernels (through the C interface) against the CPU
oracle on the same Philox streams.

FP64 path: every walk's step count must equal the oracle's, every walk's
sample must agree to 1e-12 of the station's sample scale, and every station
mean to 1e-12 of max(|mean|, scale) -- the two sides differ only in the last
bits of log/sincos/atan (device library vs glibc).  A walk whose step count
differs (a point landing within rounding of a face) is counted and reported;
these tests expect none.

Mixed precision (FP32 stream and stepping): compared with the oracle's
FP32-stream mode (same uniforms, FP64 arithmetic); a small fraction of walks
take a different number of steps, and station means must agree to a small
fraction of a standard error.
"""
import math

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
    from paper_1709_07469_amd import fkgrav as F
    F.lib()


def _scale(o_vals, o_steps):
    ok = (o_steps & CAP) == 0
    v = np.where(ok, np.abs(o_vals), np.nan)
    return np.nanmean(v.reshape(v.shape[0], -1), axis=1)


def _check_f64_potential(prob, max_step_mismatch=0):
    say("case", prob.name, "S", prob.n_stations, "N", prob.paths_per_station)
    stats, gv, gs = gpu_solve(prob, 0)
    ost, ou, osteps = oracle.solve(prob, 0)
    scale = _scale(ou, osteps)
    r = compare_walks(gv, gs, ou, osteps, scale[:, None] * np.ones_like(ou))
    say("  walks", r)
    assert r["step_mismatch"] <= max_step_mismatch
    assert r["value_mismatch"] == 0 and r["capped_nan"]
    mism = (gs != osteps).reshape(len(stats), -1).any(axis=1)
    for s in range(len(stats)):
        assert stats["n"][s] == ost[s]["n"] and stats["n_trunc"][s] == ost[s]["n_trunc"]
        assert stats["sum_steps"][s] == int((osteps[s] & np.uint32(0x7FFFFFFF)).astype(np.int64).sum()) or mism[s]
        if mism[s] or ost[s]["n"] == 0:
            continue
        tol = 1e-12 * max(abs(ost[s]["mean"]), scale[s])
        assert abs(stats["mean"][s] - ost[s]["mean"]) <= tol, (s, stats["mean"][s], ost[s]["mean"])
        assert stats["var"][s] == pytest.approx(ost[s]["var"], rel=1e-9)
        assert stats["max_steps"][s] == ost[s]["max_steps"]
    return stats, ost


def test_f64_ball_cfg1_parity():
    _check_f64_potential(W.cfg1(3000))


def test_f64_si_prism_cfg2_parity():
    _check_f64_potential(W.cfg2(150))


def test_f64_voxel_grid_parity_pow2_spacing():
    pr = W.cfg3(400, precision=W.PREC_F64, n=32)
    _check_f64_potential(pr.replace(stations=pr.stations[::8]))


def test_f64_voxel_grid_parity_general_spacing():
    pr = W.cfg4(n_models=1, precision=W.PREC_F64, n=16)[0]
    _check_f64_potential(pr.replace(paths_per_station=300, stations=pr.stations[:12]))


def _subgrid(precision, n_walks):
    """A 12 x 9 x 7 grid of uneven spacing over the middle of the box
    [-1, 1]^3, with stations inside and outside it: walks cross each of its
    six faces, so the lookup meets indices below 0 and at or past n on every
    axis, and points on no voxel's corner."""
    rng = np.random.default_rng(21)
    n = np.array([12, 9, 7])
    o = np.array([-0.61, -0.47, -0.53])
    d = np.array([0.1, 0.11, 0.13])
    rho = rng.choice(np.array([0.0, 0.5, 0.9, 1.3, 1.7, 2.0], dtype=np.float32), size=n[::-1])   # 6 levels
    st = np.array([[0.0, 0.0, 0.0], [-0.55, 0.4, 0.3], [0.5, -0.45, -0.5], [0.8, 0.75, 0.0], [-0.85, -0.2, 0.7]])
    return W.Problem(box_lo=np.full(3, -1.0), box_hi=np.full(3, 1.0), stations=st, dt=1e-3,
                     paths_per_station=n_walks, seed=5, G=0.9, rho=rho, grid_origin=o, grid_spacing=d,
                     precision=precision, name="subgrid")


def test_f64_voxel_grid_inside_the_box_parity():
    _check_f64_potential(_subgrid(W.PREC_F64, 400))


@pytest.mark.parametrize("precision", [W.PREC_MIXED_F64ACC, W.PREC_MIXED_KAHAN])
def test_mixed_voxel_grid_inside_the_box_against_oracle_fp32_stream(precision):
    # the FP32 lookup (one fma per axis) may pick the neighbouring voxel
    # within an ulp of a face; everything else matches the oracle's walks
    pr = _subgrid(precision, 3000)
    say("case mixed subgrid", precision)
    stats, gv, gs = gpu_solve(pr, 0)
    ost, ou, osteps = oracle.solve(pr, 0, stream=oracle.STREAM_F32)
    frac = float(np.mean(gs != osteps))
    say("  step mismatch fraction", frac)
    assert frac < 0.02
    same = gs == osteps
    rel = np.abs(gv - ou)[same] / np.maximum(np.abs(ou)[same], 1e-300)
    say("  median / 99.9% rel diff of matching walks", np.median(rel), np.quantile(rel, 0.999))
    assert np.quantile(rel, 0.999) < 1e-4
    for s in range(pr.n_stations):
        assert abs(stats["mean"][s] - ost[s]["mean"]) < 0.5 * ost[s]["se"]
    lv, _, _ = gpu_solve(pr.replace(grid_levels=True), 0)
    assert np.asarray(lv).tobytes() == np.asarray(stats).tobytes()


_HARM = np.array([0.4, 1.0, -0.5, 0.25, 0.2, 0.0, 0.3, -0.3, -0.1, 0.1])
_BOX = dict(box_lo=np.array([-1.0, -1.0, -1.0]), box_hi=np.array([1.0, 1.0, 1.0]))
_ST4 = np.array([[0.0, 0.0, 0.0], [0.5, -0.3, 0.2], [-0.7, 0.6, -0.4], [0.1, 0.85, 0.7]])


def test_f64_stations_on_grid_planes():
    # Stations placed on voxel planes of a grid whose spacings are not powers
    # of two: every walk's start density needs the floor of a quotient that
    # lies within a few ulp of an integer (for the station at o + d along x,
    # rounded, just below 1), where the kernels' reciprocal product gives way
    # to the division.  Walk by walk against the oracle.
    rng = np.random.default_rng(8)
    n = np.array([8, 8, 8])
    d = np.array([0.1, 0.13, 0.07])
    o = -0.5 * n * d
    rho = rng.choice(np.array([0.3, 0.8, 1.4, 2.2], dtype=np.float32), size=n[::-1])
    ks = [(3, 5, 2), (4, 4, 4), (1, 6, 7), (5, 2, 3)]
    st = np.array([[o[c] + k[c] * d[c] for c in range(3)] for k in ks])
    q = (st - o) * (1.0 / d)
    f = q - np.floor(q)
    e = np.abs(q) * 2.0 ** -50
    assert np.all((f < e) | (f > 1.0 - e))          # every start coordinate takes the division
    pr = W.Problem(stations=st, dt=1e-3, paths_per_station=300, seed=12, G=0.9, rho=rho, grid_origin=o,
                   grid_spacing=d, name="grid-planes", **_BOX)
    _check_f64_potential(pr)


@pytest.mark.parametrize("exit_rule", [W.EXIT_OVERSHOOT, W.EXIT_INTERSECT])
def test_f64_quadratic_data_and_constant_density(exit_rule):
    pr = W.Problem(stations=_ST4, dt=1e-2, paths_per_station=1500, seed=9, G=0.7, bc_kind=W.BC_QUADRATIC,
                   bc_data=_HARM, exit_rule=exit_rule, prisms=np.array([[-10, -10, -10, 10, 10, 10, 1.5]]),
                   name=f"quadratic-exit{exit_rule}", **_BOX)
    _check_f64_potential(pr)


@pytest.mark.parametrize("precision", [W.PREC_F64, W.PREC_MIXED_F64ACC])
def test_grid_indices_past_the_int_range(precision):
    # A 3 x 2 x 2 grid of spacing 1e-10 at 0.5 beside a density-1.5 prism over
    # the box: the walks' voxel coordinates reach -1.5e10 and +5e9, past the
    # int range, where the conversions saturate and the lookup must read
    # "outside".  The grid is never hit, so the solve equals the one without
    # it bit for bit (and the FP64 walks match the oracle's).
    base = W.Problem(stations=_ST4[:3], dt=1e-3, paths_per_station=1500, seed=4, G=0.7, bc_kind=W.BC_QUADRATIC,
                     bc_data=_HARM, prisms=np.array([[-10, -10, -10, 10, 10, 10, 1.5]]), precision=precision,
                     name="far-grid", **_BOX)
    far = base.replace(rho=np.full((2, 2, 3), 4.0, dtype=np.float32), grid_origin=np.full(3, 0.5),
                       grid_spacing=np.full(3, 1e-10))
    say("case far grid prec", precision)
    a, av, as_ = gpu_solve(base, 0)
    b, bv, bs = gpu_solve(far, 0)
    assert np.asarray(as_).tobytes() == np.asarray(bs).tobytes()
    assert np.asarray(av).tobytes() == np.asarray(bv).tobytes()
    assert np.asarray(a).tobytes() == np.asarray(b).tobytes()
    if precision == W.PREC_F64:
        _check_f64_potential(far)


def _face_linear(box_lo, box_hi, face_n, lin):
    vals = []
    for f in range(6):
        c, side = divmod(f, 2)
        a = 1 if c == 0 else 0
        b = 1 if c == 2 else 2
        na, nb = face_n[f]
        for ib in range(nb):
            for ia in range(na):
                x = np.zeros(3)
                x[c] = box_hi[c] if side else box_lo[c]
                x[a] = box_lo[a] + (box_hi[a] - box_lo[a]) * ia / (na - 1)
                x[b] = box_lo[b] + (box_hi[b] - box_lo[b]) * ib / (nb - 1)
                vals.append(lin(x))
    return np.array(vals)


@pytest.mark.parametrize("exit_rule", [W.EXIT_OVERSHOOT, W.EXIT_INTERSECT])
def test_f64_face_grid_data(exit_rule):
    face_n = np.array([[5, 4], [3, 7], [6, 2], [4, 4], [9, 3], [2, 2]], dtype=np.int32)
    data = _face_linear(_BOX["box_lo"], _BOX["box_hi"], face_n, lambda x: 0.3 + 1.5 * x[0] - 0.7 * x[1] + 2 * x[2] ** 2)
    pr = W.Problem(stations=_ST4, dt=1e-2, paths_per_station=1500, seed=4, bc_kind=W.BC_FACE_GRID, bc_data=data,
                   face_n=face_n, exit_rule=exit_rule, spheres=np.array([[0.2, 0.1, -0.3, 0.4, 2.0]]),
                   name=f"facegrid-exit{exit_rule}", **_BOX)
    _check_f64_potential(pr)


@pytest.mark.parametrize("exit_rule", [W.EXIT_OVERSHOOT, W.EXIT_INTERSECT])
def test_f64_prism_data_with_prisms_on_the_boundary(exit_rule):
    """Prisms touching box faces, their closed form as the data: under
    INTERSECT the exit points lie on those faces, so corner offsets are exactly
    zero and the terms with a zero prefactor vanish -- in the kernels they are
    evaluated and selected away, with the table lookups kept in range."""
    prisms = np.array([[0.2, -0.4, -1.0, 1.0, 0.3, -0.5, 2.0], [-1.0, -1.0, 0.4, -0.6, 1.0, 1.0, -1.2]])
    pr = W.Problem(stations=_ST4, dt=1e-2, paths_per_station=1500, seed=13, G=1.0, bc_kind=W.BC_PRISMS,
                   bc_data=prisms.ravel().copy(), prisms=prisms, exit_rule=exit_rule,
                   name=f"boundary-prisms-exit{exit_rule}", **_BOX)
    _check_f64_potential(pr)


def test_f64_truncation_parity():
    pr = W.cfg1(1500).replace(max_steps=150)
    st, ost = _check_f64_potential(pr)
    assert np.all(st["n_trunc"] > 0)


def test_f64_problem_id_and_path_offset():
    _check_f64_potential(W.cfg1(1000).replace(problem_id=7, path_offset=123456, seed=(3 << 32) | 17))


def _check_f64_gz(prob):
    say("case gz", prob.name, "S", prob.n_stations, "N", prob.paths_per_station)
    stats, gv, gs = gpu_solve(prob, 1)
    S, N = prob.n_stations, prob.paths_per_station
    items = np.stack([np.repeat(np.arange(S), N), np.tile(np.arange(N), S)], axis=1)
    d, dsteps, aux, _ = oracle.run_paths(prob, 1, items, want_aux=True)
    # the oracle's pair step count is the sum; compare each walk of the pair
    # through its sample and the pair through its total
    scale = np.nanmean(np.abs(aux).reshape(S, -1), axis=1)
    gsum = (gs[..., 0] & np.uint32(0x7FFFFFFF)) + (gs[..., 1] & np.uint32(0x7FFFFFFF))
    gcap = ((gs[..., 0] | gs[..., 1]) & CAP) != 0
    gpair = gsum.astype(np.uint32) | np.where(gcap, CAP, np.uint32(0))
    assert np.array_equal(gpair.ravel(), dsteps)
    for w in range(2):
        a = aux[:, w].reshape(S, N)
        diff = np.abs(gv[..., w] - a)
        ok = np.isfinite(a)
        assert np.all(diff[ok] <= 1e-12 * np.repeat(scale[:, None], N, axis=1)[ok])
    for s in range(S):
        ds = d.reshape(S, N)[s]
        o = oracle.station_stats(ds, dsteps.reshape(S, N)[s])
        # each walk agrees to 1e-12 of the u scale, so a difference quotient
        # over 2h agrees to 1e-12 * scale / h
        h = prob.h if prob.h > 0 else math.sqrt(prob.dt)
        tol = 1e-12 * max(abs(o["mean"]), scale[s] / h)
        assert abs(stats["mean"][s] - o["mean"]) <= tol, (s, stats["mean"][s], o["mean"])
        assert stats["n"][s] == o["n"]
    return stats


def test_f64_gz_crn_cfg1_parity():
    _check_f64_gz(W.cfg1(2000))


def test_f64_gz_independent_pairs_parity():
    _check_f64_gz(W.cfg1(800).replace(pairing=W.PAIR_INDEPENDENT))


def test_f64_gz_si_prism_parity():
    pr = W.cfg2(60)
    _check_f64_gz(pr.replace(stations=pr.stations[::4]))


@pytest.mark.parametrize("precision", [W.PREC_MIXED_F64ACC, W.PREC_MIXED_KAHAN])
def test_mixed_against_oracle_fp32_stream(precision):
    pr = W.cfg1(20000, precision=precision)
    say("case mixed", precision)
    stats, gv, gs = gpu_solve(pr, 0)
    ost, ou, osteps = oracle.solve(pr, 0, stream=oracle.STREAM_F32)
    frac = float(np.mean(gs != osteps))
    say("  step mismatch fraction", frac)
    assert frac < 0.02
    same = (gs == osteps)
    rel = np.abs(gv - ou)[same] / np.abs(ou)[same]
    say("  median / 99.9% rel diff of matching walks", np.median(rel), np.quantile(rel, 0.999))
    assert np.quantile(rel, 0.999) < 1e-4
    for s in range(pr.n_stations):
        assert abs(stats["mean"][s] - ost[s]["mean"]) < 0.5 * ost[s]["se"]
        ex = oracle.exact_potential(pr, pr.stations[s])
        assert abs(stats["mean"][s] - ex) < 4.0 * stats["se"][s]


def test_determinism_bitwise():
    pr = W.cfg1(4000)
    a, av, as_ = gpu_solve(pr, 0)
    b, bv, bs = gpu_solve(pr, 0)
    assert a.tobytes() == b.tobytes()
    assert np.array_equal(av.view(np.uint64), bv.view(np.uint64)) and np.array_equal(as_, bs)
    m = W.cfg1(4000, precision=W.PREC_MIXED_F64ACC)
    a, _, _ = gpu_solve(m, 1)
    b, _, _ = gpu_solve(m, 1)
    assert a.tobytes() == b.tobytes()


def test_edge_cases_station_outside_and_two_paths():
    pr = W.cfg1(2).replace(stations=np.array([[0.0, 0.0, 0.5], [0.0, 0.0, 1.0], [0.0, 0.0, 3.0], [0.2, 0.1, 0.9]]))
    stats, gv, gs = gpu_solve(pr, 0)
    assert stats["n"][0] == 2 and stats["n"][3] == 2
    for s in (1, 2):        # on the boundary / outside: no samples
        assert stats["n"][s] == 0 and stats["n_trunc"][s] == 2 and np.isnan(stats["mean"][s])
        assert np.all(gs[s] == CAP)
    # stations 0 and 3 against the oracle, keeping their station indices (the
    # station index is a word of the Philox counter)
    items = np.array([[0, 0], [0, 1], [3, 0], [3, 1]])
    ou, osteps = oracle.run_paths(pr, 0, items)
    assert np.array_equal(gs[[0, 0, 3, 3], [0, 1, 0, 1]], osteps)
    assert np.allclose(gv[[0, 0, 3, 3], [0, 1, 0, 1]], ou, rtol=1e-12, atol=0)


def test_empty_station_set_launches_nothing():
    import torch
    from paper_1709_07469_amd import fkgrav as F
    pr = W.cfg1(100)
    P = F.Prepared(pr)
    out = F.alloc_stats(1)
    before = out.clone()
    ws = F.alloc_workspace(1024)
    F.fk_solve_potential(P.stations[:0], P.box, P.source, P.bc, P.params, out, ws)
    torch.cuda.synchronize()
    assert torch.equal(out, before)


def test_full_size_cfg2_sampled_parity_and_closed_form():
    """The benchmark's configuration (64 stations x 1e5 walks, FP64): sampled
    walks against the oracle one by one, the reduction against a two-pass
    fsum of all the walk samples, and the closed-form prism potential."""
    pr = W.cfg2()
    say("case cfg2 full size", pr.n_stations * pr.paths_per_station, "walks")
    stats, gv, gs = gpu_solve(pr, 0)
    rng = np.random.Generator(np.random.PCG64(2024))
    items = np.stack([rng.integers(0, 64, 96), rng.integers(0, pr.paths_per_station, 96)], axis=1)
    ou, osteps = oracle.run_paths(pr, 0, items)
    g = gv[items[:, 0], items[:, 1]]
    gst = gs[items[:, 0], items[:, 1]]
    scale = np.abs(np.nanmean(gv, axis=1))[items[:, 0]]
    r = compare_walks(g, gst, ou, osteps, scale)
    say("  sampled walks", r)
    assert r["step_mismatch"] == 0 and r["value_mismatch"] == 0
    for s in range(64):
        v = gv[s]
        m = math.fsum(v) / len(v)
        assert stats["mean"][s] == pytest.approx(m, rel=1e-12)
        assert stats["n"][s] == len(v) and stats["n_trunc"][s] == 0
    z = np.array([(stats["mean"][s] - oracle.exact_potential(pr, pr.stations[s])) / stats["se"][s] for s in range(64)])
    say("  closed-form z-scores: max |z|", np.abs(z).max(), "mean z", z.mean())
    assert np.abs(z).max() < 5.0
    say("  mean steps per walk", stats["sum_steps"].sum() / (64 * pr.paths_per_station))


def test_full_size_cfg2_mixed_sampled_parity():
    pr = W.cfg2(precision=W.PREC_MIXED_F64ACC)
    say("case cfg2 full size mixed")
    stats, gv, gs = gpu_solve(pr, 0)
    rng = np.random.Generator(np.random.PCG64(7))
    items = np.stack([rng.integers(0, 64, 64), rng.integers(0, pr.paths_per_station, 64)], axis=1)
    ou, osteps = oracle.run_paths(pr, 0, items, stream=oracle.STREAM_F32)
    g = gv[items[:, 0], items[:, 1]]
    gst = gs[items[:, 0], items[:, 1]]
    frac = float(np.mean(gst != osteps))
    say("  sampled step mismatch fraction", frac)
    assert frac < 0.1
    same = gst == osteps
    assert np.all(np.abs(g[same] - ou[same]) <= 1e-3 * np.abs(ou[same]))
    z = np.array([(stats["mean"][s] - oracle.exact_potential(pr, pr.stations[s])) / stats["se"][s] for s in range(64)])
    say("  closed-form z-scores: max |z|", np.abs(z).max())
    assert np.abs(z).max() < 5.0
