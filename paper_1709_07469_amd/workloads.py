"""Seeded synthetic problem descriptions for the Monte Carlo gravity solver.

This module only builds inputs: boxes, station sets, density models (analytic
prisms and spheres, voxel grids filled from voxel-aligned prisms) and the
parameters of a run.  It holds none of the estimator's arithmetic, so both the
HIP library's binding and the independent CPU oracle can consume the same
``Problem`` objects.

Workloads follow the paper's set-up (section 3: a homogeneous 100 m cube of
2000 kg/m^3 observed from stations on lines and grids above it) scaled to the
five concrete configurations used for testing and measurement:

  cfg1  uniform ball in the cube [-1,1]^3, G = 1, exact point-mass data
  cfg2  one SI prism below an 8x8 station grid, exact prism data (bench)
  cfg3  128^3 voxel grid of 5 random prisms, 16x16 stations, mixed precision
  cfg4  32 random voxel models of uneven size in one batched launch
  cfg5  32^3 voxel grid, 32 stations, adjoint d g_z / d rho

and the paper's own model (section 3): the ball of radius 10 km with zero
Dirichlet data around the 100 m cube, observed on the lines and the grid of
its experiments 1-3 (lengths in km).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

# Boundary-data kinds, exit rules, precisions and g_z pairings (the values of
# the C interface's enumerations).
BC_ZERO, BC_QUADRATIC, BC_POINT_MASSES, BC_PRISMS, BC_FACE_GRID = 0, 1, 2, 3, 4
EXIT_OVERSHOOT, EXIT_INTERSECT, EXIT_BRIDGE = 0, 1, 2
PREC_F64, PREC_MIXED_F64ACC, PREC_MIXED_KAHAN = 0, 1, 2
PAIR_CRN, PAIR_INDEPENDENT = 0, 1
DOMAIN_BOX, DOMAIN_BALL = 0, 1

G_SI = 6.674e-11
G_KM = 6.674e-20          # km^3 kg^-1 s^-2


@dataclass
class Problem:
    """One forward problem: domain, stations, density, boundary data and
    run parameters.  Arrays are host numpy arrays.

    The domain is the box [box_lo, box_hi], or with domain = DOMAIN_BALL the
    ball inscribed in it (the box must then be a cube).

    rho is indexed [k, j, i] (x fastest) over voxels whose (0,0,0) corner is
    grid_origin with edge lengths grid_spacing.  prisms rows are
    (x1, y1, z1, x2, y2, z2, rho); spheres rows are (cx, cy, cz, radius, rho).
    bc_data rows depend on bc_kind: QUADRATIC 10 coefficients (c0, b, A00,
    A01, A02, A11, A12, A22); POINT_MASSES rows (cx, cy, cz, mass); PRISMS
    rows as prisms; FACE_GRID the node values of the six faces in the order
    -x, +x, -y, +y, -z, +z with face_n[f] nodes along the face's two axes."""

    box_lo: np.ndarray
    box_hi: np.ndarray
    stations: np.ndarray
    dt: float
    paths_per_station: int
    seed: int = 0
    G: float = 1.0
    h: float = 0.0
    rho: np.ndarray | None = None
    grid_origin: np.ndarray = field(default_factory=lambda: np.zeros(3))
    grid_spacing: np.ndarray = field(default_factory=lambda: np.ones(3))
    prisms: np.ndarray = field(default_factory=lambda: np.zeros((0, 7)))
    spheres: np.ndarray = field(default_factory=lambda: np.zeros((0, 5)))
    bc_kind: int = BC_ZERO
    bc_data: np.ndarray = field(default_factory=lambda: np.zeros(0))
    face_n: np.ndarray = field(default_factory=lambda: np.zeros((6, 2), dtype=np.int32))
    precision: int = PREC_F64
    exit_rule: int = EXIT_OVERSHOOT
    pairing: int = PAIR_CRN
    domain: int = DOMAIN_BOX
    max_steps: int = 1 << 30
    problem_id: int = 0
    path_offset: int = 0
    # Reporting and workspace options of the HIP library (no effect on what
    # is computed): strict = report capped walks as an error; slice_walks > 0
    # = bounded workspace, walks run in slices of at most that many.
    strict: int = 0
    slice_walks: int = 0
    # the grid passed by levels (an index grid of bytes and 256 densities)
    # instead of FP32 densities: the same densities, a quarter of the memory
    grid_levels: bool = False
    name: str = ""
    # Prisms that the voxel grid represents exactly; kept for closed-form
    # targets only and never part of the source.
    model_prisms: np.ndarray = field(default_factory=lambda: np.zeros((0, 7)))

    @property
    def bc_n_items(self) -> int:
        d = np.asarray(self.bc_data).size
        if self.bc_kind == BC_POINT_MASSES:
            return d // 4
        if self.bc_kind == BC_PRISMS:
            return d // 7
        if self.bc_kind == BC_QUADRATIC:
            return 1
        if self.bc_kind == BC_FACE_GRID:
            return 6
        return 0

    @property
    def n_stations(self) -> int:
        return int(np.asarray(self.stations).reshape(-1, 3).shape[0])

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def line_stations(x, y, zs):
    zs = np.asarray(zs, dtype=np.float64)
    return np.stack([np.full_like(zs, x), np.full_like(zs, y), zs], axis=1)


def grid_stations(xs, ys, z):
    X, Y = np.meshgrid(np.asarray(xs, float), np.asarray(ys, float), indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, float(z))], axis=1)


def voxelize_prisms(prisms, n, origin, spacing):
    """Voxel grid (nz, ny, nx) float32 holding the sum of the densities of
    voxel-aligned prisms (each prism covers whole voxels)."""
    nx, ny, nz = (int(v) for v in n)
    rho = np.zeros((nz, ny, nx), dtype=np.float64)
    o = np.asarray(origin, float)
    d = np.asarray(spacing, float)
    for q in np.asarray(prisms, float).reshape(-1, 7):
        i0 = np.rint((q[:3] - o) / d).astype(int)
        i1 = np.rint((q[3:6] - o) / d).astype(int)
        rho[i0[2]:i1[2], i0[1]:i1[1], i0[0]:i1[0]] += q[6]
    return rho.astype(np.float32)


def random_aligned_prisms(rng, n_prisms, n, origin, spacing, edge_lo, edge_hi, z_hi, contrasts):
    """n_prisms voxel-aligned prisms with integer edge lengths in
    [edge_lo, edge_hi] voxels, lying inside the grid and below z = z_hi."""
    nx, ny, nz = n
    o = np.asarray(origin, float)
    d = np.asarray(spacing, float)
    kz_top = int(np.floor((z_hi - o[2]) / d[2]))
    rows = []
    for j in range(n_prisms):
        e = rng.integers(edge_lo, edge_hi + 1, size=3)
        e[2] = min(e[2], kz_top)
        i0 = rng.integers(0, nx - e[0] + 1)
        j0 = rng.integers(0, ny - e[1] + 1)
        k0 = rng.integers(0, kz_top - e[2] + 1)
        lo = o + d * np.array([i0, j0, k0])
        hi = o + d * np.array([i0 + e[0], j0 + e[1], k0 + e[2]])
        rows.append(np.concatenate([lo, hi, [contrasts[j]]]))
    return np.array(rows, dtype=np.float64).reshape(-1, 7)


# --------------------------------------------------------------------------
# The five configurations.
# --------------------------------------------------------------------------

def cfg1(paths_per_station=10_000, precision=PREC_F64) -> Problem:
    """Uniform ball (radius 0.25, density 1) at the centre of [-1,1]^3, G = 1,
    data = its exterior potential -M/|x| (a point mass), 8 stations on the
    z axis at z = 0.30 ... 0.65, dt = 1e-3."""
    a, rho = 0.25, 1.0
    M = 4.0 / 3.0 * np.pi * a ** 3 * rho
    return Problem(
        box_lo=np.array([-1.0, -1.0, -1.0]), box_hi=np.array([1.0, 1.0, 1.0]),
        stations=line_stations(0.0, 0.0, np.linspace(0.30, 0.65, 8)),
        dt=1e-3, paths_per_station=paths_per_station, seed=0, G=1.0,
        spheres=np.array([[0.0, 0.0, 0.0, a, rho]]),
        bc_kind=BC_POINT_MASSES, bc_data=np.array([0.0, 0.0, 0.0, M]),
        precision=precision, name="cfg1-sphere")


def cfg2(paths_per_station=100_000, precision=PREC_F64) -> Problem:
    """SI prism [400,600]x[450,550]x[-300,-150] m, contrast 300 kg/m^3, in the
    box [0,1000]^2 x [-500,100] m; data = the prism's closed-form potential;
    64 stations on the cell-centred 8x8 grid at z = 0; sqrt(dt) = 2 m."""
    prism = np.array([[400.0, 450.0, -300.0, 600.0, 550.0, -150.0, 300.0]])
    xs = 62.5 + 125.0 * np.arange(8)
    return Problem(
        box_lo=np.array([0.0, 0.0, -500.0]), box_hi=np.array([1000.0, 1000.0, 100.0]),
        stations=grid_stations(xs, xs, 0.0),
        dt=4.0, paths_per_station=paths_per_station, seed=0, G=G_SI, h=2.0,
        prisms=prism, bc_kind=BC_PRISMS, bc_data=prism.ravel().copy(),
        precision=precision, name="cfg2-prism-si")


def cfg3(paths_per_station=1_000_000, precision=PREC_MIXED_F64ACC, model_seed=3, n=128) -> Problem:
    """[-1,1]^3, G = 1, n^3 FP32 grid (spacing 2/n) holding 5 voxel-aligned
    prisms with edges of 8-32 voxels (scaled with n) below z = 0.25 and
    log-normal contrasts exp(N(ln 200, 0.5^2)); data = the prisms' closed-form
    potential; 16x16 stations at z = 0.5; dt = 1e-3."""
    rng = np.random.Generator(np.random.PCG64(model_seed))
    o = np.array([-1.0, -1.0, -1.0])
    d = np.full(3, 2.0 / n)
    contrasts = np.exp(rng.normal(np.log(200.0), 0.5, size=5))
    s = n / 128.0
    prisms = random_aligned_prisms(rng, 5, (n, n, n), o, d, max(1, int(8 * s)), max(2, int(32 * s)),
                                   0.25, contrasts)
    xs = np.linspace(-0.75, 0.75, 16)
    return Problem(
        box_lo=o.copy(), box_hi=-o, stations=grid_stations(xs, xs, 0.5),
        dt=1e-3, paths_per_station=paths_per_station, seed=0, G=1.0,
        rho=voxelize_prisms(prisms, (n, n, n), o, d), grid_origin=o, grid_spacing=d,
        bc_kind=BC_PRISMS, bc_data=prisms.ravel().copy(), precision=precision,
        name=f"cfg3-voxel{n}", model_prisms=prisms)


def cfg4(n_models=32, precision=PREC_MIXED_F64ACC, paths_scale=1.0, n=64) -> list[Problem]:
    """32 independent models: box [0,2] x [0,2a] x [-(5/6)2b, (1/6)2b] with
    a, b ~ U[1,4]; n^3 FP32 grid over the box with 1-8 voxel-aligned prisms
    (edges 4-16 voxels) below z = 0 and contrasts U[50,500]; 8-256 stations on
    a near-square grid at z = 0 over the central 75% of x and y; paths per
    station 10^U[4,6] (times paths_scale), dt = 1e-3, G = 1."""
    out = []
    for m in range(n_models):
        rng = np.random.Generator(np.random.PCG64(4000 + m))
        a, b = rng.uniform(1.0, 4.0, size=2)
        lo = np.array([0.0, 0.0, -(5.0 / 6.0) * 2.0 * b])
        hi = np.array([2.0, 2.0 * a, (1.0 / 6.0) * 2.0 * b])
        d = (hi - lo) / n
        n_pr = int(rng.integers(1, 9))
        contrasts = rng.uniform(50.0, 500.0, size=n_pr)
        e_hi = max(2, int(16 * n / 64))
        e_lo = max(1, int(4 * n / 64))
        prisms = random_aligned_prisms(rng, n_pr, (n, n, n), lo, d, e_lo, e_hi, 0.0, contrasts)
        ns = int(rng.integers(8, 257))
        nx = int(np.ceil(np.sqrt(ns)))
        ny = int(np.ceil(ns / nx))
        cx = np.linspace(lo[0] + 0.125 * (hi[0] - lo[0]), hi[0] - 0.125 * (hi[0] - lo[0]), nx)
        cy = np.linspace(lo[1] + 0.125 * (hi[1] - lo[1]), hi[1] - 0.125 * (hi[1] - lo[1]), ny)
        st = grid_stations(cx, cy, 0.0)[:ns]
        N = int(round(10.0 ** rng.uniform(4.0, 6.0) * paths_scale))
        out.append(Problem(
            box_lo=lo, box_hi=hi, stations=st, dt=1e-3, paths_per_station=max(N, 2), seed=0, G=1.0,
            rho=voxelize_prisms(prisms, (n, n, n), lo, d), grid_origin=lo.copy(), grid_spacing=d,
            bc_kind=BC_PRISMS, bc_data=prisms.ravel().copy(), precision=precision,
            problem_id=m, name=f"cfg4-model{m}", model_prisms=prisms))
    return out


def cfg5(paths_per_station=1_000_000, precision=PREC_F64, model_seed=5) -> Problem:
    """cfg3's generator on a 32^3 grid (spacing 1/16) with 5 prisms of 2-8
    voxel edges; fixed zero boundary data; 32 stations (8 x 4) at z = 0.5;
    dt = 1e-3; h = sqrt(dt)."""
    rng = np.random.Generator(np.random.PCG64(model_seed))
    n = 32
    o = np.array([-1.0, -1.0, -1.0])
    d = np.full(3, 2.0 / n)
    contrasts = np.exp(rng.normal(np.log(200.0), 0.5, size=5))
    prisms = random_aligned_prisms(rng, 5, (n, n, n), o, d, 2, 8, 0.25, contrasts)
    st = grid_stations(np.linspace(-0.6, 0.6, 8), np.linspace(-0.45, 0.45, 4), 0.5)
    return Problem(
        box_lo=o.copy(), box_hi=-o, stations=st, dt=1e-3, paths_per_station=paths_per_station,
        seed=0, G=1.0, rho=voxelize_prisms(prisms, (n, n, n), o, d), grid_origin=o, grid_spacing=d,
        bc_kind=BC_ZERO, precision=precision, name="cfg5-voxel32", model_prisms=prisms)


def cfg5_fd_voxels(n_vox=32 ** 3, count=64, seed=55):
    """The 64 voxel indices probed by the finite-difference check of cfg5."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n_vox, size=count, replace=False))


# --------------------------------------------------------------------------
# The paper's model (section 3), in km: lengths in km make the reported run
# times consistent with the expected exit time of a 10 km ball.
# --------------------------------------------------------------------------

PAPER_R_KM = 10.0
PAPER_CUBE_KM = np.array([0.0, 0.0, 0.0, 0.1, 0.1, 0.1])
PAPER_RHO = 2.0e12        # 2000 kg/m^3 in kg/km^3


def paper_exp1_stations() -> np.ndarray:
    """Experiment 1: the line y = 50 m, z = 200 m, x = -100 m .. 200 m every 10 m."""
    x = np.round(np.arange(-10, 21) * 0.01, 12)
    return np.stack([x, np.full_like(x, 0.05), np.full_like(x, 0.2)], axis=1)


def paper_exp2_stations() -> np.ndarray:
    """Experiment 2: the vertical line x = y = 50 m, z = -100 m .. 200 m every 10 m."""
    z = np.round(np.arange(-10, 21) * 0.01, 12)
    return np.stack([np.full_like(z, 0.05), np.full_like(z, 0.05), z], axis=1)


def paper_exp3_stations() -> np.ndarray:
    """Experiment 3: a 21 x 11 grid in the plane y = 50 m, x spread evenly
    over -100 m .. 200 m and z = 195 m .. 205 m every metre (z fastest)."""
    x = np.linspace(-0.1, 0.2, 21)
    z = np.round(0.2 + np.arange(-5, 6) * 0.001, 12)
    X, Z = np.meshgrid(x, z, indexing="ij")
    return np.stack([X.ravel(), np.full(X.size, 0.05), Z.ravel()], axis=1)


def paper_ball(stations=None, dt_paper=0.01, paths_per_station=51200, precision=PREC_F64,
               radius=PAPER_R_KM) -> Problem:
    """The paper's model: ball of radius 10 km about the origin with zero
    Dirichlet data, a homogeneous cube [0, 100 m]^3 of 2000 kg/m^3, G in km
    units.  The paper's walk is sqrt(2) W with step sqrt(2 Delta t), the same
    paths as standard Brownian motion with dt = 2 Delta t."""
    st = paper_exp1_stations() if stations is None else np.asarray(stations, dtype=np.float64).reshape(-1, 3)
    cube = np.concatenate([PAPER_CUBE_KM, [PAPER_RHO]])[None, :]
    return Problem(
        box_lo=np.full(3, -radius), box_hi=np.full(3, radius), stations=st,
        dt=2.0 * dt_paper, paths_per_station=paths_per_station, seed=0, G=G_KM,
        prisms=cube, bc_kind=BC_ZERO, precision=precision, domain=DOMAIN_BALL,
        name="paper-ball-10km")
