"""Pins for the closed forms the oracle uses as boundary data and as exact
targets: the homogeneous prism's Newtonian integral (the paper compares with
the cube's analytic potential, section 1 and section 3) and its vertical
derivative (the analytic g_z of section 4.2), and the uniform ball.

The prism integral is pinned against direct numerical quadrature with scipy,
the far field, superposition and the Laplacian (Poisson's equation, eq. 4),
so a wrong sign, corner or log branch fails here."""
import numpy as np
import pytest
from scipy import integrate

import oracle


def _quad_newton(lo, hi, P, kernel="V"):
    def f(z, y, x):
        dx, dy, dz = x - P[0], y - P[1], z - P[2]
        r = np.sqrt(dx * dx + dy * dy + dz * dz)
        return 1.0 / r if kernel == "V" else dz / r ** 3
    val, err = integrate.tplquad(f, lo[0], hi[0], lo[1], hi[1], lo[2], hi[2], epsabs=1e-12, epsrel=1e-11)
    return val


LO = np.array([0.0, 0.0, 0.0])
HI = np.array([1.0, 2.0, 0.5])

EXTERIOR = [np.array(p) for p in ([0.5, 1.0, 2.0], [-1.0, 0.3, 0.2], [3.0, -2.0, -1.5],
                                  [0.0, 0.0, 1.0], [1.0, 2.0, 0.5 + 1e-3], [0.5, 3.0, 0.25])]


@pytest.mark.parametrize("P", EXTERIOR)
def test_prism_newton_matches_quadrature_exterior(P):
    assert oracle.prism_newton(LO, HI, P) == pytest.approx(_quad_newton(LO, HI, P), rel=2e-9)


def test_prism_newton_matches_quadrature_interior():
    # interior point: split the prism at P so each piece has P on a corner
    P = np.array([0.3, 0.7, 0.2])
    tot = 0.0
    for xs in ((LO[0], P[0]), (P[0], HI[0])):
        for ys in ((LO[1], P[1]), (P[1], HI[1])):
            for zs in ((LO[2], P[2]), (P[2], HI[2])):
                tot += _quad_newton([xs[0], ys[0], zs[0]], [xs[1], ys[1], zs[1]], P)
    assert oracle.prism_newton(LO, HI, P) == pytest.approx(tot, rel=1e-8)


@pytest.mark.parametrize("P", EXTERIOR[:4])
def test_prism_gz_matches_quadrature(P):
    # g_z = dPhi/dz_P with Phi = -G rho V  =>  g_z = -G rho int (z - zP)/r^3 dV
    G, rho = 1.7, 2.3
    ref = -G * rho * _quad_newton(LO, HI, P, kernel="gz")
    assert oracle.prism_gz(LO, HI, rho, G, P) == pytest.approx(ref, rel=1e-8)


def test_prism_gz_is_derivative_of_potential():
    for P in EXTERIOR + [np.array([0.3, 0.7, 0.2])]:
        h = 1e-5
        up = oracle.prism_potential(LO, HI, 1.0, 1.0, P + [0, 0, h])
        um = oracle.prism_potential(LO, HI, 1.0, 1.0, P - [0, 0, h])
        assert oracle.prism_gz(LO, HI, 1.0, 1.0, P) == pytest.approx((up - um) / (2 * h), rel=1e-6, abs=1e-9)


def test_prism_far_field_and_sign():
    P = np.array([300.0, -200.0, 500.0])
    c = 0.5 * (LO + HI)
    M = np.prod(HI - LO)
    r = np.linalg.norm(P - c)
    assert oracle.prism_potential(LO, HI, 1.0, 1.0, P) == pytest.approx(-M / r, rel=1e-6)
    # the potential is negative and g_z points toward the mass: positive above
    assert oracle.prism_gz(LO, HI, 1.0, 1.0, [0.5, 1.0, 3.0]) > 0
    assert oracle.prism_gz(LO, HI, 1.0, 1.0, [0.5, 1.0, -3.0]) < 0


def test_prism_superposition():
    P = np.array([0.37, -0.8, 1.3])
    whole = oracle.prism_newton(LO, HI, P)
    mid = 0.5 * (LO + HI) + np.array([0.1, -0.2, 0.05])
    parts = 0.0
    for xs in ((LO[0], mid[0]), (mid[0], HI[0])):
        for ys in ((LO[1], mid[1]), (mid[1], HI[1])):
            for zs in ((LO[2], mid[2]), (mid[2], HI[2])):
                parts += oracle.prism_newton([xs[0], ys[0], zs[0]], [xs[1], ys[1], zs[1]], P)
    assert parts == pytest.approx(whole, rel=1e-12)


def _laplacian(f, P, h=1e-3):
    tot = -6.0 * f(P)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        tot += f(P + e) + f(P - e)
    return tot / h ** 2


def test_prism_poisson_equation():
    # Laplacian of Phi = -G rho V is 4 pi G rho inside and 0 outside
    G, rho = 1.0, 1.0
    f = lambda P: oracle.prism_potential(LO, HI, rho, G, P)
    assert _laplacian(f, np.array([0.4, 1.1, 0.3])) == pytest.approx(4 * np.pi * G * rho, rel=1e-4)
    assert abs(_laplacian(f, np.array([1.5, 1.1, 0.3]))) < 1e-4


def test_sphere_closed_form():
    c, a, rho, G = np.zeros(3), 0.25, 1.0, 1.0
    M = 4.0 / 3.0 * np.pi * a ** 3 * rho
    # continuity at the surface and the point-mass exterior
    for d in (np.array([0, 0, 1.0]), np.array([0.6, 0.0, 0.8])):
        assert oracle.sphere_potential(c, a, rho, G, a * d * (1 - 1e-12)) == pytest.approx(-M / a, rel=1e-9)
    assert oracle.sphere_potential(c, a, rho, G, [0, 0, 0.5]) == pytest.approx(-M / 0.5, rel=1e-15)
    f = lambda P: oracle.sphere_potential(c, a, rho, G, P)
    assert _laplacian(f, np.array([0.05, 0.02, 0.1])) == pytest.approx(4 * np.pi, rel=1e-6)
    assert abs(_laplacian(f, np.array([0.2, 0.3, 0.4]))) < 1e-5
    for P in (np.array([0.0, 0.0, 0.5]), np.array([0.05, 0.02, 0.1])):
        h = 1e-6
        fd = (f(P + [0, 0, h]) - f(P - [0, 0, h])) / (2 * h)
        assert oracle.sphere_gz(c, a, rho, G, P) == pytest.approx(fd, rel=1e-7)


def test_boundary_data_kinds():
    from paper_1709_07469_amd import workloads as W
    box_lo, box_hi = np.array([-1.0, -2.0, -0.5]), np.array([1.0, 2.0, 1.5])
    base = dict(box_lo=box_lo, box_hi=box_hi, stations=np.zeros((1, 3)), dt=1e-3, paths_per_station=1, G=2.0)
    x = np.array([0.3, -0.7, 1.9])
    # QUADRATIC: c0 + b.x + x^T A x with symmetric A given by its upper triangle
    q = np.array([0.5, 1.0, -2.0, 3.0, 0.1, 0.2, -0.3, 0.4, 0.5, -0.6])
    A = np.array([[0.1, 0.2, -0.3], [0.2, 0.4, 0.5], [-0.3, 0.5, -0.6]])
    pr = W.Problem(bc_kind=W.BC_QUADRATIC, bc_data=q, **base)
    assert oracle.bc_value(pr, x) == pytest.approx(0.5 + q[1:4] @ x + x @ A @ x, rel=1e-14)
    # POINT_MASSES: -sum G m / r
    pm = np.array([0.0, 0.0, 0.0, 2.0, 1.0, 1.0, 1.0, 0.5])
    pr = W.Problem(bc_kind=W.BC_POINT_MASSES, bc_data=pm, **base)
    ref = -2.0 * (2.0 / np.linalg.norm(x) + 0.5 / np.linalg.norm(x - 1.0))
    assert oracle.bc_value(pr, x) == pytest.approx(ref, rel=1e-14)
    # PRISMS: sum of prism potentials
    prs = np.array([0.0, 0.0, 0.0, 0.5, 0.5, 0.5, 3.0, -0.5, 0.0, 0.0, 0.0, 0.2, 0.2, 1.0])
    pr = W.Problem(bc_kind=W.BC_PRISMS, bc_data=prs, **base)
    ref = oracle.prism_potential(prs[:3], prs[3:6], 3.0, 2.0, x) + oracle.prism_potential(prs[7:10], prs[10:13], 1.0, 2.0, x)
    assert oracle.bc_value(pr, x) == pytest.approx(ref, rel=1e-14)


def _face_grid_linear(box_lo, box_hi, face_n, lin):
    """Node values of the linear function lin(x) on the six faces."""
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


def test_face_grid_reproduces_linear_data():
    # bilinear interpolation is exact for a linear function on every face
    from paper_1709_07469_amd import workloads as W
    box_lo, box_hi = np.array([-1.0, -2.0, -0.5]), np.array([1.0, 2.0, 1.5])
    face_n = np.array([[5, 4], [3, 7], [6, 2], [4, 4], [9, 3], [2, 2]], dtype=np.int32)
    lin = lambda x: 0.3 + 1.5 * x[0] - 0.7 * x[1] + 2.0 * x[2]
    pr = W.Problem(box_lo=box_lo, box_hi=box_hi, stations=np.zeros((1, 3)), dt=1e-3, paths_per_station=1,
                   bc_kind=W.BC_FACE_GRID, bc_data=_face_grid_linear(box_lo, box_hi, face_n, lin), face_n=face_n)
    rng = np.random.Generator(np.random.PCG64(1))
    for _ in range(200):
        x = rng.uniform(box_lo, box_hi)
        c = rng.integers(0, 3)
        x[c] = box_hi[c] if rng.random() < 0.5 else box_lo[c]
        assert oracle.bc_value(pr, x) == pytest.approx(lin(x), rel=1e-12, abs=1e-12)
    # a point beyond a face reads the clamped point on the face it is furthest beyond
    x = np.array([0.2, 0.1, 1.5 + 0.3])
    assert oracle.bc_value(pr, x) == pytest.approx(lin(np.array([0.2, 0.1, 1.5])), rel=1e-12)


def test_voxel_membership_is_half_open():
    from paper_1709_07469_amd import workloads as W
    rho = np.arange(2 * 3 * 4, dtype=np.float32).reshape(2, 3, 4)     # nz=2, ny=3, nx=4
    pr = W.Problem(box_lo=np.zeros(3), box_hi=np.ones(3), stations=np.zeros((1, 3)), dt=1e-3, paths_per_station=1,
                   rho=rho, grid_origin=np.array([0.0, 0.0, 0.0]), grid_spacing=np.array([0.25, 0.5, 0.5]))
    assert oracle.voxel_index(pr, [0.0, 0.0, 0.0]) == 0
    assert oracle.voxel_index(pr, [0.25, 0.0, 0.0]) == 1          # on a face -> upper voxel
    assert oracle.voxel_index(pr, [0.2499999, 0.5, 0.5]) == (1 * 3 + 1) * 4 + 0
    assert oracle.voxel_index(pr, [1.0, 0.1, 0.1]) == -1           # x = nx * d is outside
    assert oracle.voxel_index(pr, [-1e-300, 0.1, 0.1]) == -1
    assert oracle.rho_at(pr, [0.9, 1.4, 0.9]) == float(rho[1, 2, 3])
    assert oracle.rho_at(pr, [0.9, 1.6, 0.9]) == 0.0
