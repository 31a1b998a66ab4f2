"""The face-angle identity of the HIP kernels' prism closed form: for a face
U = const with corners (v_j, w_k), the alternating sum
sum_jk (-1)^(j+k) atan(v_j w_k / (|U| r_jk)) equals the argument of
E0 E1, E0 = c00 conj(c01), E1 = c11 conj(c10), c_jk = |U| r_jk + i v_j w_k,
plus 2 pi when both edge products have positive imaginary parts and the
product a negative one, minus 2 pi in the mirrored case.  Checked against
the four arctangents on random faces, on faces seen from just off their
plane (angles near +-2 pi) and from points over their edges and corners."""
import numpy as np


def _four_atans(U, v, w):
    s = 0.0
    for j in range(2):
        for k in range(2):
            r = np.sqrt(U * U + v[j] ** 2 + w[k] ** 2)
            s += (-1) ** (j + k) * np.arctan(v[j] * w[k] / (abs(U) * r))
    return s


def _face_angle(U, v, w):
    au = abs(U)
    c = [[complex(au * np.sqrt(U * U + v[j] ** 2 + w[k] ** 2), v[j] * w[k]) for k in range(2)] for j in range(2)]
    e0 = c[0][0] * np.conj(c[0][1])
    e1 = c[1][1] * np.conj(c[1][0])
    p = e0 * e1
    wrap = 0.0
    if e0.imag > 0 and e1.imag > 0 and p.imag < 0:
        wrap = 2 * np.pi
    elif e0.imag < 0 and e1.imag < 0 and p.imag > 0:
        wrap = -2 * np.pi
    return np.arctan2(p.imag, p.real) + wrap


def _check(U, v, w):
    a, b = _four_atans(U, v, w), _face_angle(U, v, w)
    assert abs(a - b) <= 1e-12 * max(1.0, abs(a)), (U, v, w, a, b)
    return a


def test_face_angle_random_faces():
    rng = np.random.default_rng(3)
    for _ in range(20000):
        U = rng.uniform(-5, 5)
        v = np.sort(rng.uniform(-5, 5, 2))
        w = np.sort(rng.uniform(-5, 5, 2))
        _check(U, v, w)


def test_face_angle_near_the_plane_reaches_two_pi():
    rng = np.random.default_rng(4)
    big = 0
    for _ in range(5000):
        U = rng.choice([-1, 1]) * 10.0 ** rng.uniform(-9, -1)
        v = np.array([rng.uniform(-3, -0.1), rng.uniform(0.1, 3)])   # the point projects inside the face
        w = np.array([rng.uniform(-3, -0.1), rng.uniform(0.1, 3)])
        a = _check(U, v, w)
        big += abs(a) > np.pi
    assert big > 4000                                                 # the wrap is exercised


def test_face_angle_over_edges_and_corners():
    for U in (1e-6, 0.3, -2.0):
        for v in ([0.0, 1.0], [-1.0, 0.0], [0.5, 2.0]):
            for w in ([0.0, 1.5], [-0.7, 0.0], [-2.0, -0.5]):
                _check(U, np.array(v), np.array(w))
