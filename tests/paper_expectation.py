"""Expected values of the paper's model (section 3: a ball of radius 10 km
with zero data around a 100 m cube of 2000 kg/m^3, lengths in km) for the
discrete walk and for the continuous one.

The ball is far away (10 km against a cube 100-300 m from the stations), so
the discrete walk's expected trapezoid sum is that of the unbounded Gaussian
walk,
    dt [ 1/2 1(x0 in cube) + sum_{n >= 1} P(x0 + sqrt(n dt) Z in cube) ],
each probability a product of three normal-CDF differences (the sum's tail
beyond n = NMAX taken from its n^(-3/2) asymptote), minus the occupation after
the walk has left the ball, which is the continuous walk's to well below the
statistical errors: the Kelvin-image term G rho (V/R + x0.m1/R^3).
Replacing the sum by its continuous limit gives the Green's-function solution
(the cube's potential plus the image term)."""
import math

import numpy as np
from scipy.special import erf

import oracle

NMAX = 20000


def _cube(pr):
    q = pr.prisms[0]
    return q[:3], q[3:6], q[6]


def _image(pr, x0):
    """The Kelvin-image term of the ball's Green function, to first order in
    |x0| |y| / R^2, integrated over the cube."""
    lo, hi, rho = _cube(pr)
    V = float(np.prod(hi - lo))
    m1 = V * 0.5 * (lo + hi)
    R = 0.5 * (pr.box_hi[0] - pr.box_lo[0])
    return pr.G * rho * (V / R + float(np.dot(x0, m1)) / R ** 3)


def discrete_potential(pr, x0):
    """Expected sample of the discrete walk from x0 (see the module text)."""
    lo, hi, rho = _cube(pr)
    x0 = np.asarray(x0, dtype=np.float64)
    n = np.arange(1, NMAX + 1, dtype=np.float64)[:, None]
    s = np.sqrt(2.0 * n * pr.dt)
    P = np.prod(0.5 * (erf((hi - x0) / s) - erf((lo - x0) / s)), axis=1)
    V = float(np.prod(hi - lo))
    tail = V / (2.0 * math.pi * pr.dt) ** 1.5 * 2.0 / math.sqrt(NMAX + 0.5)
    inside = float(np.all((x0 >= lo) & (x0 < hi)))
    occ = pr.dt * (0.5 * inside + float(P.sum()) + tail)
    return -2.0 * math.pi * pr.G * rho * occ + _image(pr, x0)


def green_potential(pr, x0):
    lo, hi, rho = _cube(pr)
    return oracle.prism_potential(lo, hi, rho, pr.G, x0) + _image(pr, x0)


def green_gz(pr, x0):
    lo, hi, rho = _cube(pr)
    V = float(np.prod(hi - lo))
    R = 0.5 * (pr.box_hi[0] - pr.box_lo[0])
    return oracle.prism_gz(lo, hi, rho, pr.G, x0) + pr.G * rho * V * 0.5 * (lo[2] + hi[2]) / R ** 3
