"""The FP64 voxel floor of the HIP kernels: floor(q) of q = (x - o) * inv,
inv = 1/d rounded, stands for the floor of the rounded quotient (x - o) / d
unless q lies within 2^-50 |q| of an integer (there the kernel divides).
The product is within 3 ulp of the quotient (a rounding each in inv, the
product and the division), so the margin of 8 ulp decides every case; this
checks the claim on quotients placed a few ulp from integers, and that a
zero margin would not."""
import numpy as np


def _cases(rng, n):
    d = np.exp(rng.uniform(np.log(1e-6), np.log(1e4), n))
    k = rng.integers(-2 ** 22, 2 ** 22, n).astype(np.float64)
    a = k * d
    j = rng.integers(-12, 13, n)
    a = a + j * np.spacing(np.abs(a) + 1e-300) * np.sign(rng.standard_normal(n))
    m = rng.random(n) < 0.3
    a[m] = rng.uniform(-1e3, 1e3, m.sum())
    return a, d


def _fast_floor(a, d, margin):
    q = a * (1.0 / d)
    t = np.floor(q)
    f = q - t
    e = np.abs(q) * margin
    near = (f < e) | (f > 1.0 - e)
    return np.where(near, np.floor(a / d), t), near


def test_reciprocal_floor_with_margin_is_the_quotient_floor():
    rng = np.random.default_rng(1)
    a, d = _cases(rng, 2_000_000)
    fast, near = _fast_floor(a, d, 2.0 ** -50)
    assert np.array_equal(fast, np.floor(a / d))
    assert 0.05 < near.mean() < 0.6          # the cases do sit near integers


def test_without_the_margin_the_product_floor_differs():
    rng = np.random.default_rng(1)
    a, d = _cases(rng, 2_000_000)
    fast, _ = _fast_floor(a, d, 0.0)
    assert np.sum(fast != np.floor(a / d)) > 1000
