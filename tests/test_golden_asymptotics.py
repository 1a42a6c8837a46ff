"""The oracle's asymptotic expansions and evaluation policy against the coefficients, radii and
error bound printed in the paper (Sec. 2), stored in tests/golden/asymptotic_expansion.txt."""
import os

import numpy as np

from oracle import lgf

HERE = os.path.dirname(os.path.abspath(__file__))


def golden():
    out = {}
    for line in open(os.path.join(HERE, "golden", "asymptotic_expansion.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def points():
    rng = np.random.default_rng(1)
    p = rng.integers(-700, 701, size=(200, 3))
    return p[(p * p).sum(axis=1) > 50 ** 2]


def test_a2_coefficients_as_printed():
    g = golden()
    x = points().astype(np.float64)
    r = np.sqrt((x * x).sum(axis=1))
    x1, x2, x3 = x.T
    quart = x1**4 + x2**4 + x3**4 + g["a2_c22"] * (x1**2 * x2**2 + x1**2 * x3**2 + x2**2 * x3**2)
    ref = -1.0 / (g["a2_leading_denominator"] * np.pi * r) - quart / (g["a2_quartic_denominator"] * np.pi * r**7)
    assert np.allclose(lgf.asym2(points()), ref, rtol=1e-14, atol=0)


def test_a3_coefficients_as_printed_with_the_minus_reading():
    g = golden()
    x = points().astype(np.float64)
    r = np.sqrt((x * x).sum(axis=1))
    a, b, c = (x**2).T
    p8 = (g["a3_c422"] * (b * c * a * a + b * c * c * a + b * b * c * a)
          + g["a3_c44"] * (a * a * b * b + c * c * b * b + a * a * c * c)
          + g["a3_c62"] * (b * a**3 + c * a**3 + b**3 * a + c**3 * a + b * c**3 + b**3 * c)
          + g["a3_c8"] * (a**4 + b**4 + c**4))
    # the octic polynomial itself, then the assembled expansions (their difference is formed
    # from two values of size |A_G^2|, so it carries their rounding)
    assert np.allclose(lgf.octic(points()), p8, rtol=1e-13, atol=0)
    term = p8 / (g["a3_denominator"] * np.pi * r**13)
    d_read = lgf.asym3(points(), -1.0) - lgf.asym2(points())
    d_printed = lgf.asym3(points(), +1.0) - lgf.asym2(points())
    tol = 8 * np.finfo(float).eps * np.abs(lgf.asym2(points()))
    assert np.all(np.abs(d_read + term) <= tol)
    assert np.all(np.abs(d_printed - term) <= tol)


def test_policy_radii_and_error_bound():
    g = golden()
    R1, R2, eps = int(g["table_radius"]), int(g["a3_radius"]), g["error_bound"]
    assert lgf.TABLE_R2 == R1 * R1
    # at each switch the expansion taken there agrees with the quadrature within the stated
    # (absolute) bound
    for n in (np.array([R1, 0, 0]), np.array([60, 80, 0]), np.array([36, 48, 80])):
        assert abs(lgf.asym3(n) - lgf.bessel_integral(n[None])[0]) <= eps
    far = np.array([R2 + 1, 0, 0])
    assert lgf.lgf(far) == lgf.asym2(far)
    assert lgf.lgf(np.array([R2, 0, 0])) == lgf.asym3(np.array([R2, 0, 0]))
    assert abs(lgf.asym3(np.array([R2, 0, 0])) - lgf.asym2(np.array([R2, 0, 0]))) <= eps
