"""Pins of the oracle's lattice Green's function against what the paper and mathematics fix.

* G(0) equals the closed form of Watson's integral (Glasser & Zucker 1977, cited in Sec. 2);
* L G = delta: G(1,0,0) - G(0) = 1/6 exactly and the 7-point Laplacian of G vanishes at every
  other table point (definition of the LGF, Sec. 2);
* an independent 30-digit mpmath evaluation of eq. GL_B at a few points;
* the asymptotic expansions: A_G^2 error decays like |n|^-5 and A_G^3 like |n|^-7 (the paper's
  O(|n|^{-2q-1})), which fixes the sign of the degree-8 term, and G -> -1/(4 pi |n|);
* the evaluation policy switches are continuous to well below the paper's 1e-12 bound.
"""
import mpmath
import numpy as np
import pytest

from oracle import lgf


def test_origin_closed_form():
    g0 = lgf.lgf(np.array([0, 0, 0]))
    assert abs(g0 - lgf.watson_g0()) <= 2e-15 * abs(g0)
    # decimal value of the closed form (20 digits, Glasser & Zucker): -0.25273100985866300277
    assert abs(g0 - (-0.25273100985866300277)) <= 2e-16


def test_delta_at_origin():
    g = lgf.lgf(np.array([[0, 0, 0], [1, 0, 0], [0, -1, 0], [0, 0, 1]]))
    assert abs(g[1] - g[0] - 1.0 / 6.0) <= 1e-15
    assert g[1] == g[2] == g[3]


def test_laplacian_vanishes_over_table():
    tri = lgf.sorted_triples(99 * 99 - 1)     # every neighbour still inside the table
    tri = tri[(tri != 0).any(axis=1)]
    g = lgf.lgf(tri)
    nb = 0.0
    for e in np.eye(3, dtype=np.int64):
        nb = nb + lgf.lgf(tri + e) + lgf.lgf(tri - e)
    lap = nb - 6.0 * g
    assert np.abs(lap).max() <= 1e-14


def _mp_green(n):
    mpmath.mp.dps = 30
    f = lambda t: (mpmath.exp(-6 * t) * mpmath.besseli(n[0], 2 * t) * mpmath.besseli(n[1], 2 * t)
                   * mpmath.besseli(n[2], 2 * t))
    return -mpmath.quad(f, [0, 1, 10, 100, 1000, mpmath.inf])


@pytest.mark.parametrize("n", [(1, 1, 0), (1, 1, 1), (2, 1, 0), (3, 2, 1), (5, 0, 0)])
def test_independent_mpmath(n):
    ref = float(_mp_green(n))
    val = float(lgf.lgf(np.array(n)))
    assert abs(val - ref) <= 2e-15 * abs(ref)


def test_symmetry():
    rng = np.random.default_rng(0)
    n = rng.integers(-40, 41, size=(50, 3))
    g = lgf.lgf(n)
    assert np.array_equal(g, lgf.lgf(-n))
    assert np.array_equal(g, lgf.lgf(n[:, [2, 0, 1]]))


def test_asymptotic_decay_orders_fix_the_sign():
    dirs = [np.array([1, 0, 0]), np.array([1, 1, 1]), np.array([3, 2, 1])]
    for d in dirs:
        n1, n2 = 12 * d, 24 * d
        if (n2 * n2).sum() > lgf.TABLE_R2:
            n1, n2 = 8 * d, 16 * d
        g1, g2 = lgf.bessel_integral(np.stack([n1, n2]))
        e2 = [abs(g1 - lgf.asym2(n1)), abs(g2 - lgf.asym2(n2))]
        em = [abs(g1 - lgf.asym3(n1, -1.0)), abs(g2 - lgf.asym3(n2, -1.0))]
        ep = [abs(g1 - lgf.asym3(n1, +1.0)), abs(g2 - lgf.asym3(n2, +1.0))]
        if e2[1] > 1e-16:      # A_G^2 error falls like |n|^-5: ratio 32 per doubling
            assert 20 < e2[0] / e2[1] < 50
        assert em[0] / em[1] > 80          # |n|^-7: ratio ~128
        assert ep[0] / ep[1] < 50          # printed sign: only |n|^-5
        assert em[1] < e2[1] and ep[1] >= e2[1]


def test_far_field_limit():
    n = np.array([[600, 0, 0], [300, 400, 100], [1000, 2000, 3000]])
    r = np.sqrt((n * n).sum(axis=1))
    rel = lgf.lgf(n) * (-4 * np.pi * r)
    assert np.all(np.abs(rel - 1.0) < 1.0 / r**2)


def test_policy_switches_are_continuous():
    # points just inside/outside |n| = 100 and |n| = 600 along several directions
    pts = np.array([[100, 0, 0], [60, 80, 0], [36, 48, 80], [600, 0, 0], [360, 480, 0]])
    table_side = lgf.bessel_integral(pts[:3])
    assert np.all(np.abs(table_side - lgf.asym3(pts[:3])) <= 1e-14)
    assert np.all(np.abs(lgf.asym3(pts[3:]) - lgf.asym2(pts[3:])) <= 1e-14)
    # the policy itself: table at r^2 <= 100^2, A3 up to 600^2, A2 beyond
    assert lgf.lgf(np.array([100, 0, 0])) == table_side[0]
    assert lgf.lgf(np.array([101, 0, 0])) == lgf.asym3(np.array([101, 0, 0]))
    assert lgf.lgf(np.array([601, 0, 0])) == lgf.asym2(np.array([601, 0, 0]))


def test_quadrature_converged():
    n = np.array([[0, 0, 0], [7, 3, 1], [70, 50, 30], [100, 0, 0]])
    a = lgf.bessel_integral(n, h=1.0 / 256)
    b = lgf.bessel_integral(n, h=1.0 / 128)
    assert np.all(np.abs(a - b) <= 2e-16 * 8 * np.abs(a))


def test_hankel_matches_scipy_overlap():
    from scipy import special
    x = np.array([2e5, 1e6, 5e6])
    k = np.array([0, 7, 50, 100])
    h = lgf.ive_hankel(k[None, :], x[:, None], terms=12)
    s = special.ive(k[None, :], x[:, None])
    assert np.all(np.abs(h - s) <= 1e-14 * s)
