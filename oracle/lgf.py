"""Lattice Green's function G of the 7-point Laplacian, FP64 (test infrastructure only).

Follows Sec. 2 of the paper:

* eq. GL_B: G(n) = -int_0^inf exp(-6t) I_{n1}(2t) I_{n2}(2t) I_{n3}(2t) dt, written here with the
  exponentially scaled Bessel function ive(k, x) = exp(-x) I_k(x), so the integrand is
  ive(n1,2t) ive(n2,2t) ive(n3,2t).  Sign convention: L u(n) = sum of the 6 neighbours - 6 u(n)
  (the Fourier symbol 2 cos xi_1 + 2 cos xi_2 + 2 cos xi_3 - 6 of eq. GL), so G < 0 and L G = delta.
* the two- and three-term far-field expansions A_G^2 and A_G^3;
* the evaluation policy: quadrature table for |n| <= 100, A_G^3 for 100 < |n| <= 600 and
  A_G^2 beyond.  |n| is the Euclidean norm; the switches compare the integer n.n with
  100^2 and 600^2.

Reading of the printed A_G^3: the degree-8 polynomial term enters with a MINUS sign.  With the
printed plus sign the expansion error at |n| = 40..80 is twice that of A_G^2 and decays like
|n|^-5; with the minus sign it decays like |n|^-7 as the paper's O(|n|^{-2q-1}) statement
requires.  ``tests/test_oracle_lgf.py`` re-derives this from the quadrature below.

Quadrature: exp-sinh (double exponential) substitution t = exp(pi/2 sinh u) on a uniform
u-grid (Takahasi & Mori 1974), which handles the algebraic t^{-3/2} tail.  ive comes from
scipy.special for x < 1e7 (the AMOS routines return NaN far above that) and from the Hankel
asymptotic series (Abramowitz & Stegun 9.7.1) above it.
"""
from __future__ import annotations

import functools

import numpy as np
from scipy import special

TABLE_R2 = 100 * 100      # |n| <= 100: quadrature table
ASYM3_R2 = 600 * 600      # 100 < |n| <= 600: A_G^3; beyond: A_G^2
KMAX = 100                # largest |n_i| held by the table

_HANKEL_X = 1.0e7


def ive_hankel(k: np.ndarray, x: np.ndarray, terms: int = 8) -> np.ndarray:
    """exp(-x) I_k(x) for large x by the Hankel series (A&S 9.7.1):
    (2 pi x)^{-1/2} sum_j (-1)^j a_j(k) / x^j with a_j = prod_{i<=j} (4k^2 - (2i-1)^2) / (j! 8^j)."""
    k = np.asarray(k, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    mu = 4.0 * k * k
    term = np.ones(np.broadcast(k, x).shape)
    total = term.copy()
    for j in range(1, terms + 1):
        term = -term * (mu - (2 * j - 1) ** 2) / (j * 8.0 * x)
        total = total + term
    return total / np.sqrt(2.0 * np.pi * x)


def ive_table(kmax: int, x: np.ndarray) -> np.ndarray:
    """ive(k, x) for k = 0..kmax at every x: array [len(x), kmax+1]."""
    x = np.asarray(x, dtype=np.float64)
    k = np.arange(kmax + 1, dtype=np.float64)
    out = np.empty((x.size, kmax + 1))
    small = x < _HANKEL_X
    out[small] = special.ive(k[None, :], x[small, None])
    out[~small] = ive_hankel(k[None, :], x[~small, None])
    return out


@functools.lru_cache(maxsize=4)
def exp_sinh_rule(h: float = 1.0 / 256, umin: float = -4.6, umax: float = 5.3):
    """Nodes t_j and weights w_j of int_0^inf F(t) dt ~ sum_j w_j F(t_j), t = exp(pi/2 sinh u)."""
    u = np.arange(umin, umax + 0.5 * h, h)
    t = np.exp(0.5 * np.pi * np.sinh(u))
    w = h * 0.5 * np.pi * np.cosh(u) * t
    return t, w


def bessel_integral(triples: np.ndarray, h: float = 1.0 / 256) -> np.ndarray:
    """G(n) by eq. GL_B for integer triples (any sign/order), evaluated by quadrature."""
    n = np.abs(np.asarray(triples, dtype=np.int64)).reshape(-1, 3)
    kmax = int(n.max()) if n.size else 0
    t, w = exp_sinh_rule(h)
    T = ive_table(kmax, 2.0 * t)                     # [nodes, k]
    out = np.empty(len(n))
    # group by the first two orders so the last one is a matrix-vector product
    order = np.lexsort((n[:, 2], n[:, 1], n[:, 0]))
    ns = n[order]
    keys, starts = np.unique(ns[:, :2], axis=0, return_index=True)
    bounds = list(starts) + [len(ns)]
    res = np.empty(len(ns))
    for (a, b), s, e in zip(keys, bounds[:-1], bounds[1:]):
        v = w * T[:, a] * T[:, b]
        res[s:e] = -(v @ T[:, ns[s:e, 2]])
    out[order] = res
    return out


def sorted_triples(r2max: int = TABLE_R2) -> np.ndarray:
    """All a >= b >= c >= 0 with a^2 + b^2 + c^2 <= r2max (the distinct table entries)."""
    kmax = int(np.floor(np.sqrt(r2max)))
    a, b, c = np.meshgrid(np.arange(kmax + 1), np.arange(kmax + 1), np.arange(kmax + 1),
                          indexing="ij")
    m = (a >= b) & (b >= c) & (a * a + b * b + c * c <= r2max)
    return np.stack([a[m], b[m], c[m]], axis=1)


@functools.lru_cache(maxsize=1)
def table() -> np.ndarray:
    """Dense cube tab[a, b, c] of G for sorted a >= b >= c, a^2+b^2+c^2 <= 100^2 (NaN elsewhere)."""
    tri = sorted_triples(TABLE_R2)
    vals = bessel_integral(tri)
    tab = np.full((KMAX + 1, KMAX + 1, KMAX + 1), np.nan)
    tab[tri[:, 0], tri[:, 1], tri[:, 2]] = vals
    tab.setflags(write=False)
    return tab


def asym2(x: np.ndarray) -> np.ndarray:
    """Two-term far-field expansion A_G^2 (Sec. 2)."""
    x = np.asarray(x, dtype=np.float64)
    x1, x2, x3 = x[..., 0], x[..., 1], x[..., 2]
    r2 = x1 * x1 + x2 * x2 + x3 * x3
    r = np.sqrt(r2)
    quart = x1**4 + x2**4 + x3**4 - 3.0 * (x1**2 * x2**2 + x1**2 * x3**2 + x2**2 * x3**2)
    return -1.0 / (4.0 * np.pi * r) - quart / (16.0 * np.pi * r**7)


def octic(x: np.ndarray) -> np.ndarray:
    """The degree-8 polynomial of A_G^3 with the paper's coefficients -228, 621, -244, 23."""
    x = np.asarray(x, dtype=np.float64)
    a, b, c = x[..., 0] ** 2, x[..., 1] ** 2, x[..., 2] ** 2
    return (-228.0 * (b * c * a * a + b * c * c * a + b * b * c * a)
            + 621.0 * (a * a * b * b + c * c * b * b + a * a * c * c)
            - 244.0 * (b * a**3 + c * a**3 + b**3 * a + c**3 * a + b * c**3 + b**3 * c)
            + 23.0 * (a**4 + b**4 + c**4))


def asym3(x: np.ndarray, sign: float = -1.0) -> np.ndarray:
    """Three-term expansion A_G^3 = A_G^2 + sign * octic / (128 pi |x|^13); sign -1 is the
    reading adopted here (the printed +1 is kept selectable for the regression test)."""
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt((x * x).sum(axis=-1))
    return asym2(x) + sign * octic(x) / (128.0 * np.pi * r**13)


def lgf(n: np.ndarray) -> np.ndarray:
    """G(n) for integer vectors n (shape [..., 3]) with the paper's evaluation policy."""
    n = np.asarray(n, dtype=np.int64)
    shape = n.shape[:-1]
    n = n.reshape(-1, 3)
    r2 = (n * n).sum(axis=1)
    out = np.empty(len(n))
    near = r2 <= TABLE_R2
    mid = (~near) & (r2 <= ASYM3_R2)
    far = r2 > ASYM3_R2
    if near.any():
        s = -np.sort(-np.abs(n[near]), axis=1)       # descending |n_i|
        out[near] = table()[s[:, 0], s[:, 1], s[:, 2]]
    if mid.any():
        out[mid] = asym3(n[mid])
    if far.any():
        out[far] = asym2(n[far])
    return out.reshape(shape)


def watson_g0() -> float:
    """Closed form of G(0) from Watson's integral (Glasser & Zucker 1977, cited in Sec. 2):
    G(0) = -(1/6) (sqrt(6) / (32 pi^3)) Gamma(1/24) Gamma(5/24) Gamma(7/24) Gamma(11/24)."""
    g = special.gamma
    return -(np.sqrt(6.0) / (32.0 * np.pi**3)) * g(1 / 24) * g(5 / 24) * g(7 / 24) * g(11 / 24) / 6.0
