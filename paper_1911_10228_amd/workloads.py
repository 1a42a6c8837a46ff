"""Seeded synthetic workloads shaped like the paper's test problems.

This module holds no arithmetic of the solver: it only lays out blocks and evaluates analytic
source fields at cell centres.  It is the one module that both the HIP path's tests/benchmarks
and the FP64 oracle's tests draw their inputs from.

Geometry: base-lattice cell n has its centre at position n (base spacing 1).  A level-l cell
with level index m covers [m h_l - 1/2, (m+1) h_l - 1/2) with h_l = 2^-l, so its centre is at
(m + 1/2) h_l - 1/2.  Block b at level l holds level indices b n_b + (0..n_b-1) per dimension.
Arrays of cell values are [block, z, y, x] (x fastest).

Workloads (the paper's own test problem is a set of vortex rings in the unit cube whose
streamfunction has an analytic Laplacian; there is no public dataset):

* ``uniform_gaussian``   - 2x2x2 blocks of 8^3, one isotropic Gaussian (sigma 2) at the centre;
* ``uniform_mixture``    - 8x8x8 blocks of 16^3, 16 Gaussians (centres uniform in the inner
                           half, widths U[1.5, 4], amplitudes N(0, 1));
* ``torus``              - 8^3 base blocks of 16^3 plus two refinement levels chosen by the
                           refinement criterion (eq. ref_crit, alpha = 1/32) around a
                           Gaussian-core torus (major radius L/4, core 0.03 L, random tilt);
* ``batch``              - 64 independent layouts, block counts log-uniform in [8, 512],
                           n_b in {8, 16}, 0..2 refinement levels, Gaussian mixtures;
* ``arrivals``           - Poisson arrival times and sizes for the serving stream;
* ``request_pool``       - layouts of log-uniform size (4096 .. 16.7M base unknowns, n_b in
                           {8, 16}, 1..3 levels) that serving requests draw from.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Layout:
    blocks: np.ndarray          # [n, 3] int32 block coordinates (bx, by, bz) at their level
    levels: np.ndarray          # [n] int32 refinement level, 0 = coarsest
    n_b: int                    # cells per block side
    f: np.ndarray               # [n, n_b, n_b, n_b] float64 source
    interp_order: int
    name: str = ""
    exact: np.ndarray | None = None   # analytic solution at the cells, when one is known
    meta: dict = field(default_factory=dict)

    @property
    def unknowns(self) -> int:
        return int(len(self.blocks)) * self.n_b ** 3


def cell_centres(blocks: np.ndarray, levels: np.ndarray, n_b: int) -> np.ndarray:
    """Positions (x, y, z) in base units of every cell, shape [n, n_b, n_b, n_b, 3]."""
    blocks = np.asarray(blocks, dtype=np.float64).reshape(-1, 3)
    h = 2.0 ** (-np.asarray(levels, dtype=np.float64).reshape(-1))
    i = np.arange(n_b, dtype=np.float64)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    loc = np.stack([x, y, z], axis=-1)                                   # [n_b]^3 x 3
    m = blocks[:, None, None, None, :] * n_b + loc[None]
    return (m + 0.5) * h[:, None, None, None, None] - 0.5


def gaussian_mixture(pos: np.ndarray, centres, sigmas, amps) -> np.ndarray:
    out = np.zeros(pos.shape[:-1])
    for c, s, a in zip(centres, sigmas, amps):
        r2 = ((pos - np.asarray(c)) ** 2).sum(axis=-1)
        out += a * np.exp(-r2 / (2.0 * s * s))
    return out


class Mixture:
    """Sum of isotropic Gaussians a exp(-|p - c|^2 / (2 s^2)) evaluated block by block from its
    separable 1-D factors; a Gaussian's contribution to a block is dropped where it stays below
    1e-30 |a| over the whole block."""

    def __init__(self, centres, sigmas, amps):
        self.centres = np.asarray(centres, np.float64).reshape(-1, 3)
        self.sigmas = np.asarray(sigmas, np.float64).reshape(-1)
        self.amps = np.asarray(amps, np.float64).reshape(-1)

    def __call__(self, blocks, levels, n_b):
        blocks = np.asarray(blocks, np.float64).reshape(-1, 3)
        h = 2.0 ** (-np.asarray(levels, np.float64).reshape(-1))
        j = np.arange(n_b, dtype=np.float64)
        # positions along each axis: [n, 3, n_b]
        pos = ((blocks[:, :, None] * n_b + j[None, None, :]) + 0.5) * h[:, None, None] - 0.5
        out = np.zeros((len(blocks), n_b, n_b, n_b))
        for c, sg, a in zip(self.centres, self.sigmas, self.amps):
            e = np.exp(-((pos - c[None, :, None]) ** 2) / (2.0 * sg * sg))     # [n, 3, n_b]
            m = e.max(axis=2)
            keep = np.nonzero(m[:, 0] * m[:, 1] * m[:, 2] >= 1e-30)[0]
            if len(keep) == 0:
                continue
            ek = e[keep]
            out[keep] += a * (ek[:, 2, :, None, None] * ek[:, 1, None, :, None]) * ek[:, 0, None, None, :]
        return out


def box_blocks(nx: int, ny: int, nz: int, origin=(0, 0, 0)) -> np.ndarray:
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    b = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1) + np.asarray(origin)
    return b.astype(np.int32)


def uniform_gaussian() -> Layout:
    """2x2x2 blocks of 8^3 (4096 unknowns), isotropic Gaussian of sigma 2 cells at the centre."""
    n_b = 8
    blocks = box_blocks(2, 2, 2)
    levels = np.zeros(len(blocks), np.int32)
    pos = cell_centres(blocks, levels, n_b)
    f = gaussian_mixture(pos, [(7.5, 7.5, 7.5)], [2.0], [1.0])
    return Layout(blocks, levels, n_b, f, 4, "uniform 2^3 blocks of 8^3, Gaussian")


def uniform_mixture(nblk: int = 8, n_b: int = 16, n_gauss: int = 16, seed: int = 2,
                    interp_order: int = 8) -> Layout:
    """nblk^3 blocks of n_b^3; Gaussians with centres uniform in the inner half of the domain."""
    rng = np.random.default_rng(seed)
    L = nblk * n_b
    blocks = box_blocks(nblk, nblk, nblk)
    levels = np.zeros(len(blocks), np.int32)
    centres = rng.uniform(L / 4, 3 * L / 4, size=(n_gauss, 3))
    sigmas = rng.uniform(1.5, 4.0, size=n_gauss)
    amps = rng.normal(size=n_gauss)
    f = Mixture(centres, sigmas, amps)(blocks, levels, n_b)
    return Layout(blocks, levels, n_b, f, interp_order,
                  f"uniform {nblk}^3 blocks of {n_b}^3, {n_gauss} Gaussians",
                  meta=dict(centres=centres, sigmas=sigmas, amps=amps))


def refine_by_criterion(base_blocks: np.ndarray, n_b: int, n_levels: int, source,
                        alpha: float = 1.0 / 32) -> tuple[np.ndarray, np.ndarray]:
    """Refinement criterion of eq. ref_crit, read as: a level-l block is refined (all 8
    children created) iff max over its cells of |source| exceeds alpha^(L_R-1-l) times the
    maximum of |source| over all level-l cells, with L_R = n_levels.  ``source(blocks, levels,
    n_b)`` returns the cell values [n, n_b, n_b, n_b]."""
    blocks = [np.asarray(base_blocks, np.int64)]
    for l in range(n_levels - 1):
        cur = blocks[l]
        vals = np.abs(source(cur, np.full(len(cur), l), n_b))
        bmax = vals.reshape(len(cur), -1).max(axis=1)
        thr = alpha ** (n_levels - 1 - l) * bmax.max()
        ref = cur[bmax > thr]
        kids = (2 * ref[:, None, :] + np.array(list(np.ndindex(2, 2, 2)))[None]).reshape(-1, 3)
        blocks.append(kids)
    allb = np.concatenate(blocks).astype(np.int32)
    levs = np.concatenate([np.full(len(b), l, np.int32) for l, b in enumerate(blocks)])
    return allb, levs


def torus_source(pos, centre, axis, R, sigma):
    """Gaussian-core torus exp(-d^2 / 2 sigma^2), d = distance to the ring circle."""
    q = pos - np.asarray(centre)
    zc = q @ np.asarray(axis)
    rho_v = q - zc[..., None] * np.asarray(axis)
    rho = np.sqrt((rho_v ** 2).sum(axis=-1))
    d2 = (rho - R) ** 2 + zc ** 2
    return np.exp(-d2 / (2.0 * sigma * sigma)), rho, d2


def torus_laplacian(pos, centre, axis, R, sigma):
    """Analytic Laplacian of the Gaussian-core torus (cylindrical coordinates about the axis)."""
    u, rho, d2 = torus_source(pos, centre, axis, R, sigma)
    rho = np.maximum(rho, 1e-300)
    s2 = sigma * sigma
    return u * (d2 / (s2 * s2) - 2.0 / s2 - (rho - R) / (s2 * rho))


def torus(seed: int = 3, n_b: int = 16, nblk: int = 8, n_levels: int = 3,
          interp_order: int = 6, manufactured: bool = False, alpha: float = 1.0 / 32) -> Layout:
    """Base nblk^3 blocks, refinement around a tilted Gaussian-core torus (R = L/4, core 0.03 L).
    With ``manufactured`` the source is the torus' analytic Laplacian and ``exact`` holds the
    torus itself (a solution of the Poisson problem with that source)."""
    rng = np.random.default_rng(seed)
    L = nblk * n_b
    v = rng.normal(size=3)
    axis = v / np.linalg.norm(v)
    centre = np.full(3, L / 2 - 0.5)
    R, sigma = 0.25 * L, 0.03 * L
    src = lambda b, lv, nb: torus_source(cell_centres(b, lv, nb), centre, axis, R, sigma)[0]
    blocks, levels = refine_by_criterion(box_blocks(nblk, nblk, nblk), n_b, n_levels, src, alpha)
    pos = cell_centres(blocks, levels, n_b)
    if manufactured:
        f = torus_laplacian(pos, centre, axis, R, sigma)
        exact = torus_source(pos, centre, axis, R, sigma)[0]
    else:
        f = torus_source(pos, centre, axis, R, sigma)[0]
        exact = None
    return Layout(blocks, levels, n_b, f, interp_order,
                  f"torus {nblk}^3 base blocks of {n_b}^3, {n_levels} levels", exact,
                  meta=dict(axis=axis, centre=centre, R=R, sigma=sigma))


def vortex_ring_field(pos, R: float, c1: float, c2: float):
    """The paper's manufactured test field (Sec. 3, Convergence subsection, eqs. streamfunc and
    streamfunc_f): a vortex ring of radius R about the z axis whose streamfunction is
    f(t) e_theta, t = d / R, d the
    distance to the ring's core circle, f(t) = c1 exp(-c2 / (1 - t^2)) for |t| < 1 (0 beyond).
    Returns the Cartesian components psi_x = -f y / rho, psi_y = f x / rho and their Laplacians
    (the sources of the two scalar Poisson problems): for g(rho, z) sin(theta) the Laplacian is
    (g_rr + g_zz + g_r / rho - g / rho^2) sin(theta), and g_rr + g_zz = f'' / R^2 + f' / (R d)
    because g depends on d alone.  pos: physical positions [..., 3] relative to the ring centre."""
    x, y, z = pos[..., 0], pos[..., 1], pos[..., 2]
    rho = np.sqrt(x * x + y * y)
    d = np.sqrt((rho - R) ** 2 + z * z)
    inside = d < R
    t = np.where(inside, d / R, 0.0)
    om = np.where(inside, 1.0 - t * t, 1.0)
    f = np.where(inside, c1 * np.exp(-c2 / om), 0.0)
    fp_t = -2.0 * c2 * f / om**2                        # f'(t) / t (finite on the core circle)
    fp = fp_t * t                                       # f'(t)
    fpp = fp_t * (1.0 + 4.0 * t * t / om) + fp_t * t * t * (-2.0 * c2 / om**2)  # f''(t)
    lap_rz = (fpp + fp_t) / R**2                        # g_rr + g_zz
    g_r = fp / R * np.where(d > 0, (rho - R) / np.where(d > 0, d, 1.0), 0.0)
    part = lap_rz + g_r / rho - f / rho**2
    s, c = y / rho, x / rho
    return -f * s, f * c, -part * s, part * c


def vortex_ring(nblk: int = 4, n_b: int = 16, n_levels: int = 1, interp_order: int = 8,
                R: float = 0.125, c1: float = 1e3, c2: float = 10.0, alpha: float = 1.0 / 32) -> Layout:
    """The single vortex ring of the paper's convergence test (R = 0.125, c1 = 1e3, c2 = 10) in
    the cube [-1/4, 1/4]^3 (the ring's support), nblk^3 base blocks of n_b^3 (base spacing
    h = 1 / (2 nblk n_b)) refined around the ring by the refinement criterion.  ``f`` holds the
    x component's source in base-lattice units (h^2 times the physical Laplacian) and ``exact``
    the x component psi_x; ``meta`` holds the y component's source and solution."""
    h = 0.5 / (nblk * n_b)
    def phys(b, lv, nb):
        return (cell_centres(b, lv, nb) + 0.5) * h - 0.25
    def src(b, lv, nb):                 # the vorticity magnitude, as in the refinement criterion
        _, _, ox, oy = vortex_ring_field(phys(b, lv, nb), R, c1, c2)
        return np.sqrt(ox * ox + oy * oy)
    blocks, levels = refine_by_criterion(box_blocks(nblk, nblk, nblk), n_b, n_levels, src, alpha)
    px, py, ox, oy = vortex_ring_field(phys(blocks, levels, n_b), R, c1, c2)
    return Layout(blocks, levels, n_b, h * h * ox, interp_order,
                  f"vortex ring, {nblk}^3 base blocks of {n_b}^3, {n_levels} levels", px,
                  meta=dict(f_y=h * h * oy, exact_y=py, h=h))


def most_cubic_box(B: int) -> tuple[int, int, int]:
    """Smallest-surface a x b x c >= B with a >= b >= c (ties: smallest volume)."""
    best = None
    for c in range(1, int(round(B ** (1 / 3))) + 2):
        for b in range(c, int(math.isqrt(B)) + 2):
            a = max(b, -(-B // (b * c)))
            key = (a - c, a * b * c)
            if best is None or key < best[0]:
                best = (key, (a, b, c))
    return best[1]


def batch(seed: int = 4, count: int = 64, min_blocks: int = 8, max_blocks: int = 512,
          n_b_choices=(8, 16), max_levels: int = 3) -> list[Layout]:
    """Independent solves: base block counts log-uniform, n_b in {8, 16}, 1..3 refinement
    levels (0..2 refinements) by the refinement criterion, Gaussian-mixture sources."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n_b = int(rng.choice(n_b_choices))
        B = int(round(math.exp(rng.uniform(math.log(min_blocks), math.log(max_blocks)))))
        a, b, c = most_cubic_box(B)
        nl = int(rng.integers(1, max_levels + 1))
        ng = int(rng.integers(1, 17))
        ext = np.array([a, b, c]) * n_b
        centres = rng.uniform(ext / 4, 3 * ext / 4, size=(ng, 3)) - 0.5
        sigmas = rng.uniform(1.5, 4.0, size=ng)
        amps = rng.normal(size=ng)
        srcf = Mixture(centres, sigmas, amps)
        blocks, levels = refine_by_criterion(box_blocks(a, b, c), n_b, nl, srcf)
        f = srcf(blocks, levels, n_b)
        order = 8                      # the most nodes a block of 8 cells holds
        out.append(Layout(blocks, levels, n_b, f, order,
                          f"batch[{i}] {a}x{b}x{c} blocks of {n_b}^3, {nl} levels"))
    return out


def arrivals(seed: int = 5, count: int = 1000, rate_hz: float = 100.0,
             min_unknowns: int = 4096, max_unknowns: int = 16777216):
    """Poisson arrival times (s) and requested sizes (unknowns, log-uniform)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    sizes = np.exp(rng.uniform(math.log(min_unknowns), math.log(max_unknowns), size=count))
    return np.cumsum(gaps), sizes.astype(np.int64)


def sized_layout(unknowns: int, rng, max_levels: int = 3) -> Layout:
    """A layout of about ``unknowns`` base-level unknowns: n_b in {8, 16} (16 only from 16^3
    upward), the most cubic box of base blocks (at most 16^3 blocks of 16^3 or 32^3 of 8^3),
    1..max_levels refinement levels by the refinement criterion, a Gaussian-mixture source."""
    n_b = int(rng.choice((8, 16))) if unknowns >= 16 ** 3 else 8
    B = int(min(max(1, round(unknowns / n_b ** 3)), (4096 if n_b == 16 else 32768)))
    a, b, c = most_cubic_box(B)
    nl = int(rng.integers(1, max_levels + 1))
    ng = int(rng.integers(1, 17))
    ext = np.array([a, b, c]) * n_b
    centres = rng.uniform(ext / 4, 3 * ext / 4, size=(ng, 3)) - 0.5
    sigmas = rng.uniform(1.5, 4.0, size=ng)
    amps = rng.normal(size=ng)
    srcf = Mixture(centres, sigmas, amps)
    blocks, levels = refine_by_criterion(box_blocks(a, b, c), n_b, nl, srcf)
    f = srcf(blocks, levels, n_b)
    return Layout(blocks, levels, n_b, f, 8, f"{a}x{b}x{c} blocks of {n_b}^3, {nl} levels")


def request_pool(seed: int = 5, count: int = 24, min_unknowns: int = 4096,
                 max_unknowns: int = 16777216) -> list[Layout]:
    """The distinct layouts a serving stream draws from (sizes log-uniform): a service keeps
    one plan per layout resident and requests name a layout and bring a source."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(min_unknowns), math.log(max_unknowns), size=count))
    return [sized_layout(int(u), rng) for u in sizes]
