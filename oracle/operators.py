"""Forward operators on the block-refined mesh, FP64 (test infrastructure only).

The refined solve (Sec. 3) inverts the 7-point Laplacian of every level; applications also need
the gradient of the computed field, and the source correction is what makes each level's 7-point
operator consistent with the computed inverse.  Each operator acts on a block with its one-cell
halo: a neighbour cell in a same-level block is that block's value; at a level boundary (no
same-level block across the face of a level l >= 1 block) it is the ghost value of the block's
parent field, the parent's quadratic extended one child cell outward (``multires.refine_ext``,
the ghost the source correction takes; reading: the paper asks for operators consistent with
the computed inverse and names no boundary stencil).  The operators are evaluated on every leaf
cell of levels l >= 1 and on the leaf cells of level 0 whose neighbours lie in level-0 blocks
(the outer boundary of the coarsest level has nothing outside it); every other cell, and every
non-leaf block, is 0.  Level l has spacing h_l = 2^-l base cells; arrays are [block, z, y, x],
vector fields [component, block, ...].

- laplacian: h_l^-2 (sum of the six neighbours - 6 centre), the operator the solve inverts;
- gradient: central differences (u(x + e_a) - u(x - e_a)) / (2 h_l), components (x, y, z);
- curl of (u_x, u_y, u_z) from the same central differences.

Pinned by exactness on polynomials (central differences are exact for quadratics, the 7-point
Laplacian for cubics, and the parent's quadratic reproduces quadratics, so every evaluated cell,
interface cells included, is exact for quadratics), curl of a gradient = 0 where both are
defined, and L^l u = f where the solve makes the 7-point equation hold, for a corrected refined
solve u of f.
"""
from __future__ import annotations

import numpy as np

from . import multires

OPS = ("laplacian", "gradient", "curl")


def op_mask(blocks, levels, n_b: int) -> np.ndarray:
    """Boolean [n, n_b, n_b, n_b]: the cells the operators are evaluated on (module header)."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    levels = np.asarray(levels, dtype=np.int64).reshape(-1)
    mask = multires.residual_mask(blocks, levels, n_b)
    keys = {(int(l),) + tuple(int(v) for v in b) for b, l in zip(blocks, levels)}
    for i, (b, l) in enumerate(zip(blocks, levels)):
        leaf = (int(l) + 1,) + tuple(int(v) for v in 2 * b) not in keys
        if l > 0 and leaf:
            mask[i] = True
    return mask


def _halo(coords: dict, b, field: np.ndarray, i: int, n_b: int, ghost=None) -> np.ndarray:
    """Block i of ``field`` with its one-cell halo from the same-level blocks across its faces;
    where there is none, from ``ghost`` (the parent's extended quadratic, [(n_b+2)]^3), else 0
    (the halo's edges and corners are never used)."""
    E = np.zeros((n_b + 2,) * 3) if ghost is None else ghost.copy()
    E[1:-1, 1:-1, 1:-1] = field[i]
    nb = multires._face_neighbours(coords, b)       # (-x, +x, -y, +y, -z, +z)
    if nb[0] is not None: E[1:-1, 1:-1, 0] = field[nb[0]][:, :, -1]
    if nb[1] is not None: E[1:-1, 1:-1, -1] = field[nb[1]][:, :, 0]
    if nb[2] is not None: E[1:-1, 0, 1:-1] = field[nb[2]][:, -1, :]
    if nb[3] is not None: E[1:-1, -1, 1:-1] = field[nb[3]][:, 0, :]
    if nb[4] is not None: E[0, 1:-1, 1:-1] = field[nb[4]][-1, :, :]
    if nb[5] is not None: E[-1, 1:-1, 1:-1] = field[nb[5]][0, :, :]
    return E


def _diff(E: np.ndarray, axis: int, h: float) -> np.ndarray:
    """Central difference of a haloed block along axis 0 = x, 1 = y, 2 = z."""
    c = slice(1, -1)
    if axis == 0:
        return (E[c, c, 2:] - E[c, c, :-2]) / (2.0 * h)
    if axis == 1:
        return (E[c, 2:, c] - E[c, :-2, c]) / (2.0 * h)
    return (E[2:, c, c] - E[:-2, c, c]) / (2.0 * h)


def apply(blocks, levels, u, n_b: int, op: str) -> np.ndarray:
    """op(u): u [n, n_b, n_b, n_b] ([3, n, ...] for the curl); returns [n, ...] for the
    Laplacian and [3, n, ...] for the gradient and the curl."""
    if op not in OPS:
        raise ValueError(f"unknown operator {op!r}")
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    levels = np.asarray(levels, dtype=np.int64).reshape(-1)
    n = len(blocks)
    comps = [np.asarray(u[c], np.float64) for c in range(3)] if op == "curl" else [np.asarray(u, np.float64)]
    mask = op_mask(blocks, levels, n_b)
    out = np.zeros((1 if op == "laplacian" else 3, n, n_b, n_b, n_b))
    c = slice(1, -1)
    coords_of = []
    for l in range(int(levels.max()) + 1):
        ids = np.nonzero(levels == l)[0]
        coords_of.append({tuple(int(v) for v in blocks[i]): i for i in ids})
    for l in range(int(levels.max()) + 1):
        ids = np.nonzero(levels == l)[0]
        coords = coords_of[l]
        h = 2.0 ** (-l)
        for i in ids:
            if not mask[i].any():
                continue
            ghosts = [None] * len(comps)
            if l > 0:
                par = coords_of[l - 1][tuple(int(v) for v in np.floor_divide(blocks[i], 2))]
                octant = tuple(int(v) for v in blocks[i] - 2 * np.floor_divide(blocks[i], 2))
                ghosts = [multires.refine_ext(f[par], octant) for f in comps]
            E = [_halo(coords, blocks[i], f, i, n_b, g) for f, g in zip(comps, ghosts)]
            if op == "laplacian":
                e = E[0]
                vals = [(e[2:, c, c] + e[:-2, c, c] + e[c, 2:, c] + e[c, :-2, c] + e[c, c, 2:]
                         + e[c, c, :-2] - 6.0 * e[c, c, c]) / (h * h)]
            elif op == "gradient":
                vals = [_diff(E[0], a, h) for a in range(3)]
            else:
                def d(comp, a):
                    return _diff(E[comp], a, h)
                vals = [d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)]
            for k, v in enumerate(vals):
                out[k, i] = np.where(mask[i], v, 0.0)
    return out[0] if op == "laplacian" else out
