"""Block-refined FLGF (Sec. 3, Algorithm 2), FP64 (test infrastructure only).

Parity note: the multi-resolution result has no plain closed form; this module takes
Algorithm 2's steps in order and is pinned by invariants only (consistency of the 7-point
operator with the computed inverse on interior cells, second-order convergence against a
manufactured solution, reduction to the uniform FLGF for one level).

Layout: blocks [n, 3] with refinement levels [n] (0 = coarsest).  Level l has spacing
h_l = 2^-l base cells; cell x of block b at level l is the lattice point b n_b + x of that level.
A level-(l+1) block's parent is floor(b / 2) at level l.  A block with children (all eight must
exist) is non-leaf.

Steps and the readings taken where the paper is silent or garbled:

1. regularization: the source of a non-leaf block is the average of the 2x2x2 child cells
   (coarsening C, Sec. 3 last paragraph), bottom-up, on the given source before any correction;
2. per level l = 0 .. L_R-1, in order (the correction depends on the coarser levels):
   a. Jw = J^{l-1} w^{l-1}: quadratic (3-node) Lagrange interpolation of the parent's leaf-only
      field onto every level-l block, one-sided inside the parent at its faces (reading of
      "second-order Lagrangian polynomials ... unbiased interpolation for each octant");
   b. source correction g = f^l - L^l(Jw) on every level-l block (reading of the garbled
      operand of step 2b: the Laplacian acts on the interpolated FIELD, as in eq. amr_formular,
      not on the source).  L^l = h_l^-2 (6 neighbours - 6 centre).  A neighbour value in another
      level-l block is that block's Jw; a neighbour outside all level-l blocks takes the ghost
      value of the block's own parent polynomial extended one child cell outward;
   c. convolution (eq. amr_convs): the total field T = h_l^2 G^l[g over all level-l blocks]
      (leaf targets) and the leaf-only field A = h_l^2 G^l[g over leaf blocks] (non-leaf
      targets), each by the FLGF of ``fmm`` on the octree of all level-l blocks - the paper's
      "FMM twice and subtract" gives the same A by linearity;
   d. accumulation: u^l = Jw + T on every block (non-leaf blocks report the level's total
      field), w^l = Jw + A on non-leaf blocks (passed to level l+1).
"""
from __future__ import annotations

import numpy as np

from . import fmm, interp


def validate(blocks, levels):
    """Raise ValueError for duplicates, orphans, or non-leaf blocks with fewer than 8 children."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    levels = np.asarray(levels, dtype=np.int64).reshape(-1)
    seen = set()
    for b, l in zip(blocks, levels):
        key = (int(l),) + tuple(int(v) for v in b)
        if key in seen:
            raise ValueError(f"duplicate block {key}")
        seen.add(key)
    for b, l in zip(blocks, levels):
        if l > 0:
            p = (int(l) - 1,) + tuple(int(v) for v in np.floor_divide(b, 2))
            if p not in seen:
                raise ValueError(f"block {(int(l),) + tuple(b)} has no parent")
    for b, l in zip(blocks, levels):
        kids = [(int(l) + 1,) + tuple(int(v) for v in 2 * b + np.array(c))
                for c in np.ndindex(2, 2, 2)]
        have = sum(k in seen for k in kids)
        if 0 < have < 8:
            raise ValueError(f"block {(int(l),) + tuple(b)} has {have} of 8 children")


def _octants(n_b):
    """Child octant c=(cx,cy,cz) -> slice of the parent's [z, y, x] cells it covers."""
    h = n_b // 2
    return {c: (slice(c[2] * h, (c[2] + 1) * h), slice(c[1] * h, (c[1] + 1) * h),
                slice(c[0] * h, (c[0] + 1) * h)) for c in np.ndindex(2, 2, 2)}


def coarsen(children: dict, n_b: int) -> np.ndarray:
    """Parent cells = mean of the 2x2x2 child cells (children keyed by octant (cx,cy,cz))."""
    out = np.zeros((n_b, n_b, n_b))
    for c, sl in _octants(n_b).items():
        ch = children[c]
        out[sl] = ch.reshape(n_b // 2, 2, n_b // 2, 2, n_b // 2, 2).mean(axis=(1, 3, 5))
    return out


def refine_ext(w_parent: np.ndarray, octant) -> np.ndarray:
    """Quadratic interpolation of a parent field onto child block ``octant`` extended by one
    child cell on every side: array [(n_b+2)]^3 whose interior is the child block."""
    n_b = w_parent.shape[0]
    W = interp.child_matrix(n_b, 3, rows=range(-1, 2 * n_b + 1))    # row r <-> child row r-1
    cx, cy, cz = (int(v) for v in octant)
    rows = lambda c: W[c * n_b:c * n_b + n_b + 2]
    return interp.apply3(rows(cz), rows(cy), rows(cx), w_parent)


def _face_neighbours(coords: dict, b):
    """Index of the same-level block across each face (-x,+x,-y,+y,-z,+z) or None."""
    b = tuple(int(v) for v in b)
    out = []
    for axis in range(3):
        for sgn in (-1, 1):
            nb = list(b)
            nb[axis] += sgn
            out.append(coords.get(tuple(nb)))
    return out


def _laplace_with_halo(ext: np.ndarray, own: np.ndarray, nbrs, fields) -> np.ndarray:
    """7-point operator (unscaled) on a block whose one-cell halo comes from the neighbour blocks'
    fields where they exist and from ``ext`` (ghost values) elsewhere."""
    E = ext.copy()
    E[1:-1, 1:-1, 1:-1] = own
    # faces, order (-x,+x,-y,+y,-z,+z); arrays are [z, y, x]
    sl = {0: (slice(1, -1), slice(1, -1), 0), 1: (slice(1, -1), slice(1, -1), -1),
          2: (slice(1, -1), 0, slice(1, -1)), 3: (slice(1, -1), -1, slice(1, -1)),
          4: (0, slice(1, -1), slice(1, -1)), 5: (-1, slice(1, -1), slice(1, -1))}
    src = {0: (slice(None), slice(None), -1), 1: (slice(None), slice(None), 0),
           2: (slice(None), -1, slice(None)), 3: (slice(None), 0, slice(None)),
           4: (-1, slice(None), slice(None)), 5: (0, slice(None), slice(None))}
    for face, j in enumerate(nbrs):
        if j is not None:
            E[sl[face]] = fields[j][src[face]]
    c = E[1:-1, 1:-1, 1:-1]
    return (E[2:, 1:-1, 1:-1] + E[:-2, 1:-1, 1:-1] + E[1:-1, 2:, 1:-1] + E[1:-1, :-2, 1:-1]
            + E[1:-1, 1:-1, 2:] + E[1:-1, 1:-1, :-2] - 6.0 * c)


def solve(blocks, levels, f, n_b: int, n_i: int, correction: bool = True, return_parts=False,
          dtype=np.float64):
    """Algorithm 2.  f: [n, n_b, n_b, n_b] (values on non-leaf blocks are ignored).
    Returns u: [n, n_b, n_b, n_b] (each block's level field).  ``dtype`` is passed to the
    convolutions (``fmm.flgf``); the other steps run in FP64."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    levels = np.asarray(levels, dtype=np.int64).reshape(-1)
    f = np.asarray(f, dtype=np.float64).reshape(-1, n_b, n_b, n_b)
    validate(blocks, levels)
    LR = int(levels.max()) + 1
    idx = [np.nonzero(levels == l)[0] for l in range(LR)]
    coords = [{tuple(int(v) for v in blocks[i]): i for i in idx[l]} for l in range(LR)]
    leaf = np.ones(len(blocks), bool)
    for l in range(LR - 1):
        for i in idx[l]:
            if tuple(int(v) for v in 2 * blocks[i]) in coords[l + 1]:
                leaf[i] = False

    # 1. regularization, bottom-up
    feff = f.copy()
    for l in range(LR - 2, -1, -1):
        for i in idx[l]:
            if not leaf[i]:
                kids = {c: feff[coords[l + 1][tuple(int(v) for v in 2 * blocks[i] + np.array(c))]]
                        for c in np.ndindex(2, 2, 2)}
                feff[i] = coarsen(kids, n_b)

    u = np.zeros_like(f)
    w = np.zeros_like(f)
    g_all = np.zeros_like(f)
    Jw_all = np.zeros_like(f)
    for l in range(LR):
        h = 2.0 ** (-l)
        ids = idx[l]
        Jw = np.zeros((len(ids), n_b, n_b, n_b))
        g = feff[ids].copy()
        if l > 0:
            ext = []
            for a, i in enumerate(ids):
                p = coords[l - 1][tuple(int(v) for v in np.floor_divide(blocks[i], 2))]
                e = refine_ext(w[p], blocks[i] - 2 * np.floor_divide(blocks[i], 2))
                ext.append(e)
                Jw[a] = e[1:-1, 1:-1, 1:-1]
            if correction:
                local = {i: a for a, i in enumerate(ids)}
                for a, i in enumerate(ids):
                    nbrs = [None if j is None else local[j] for j in _face_neighbours(coords[l], blocks[i])]
                    g[a] -= _laplace_with_halo(ext[a], Jw[a], nbrs, Jw) / (h * h)
        lb = blocks[ids]
        lleaf = leaf[ids]
        T = fmm.flgf(lb, g, n_b, n_i, scale=h * h, dtype=dtype)
        u[ids] = Jw + T
        if (~lleaf).any():
            A = fmm.flgf(lb, g, n_b, n_i, sources=lleaf, targets=~lleaf, scale=h * h, dtype=dtype)
            w[ids[~lleaf]] = (Jw + A)[~lleaf]
        g_all[ids] = g
        Jw_all[ids] = Jw
    if return_parts:
        return u, dict(feff=feff, g=g_all, Jw=Jw_all, w=w, leaf=leaf)
    return u


def level_residual(blocks, levels, u, f, n_b: int):
    """max |L^l u - f^l| over leaf cells whose six neighbours all lie in level-l blocks, per
    level, with f^l the coarsened source (the consistency check of Sec. 3, Convergence)."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    levels = np.asarray(levels, dtype=np.int64).reshape(-1)
    _, parts = solve_parts_free(blocks, levels, f, n_b)
    feff, leaf = parts["feff"], parts["leaf"]
    out = []
    for l in range(int(levels.max()) + 1):
        out.append(_masked_residual(blocks, levels, u, feff, leaf, n_b, l))
    return out


def solve_parts_free(blocks, levels, f, n_b):
    """Coarsened source and leaf flags without running any convolution."""
    levels = np.asarray(levels, dtype=np.int64).reshape(-1)
    LR = int(levels.max()) + 1
    idx = [np.nonzero(levels == l)[0] for l in range(LR)]
    coords = [{tuple(int(v) for v in blocks[i]): i for i in idx[l]} for l in range(LR)]
    f = np.asarray(f, dtype=np.float64).reshape(-1, n_b, n_b, n_b)
    leaf = np.ones(len(blocks), bool)
    for l in range(LR - 1):
        for i in idx[l]:
            if tuple(int(v) for v in 2 * blocks[i]) in coords[l + 1]:
                leaf[i] = False
    feff = f.copy()
    for l in range(LR - 2, -1, -1):
        for i in idx[l]:
            if not leaf[i]:
                kids = {c: feff[coords[l + 1][tuple(int(v) for v in 2 * blocks[i] + np.array(c))]]
                        for c in np.ndindex(2, 2, 2)}
                feff[i] = coarsen(kids, n_b)
    return None, dict(feff=feff, leaf=leaf)


def residual_mask(blocks, levels, n_b: int):
    """Boolean [n, n_b, n_b, n_b]: leaf cells whose 6 neighbours all lie in same-level blocks."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    levels = np.asarray(levels, dtype=np.int64).reshape(-1)
    _, parts = solve_parts_free(blocks, levels, np.zeros((len(blocks), n_b, n_b, n_b)), n_b)
    leaf = parts["leaf"]
    LR = int(levels.max()) + 1
    mask = np.zeros((len(blocks), n_b, n_b, n_b), bool)
    for l in range(LR):
        ids = np.nonzero(levels == l)[0]
        coords = {tuple(int(v) for v in blocks[i]): i for i in ids}
        for i in ids:
            if not leaf[i]:
                continue
            m = np.ones((n_b, n_b, n_b), bool)
            nb = _face_neighbours(coords, blocks[i])
            if nb[0] is None: m[:, :, 0] = False
            if nb[1] is None: m[:, :, -1] = False
            if nb[2] is None: m[:, 0, :] = False
            if nb[3] is None: m[:, -1, :] = False
            if nb[4] is None: m[0, :, :] = False
            if nb[5] is None: m[-1, :, :] = False
            mask[i] = m
    return mask


def apply_laplace(blocks, levels, u, n_b: int):
    """L^l u on every cell of every block, using same-level neighbour blocks (0 where absent;
    such cells are outside ``residual_mask``)."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    levels = np.asarray(levels, dtype=np.int64).reshape(-1)
    out = np.zeros_like(u)
    for l in range(int(levels.max()) + 1):
        ids = np.nonzero(levels == l)[0]
        coords = {tuple(int(v) for v in blocks[i]): i for i in ids}
        h = 2.0 ** (-l)
        for i in ids:
            nbrs = _face_neighbours(coords, blocks[i])
            ext = np.zeros((n_b + 2,) * 3)
            out[i] = _laplace_with_halo(ext, u[i], nbrs, u) / (h * h)
    return out


def _masked_residual(blocks, levels, u, feff, leaf, n_b, l):
    mask = residual_mask(blocks, levels, n_b)
    Lu = apply_laplace(blocks, levels, u, n_b)
    sel = (np.asarray(levels) == l)[:, None, None, None] & mask
    if not sel.any():
        return 0.0
    return float(np.abs(Lu - feff)[sel].max())
