"""Lagrange interpolation J between octree levels and its adjoint R (test infrastructure only).

Sec. 2.1 (Algorithm 1, steps 1 and 3, and the paragraph after it): the interpolation J^l from a
parent block onto its children uses Lagrange polynomials on the uniform block grid with n_I
nodes per dimension; the regularization (anterpolation) R is its adjoint.  Sec. 3 (refinement
operators) reuses the same polynomials with n_I = 3 for the coarse-to-fine interpolation of
refined levels.

Geometry (cell-centred storage, Fig. mesh_1d): the 2 n_b child cells spanning a parent block sit
at parent-index coordinate x_j = j/2 - 1/4 (j = 0 .. 2 n_b - 1).  Child octant c in {0,1} of a
dimension holds rows j = c n_b .. c n_b + n_b - 1.

Stencil placement (the paper defers it to Liska & Colonius 2014; reading): an even number of
nodes sits symmetrically around the bracketing pair (floor x, floor x + 1); an odd number is
centred on the nearest node; the stencil is shifted inward to stay inside [0, n_b - 1], so it
is one-sided at the block faces.
"""
from __future__ import annotations

import numpy as np


def stencil(x: float, n_i: int, n_b: int) -> tuple[int, np.ndarray]:
    """First node index and the n_i Lagrange weights that interpolate to coordinate x."""
    if n_i % 2 == 0:
        lo = int(np.floor(x)) - n_i // 2 + 1
    else:
        lo = int(np.floor(x + 0.5)) - (n_i - 1) // 2
    lo = min(max(lo, 0), n_b - n_i)
    nodes = lo + np.arange(n_i, dtype=np.float64)
    w = np.ones(n_i)
    for j in range(n_i):
        for m in range(n_i):
            if m != j:
                w[j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return lo, w


def child_matrix(n_b: int, n_i: int, rows=None) -> np.ndarray:
    """Dense 1-D interpolation matrix W with W[j - rows[0], :] the weights for child row j.

    Default rows are 0 .. 2 n_b - 1; the refinement operator also evaluates row -1 and row 2 n_b
    (x = -3/4 and x = n_b - 1/4, one cell outside the parent) for ghost values."""
    if rows is None:
        rows = range(2 * n_b)
    rows = list(rows)
    W = np.zeros((len(rows), n_b))
    for r, j in enumerate(rows):
        lo, w = stencil(j / 2.0 - 0.25, n_i, n_b)
        W[r, lo:lo + n_i] = w
    return W


def apply3(Wz: np.ndarray, Wy: np.ndarray, Wx: np.ndarray, a: np.ndarray) -> np.ndarray:
    """(Wz (x) Wy (x) Wx) a for a block stored [z, y, x]."""
    return np.einsum("Zz,Yy,Xx,zyx->ZYX", Wz, Wy, Wx, a, optimize=True)


def interp_child(W: np.ndarray, octant, parent: np.ndarray) -> np.ndarray:
    """J_c: parent block -> child block c = (cx, cy, cz)."""
    n_b = parent.shape[0]
    cx, cy, cz = (int(v) for v in octant)
    return apply3(W[cz * n_b:(cz + 1) * n_b], W[cy * n_b:(cy + 1) * n_b],
                  W[cx * n_b:(cx + 1) * n_b], parent)


def anterp_child(W: np.ndarray, octant, child: np.ndarray) -> np.ndarray:
    """R_c = J_c^T: child block c -> its contribution to the parent block."""
    n_b = child.shape[0]
    cx, cy, cz = (int(v) for v in octant)
    return apply3(W[cz * n_b:(cz + 1) * n_b].T, W[cy * n_b:(cy + 1) * n_b].T,
                  W[cx * n_b:(cx + 1) * n_b].T, child)
