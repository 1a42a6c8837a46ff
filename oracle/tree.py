"""Octree of Cartesian blocks and its interaction lists (test infrastructure only).

Sec. 2.1: the tree nodes are Cartesian blocks of n_b^3 cells; the base level is the physical
block set, each coarser level holds the parents floor(b / 2) of the level below.  Reading of the
root: the tree stops at the first level whose nodes are all mutual neighbours (Chebyshev
distance <= 1), where no influence list can be non-empty any more; for blocks with non-negative
coordinates this differs from going up to a single root only by levels with empty lists, and it
stays finite for negative coordinates, where floor(-1/2) = -1 never merges with 0.
For a block B:

* near region N(B): B itself and its same-level neighbours (Chebyshev distance <= 1), used
  with the exact kernel at the base level only;
* influence list I(B): the children of the neighbours of B's parent that are not neighbours of
  B, i.e. same-level blocks B' with ||B' - B||_inf >= 2 and ||parent(B') - parent(B)||_inf <= 1
  (Fig. fmm_regions caption).

Reading: Algorithm 1's level-interaction step lists only I(B); the near field stated just before
it is added at the base level.  Lists are built here straight from those definitions by
comparing every pair of same-level nodes.
"""
from __future__ import annotations

import numpy as np


def parent_of(b: np.ndarray) -> np.ndarray:
    return np.floor_divide(b, 2)


def build_levels(blocks: np.ndarray) -> list[np.ndarray]:
    """levels[0] = base blocks (in the given order), levels[k+1] = sorted unique parents, up to
    the first level whose bounding box spans at most 2 nodes per dimension."""
    levels = [np.asarray(blocks, dtype=np.int64).reshape(-1, 3)]
    while (levels[-1].max(axis=0) - levels[-1].min(axis=0)).max() > 1:
        levels.append(np.unique(parent_of(levels[-1]), axis=0))
    return levels


def index_of(nodes: np.ndarray) -> dict:
    return {tuple(int(v) for v in b): i for i, b in enumerate(nodes)}


def interactions(nodes: np.ndarray, base: bool):
    """List of (target index, source index) pairs at one level: N(B) (base only) and I(B)."""
    nodes = np.asarray(nodes, dtype=np.int64)
    out = []
    par = parent_of(nodes)
    for t in range(len(nodes)):
        d = np.abs(nodes[t][None, :] - nodes).max(axis=1)
        dp = np.abs(par[t][None, :] - par).max(axis=1)
        far = (d >= 2) & (dp <= 1)
        sel = far | (d <= 1) if base else far
        for s in np.nonzero(sel)[0]:
            out.append((t, int(s)))
    return out
