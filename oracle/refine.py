"""Refinement criterion and one adaptation step of a block layout (test infrastructure only).

Sec. 3 (Convergence subsection, eq. ref_crit): a block on level l is initialised or refined when
its vorticity exceeds alpha^(L_R - l) times the level's maximum, alpha = 1/32 unless stated.
Readings (the paper leaves them open):

* omega^l of a block is the largest |value| over its cells, omega^l_max the largest over all
  level-l cells of the layout;
* the exponent is L_R - 1 - l with L_R the number of refinement levels (so the finest level,
  l = L_R - 1, is never refined);
* a refined block gets all 8 children (every non-leaf block has 8, as Algorithm 2 needs);
* one adaptation step starts from a layout and the field on its cells: the base level stays; a
  level-(l+1) block of the new layout is a child of a level-l block flagged by the criterion;
  a block is flagged only if it is in the old layout (only there is its field known) and
  survives into the new one.  Repeating the step L_R - 1 times from the base layout, with the
  field evaluated on each new layout, builds the layout level by level.
* Order of the new layout: the base blocks in their old order, then level by level the 8
  children of each flagged block, in the new order of the flagged blocks, child offset
  (cx, cy, cz) with cz fastest.

Plain loops over blocks with a dictionary of (level, x, y, z); integer output.
"""
from __future__ import annotations

import numpy as np


def block_absmax(field: np.ndarray) -> np.ndarray:
    """omega per block: max over the block's cells of |value| (field [n, N_b, N_b, N_b])."""
    n = field.shape[0]
    return np.abs(field.reshape(n, -1)).max(axis=1)


def adapt(blocks: np.ndarray, levels: np.ndarray, field: np.ndarray, n_levels: int,
          alpha: float = 1.0 / 32) -> tuple[np.ndarray, np.ndarray]:
    """One adaptation step (see the module header).  Returns (blocks [m, 3], levels [m])."""
    blocks = np.asarray(blocks, np.int64).reshape(-1, 3)
    levels = np.asarray(levels, np.int64).reshape(-1)
    omega = block_absmax(np.asarray(field, np.float64))
    top = int(levels.max()) + 1
    # omega_max per level, then the threshold alpha^(L_R - 1 - l) omega_max (alpha^k by repeated
    # multiplication)
    thr = {}
    for l in range(top):
        sel = levels == l
        if not sel.any():
            continue
        a = 1.0
        for _ in range(n_levels - 1 - l):
            a *= alpha
        thr[l] = a * float(omega[sel].max())
    where = {(int(levels[i]), int(b[0]), int(b[1]), int(b[2])): i for i, b in enumerate(blocks)}

    def criterion(i):
        l = int(levels[i])
        return l < n_levels - 1 and omega[i] > thr[l]

    out_b, out_l = [], []
    current = [(int(b[0]), int(b[1]), int(b[2])) for b, l in zip(blocks, levels) if l == 0]
    l = 0
    while current:
        out_b.extend(current)
        out_l.extend([l] * len(current))
        nxt = []
        for c in current:
            i = where.get((l,) + c)          # None: a block new in this step (field unknown)
            if i is None or not criterion(i):
                continue
            for cx in (0, 1):
                for cy in (0, 1):
                    for cz in (0, 1):
                        nxt.append((2 * c[0] + cx, 2 * c[1] + cy, 2 * c[2] + cz))
        current = nxt
        l += 1
    return np.array(out_b, np.int32).reshape(-1, 3), np.array(out_l, np.int32)
