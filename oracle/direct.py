"""The plain definition of the solution, u(n) = sum_m G(n - m) f(m) (eq. discretConv), FP64.

Test infrastructure only.  Two evaluations of the same sum:

* ``direct_sum``: brute force over every source cell, for all targets of tiny grids or for a
  sample of target cells of larger ones;
* ``direct_fft``: the full lattice convolution over the bounding box of the blocks as one
  zero-padded FFT (the kernel sampled on every offset of the doubled box), which is exact up to
  FFT rounding and has no far-field approximation at all.
"""
from __future__ import annotations

import numpy as np

from . import lgf


def cell_coords(blocks, n_b: int) -> np.ndarray:
    """Lattice index (x, y, z) of every cell, ordered [block, z, y, x]."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    i = np.arange(n_b)
    z, y, x = np.meshgrid(i, i, i, indexing="ij")
    loc = np.stack([x, y, z], axis=-1).reshape(-1, 3)
    return (blocks[:, None, :] * n_b + loc[None, :, :]).reshape(-1, 3)


def direct_sum(blocks, f, n_b: int, target_cells=None, chunk: int = 256) -> np.ndarray:
    """u at the given flat cell indices (default: all cells) by brute-force summation."""
    pos = cell_coords(blocks, n_b)
    fv = np.asarray(f, dtype=np.float64).reshape(-1)
    nz = fv != 0.0
    spos, sval = pos[nz], fv[nz]
    tgt = np.arange(len(pos)) if target_cells is None else np.asarray(target_cells)
    out = np.empty(len(tgt))
    for a in range(0, len(tgt), chunk):
        tp = pos[tgt[a:a + chunk]]
        G = lgf.lgf(tp[:, None, :] - spos[None, :, :])
        out[a:a + chunk] = G @ sval
    return out


def direct_fft(blocks, f, n_b: int) -> np.ndarray:
    """u on every cell of every block by one zero-padded FFT over the bounding box."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    f = np.asarray(f, dtype=np.float64).reshape(-1, n_b, n_b, n_b)
    lo = blocks.min(axis=0)
    ext = (blocks.max(axis=0) - lo + 1) * n_b          # box size per dim (x, y, z)
    box = np.zeros((ext[2], ext[1], ext[0]))
    for b, fb in zip(blocks - lo, f):
        box[b[2] * n_b:(b[2] + 1) * n_b, b[1] * n_b:(b[1] + 1) * n_b, b[0] * n_b:(b[0] + 1) * n_b] = fb
    M = 2 * ext
    rz = np.arange(-(ext[2] - 1), ext[2])
    ry = np.arange(-(ext[1] - 1), ext[1])
    rx = np.arange(-(ext[0] - 1), ext[0])
    Z, Y, X = np.meshgrid(rz, ry, rx, indexing="ij")
    K = np.zeros((M[2], M[1], M[0]))
    K[np.ix_(rz % M[2], ry % M[1], rx % M[0])] = lgf.lgf(np.stack([X, Y, Z], axis=-1))
    u = np.fft.irfftn(np.fft.rfftn(K) * np.fft.rfftn(box, s=K.shape, axes=(0, 1, 2)),
                     s=K.shape, axes=(0, 1, 2))
    u = u[:ext[2], :ext[1], :ext[0]]
    out = np.empty_like(f)
    for i, b in enumerate(blocks - lo):
        out[i] = u[b[2] * n_b:(b[2] + 1) * n_b, b[1] * n_b:(b[1] + 1) * n_b, b[0] * n_b:(b[0] + 1) * n_b]
    return out


def laplace7(u_box: np.ndarray) -> np.ndarray:
    """7-point Laplacian (sum of 6 neighbours - 6 u) on the interior of a [z, y, x] box."""
    c = u_box[1:-1, 1:-1, 1:-1]
    return (u_box[2:, 1:-1, 1:-1] + u_box[:-2, 1:-1, 1:-1] + u_box[1:-1, 2:, 1:-1]
            + u_box[1:-1, :-2, 1:-1] + u_box[1:-1, 1:-1, 2:] + u_box[1:-1, 1:-1, :-2] - 6.0 * c)
