"""Defect correction of a reduced-precision solve (test infrastructure only).

The problem is L u = f with the 7-point operator (Sec. 2, the discrete Poisson equation; per
refinement level L^l = h_l^-2 (6 neighbours - 6 centre), Sec. 3).  Given any approximate solver
S (here the FLGF of ``fmm`` / ``multires`` run in FP32 arithmetic):

    u_0 = S(f);   r_k = M (f - L u_k) in FP64;   u_{k+1} = u_k + S(r_k)  (update in FP64)

with M the leaf cells whose six neighbours all lie in blocks of the same level (elsewhere the
residual cannot be formed from stored values).  The FP32 emulation uses scipy.fft on float32
inputs (complex64 transforms) and float32 products and sums.
"""
from __future__ import annotations

import numpy as np

from . import multires


def solve_dc(blocks, levels, f, n_b: int, n_i: int, iters: int, dtype=np.float32):
    """Returns the list [u_0, u_1, ..., u_iters] of FP64 iterates."""
    f = np.asarray(f, dtype=np.float64)
    solve = lambda src: multires.solve(blocks, levels, src, n_b, n_i, dtype=dtype).astype(np.float64)
    mask = multires.residual_mask(blocks, levels, n_b)
    u = solve(f)
    out = [u]
    for _ in range(iters):
        r = np.where(mask, f - multires.apply_laplace(blocks, levels, u, n_b), 0.0)
        u = u + solve(r)
        out.append(u)
    return out
