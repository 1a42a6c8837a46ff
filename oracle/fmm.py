"""Fast lattice Green's function method on one uniform block level, FP64 (test infrastructure only).

Sec. 2.1 and Algorithm 1 of the paper:

1. upward pass: the effective source of a node is the sum over its children of R applied to the
   child's effective source (R = J^T, ``interp``);
2. level interaction: on every tree level, each target block is convolved with the blocks of its
   influence list I(B) (and, on the base level, its near region N(B)); each block convolution is
   a zero-padded FFT convolution, i.e. a Hadamard product in Fourier space;
3. downward pass: from the root to the base, every node adds the interpolation J of its parent's
   accumulated field to its own level-interaction result.

Readings where the paper is silent (it defers the details to Liska & Colonius 2014):

* coarse-level kernel: a level-k node holds n_b^3 interpolation nodes at the centres of cells of
  size s = 2^k base cells, so node offsets are s (d n_b + r) with d the block offset and
  r in [-(n_b-1), n_b-1]^3; the kernel is the base-lattice G sampled there (the K(x_p, y_q) of
  eq. fmm_conv_combined);
* zero padding to P = 2 n_b: the kernel value of offset r sits at index r mod P and index n_b is
  zero; the output block is the first n_b^3 entries.

The per-interaction products are summed in Fourier space before one inverse FFT per target; by
linearity of the inverse transform this equals summing the individual block convolutions.
Blocks are arrays [z, y, x] (x fastest in memory); block coordinates are (bx, by, bz).
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from . import interp, lgf, tree


def kernel_block(n_b: int, s: int, d) -> np.ndarray:
    """Real P^3 array K[r mod P] = G(s (d n_b + r)) for r in [-(n_b-1), n_b-1]^3, zero elsewhere."""
    P = 2 * n_b
    r = np.arange(-(n_b - 1), n_b)
    rz, ry, rx = np.meshgrid(r, r, r, indexing="ij")
    dx, dy, dz = (int(v) for v in d)
    n = np.stack([s * (dx * n_b + rx), s * (dy * n_b + ry), s * (dz * n_b + rz)], axis=-1)
    K = np.zeros((P, P, P))
    K[np.ix_(r % P, r % P, r % P)] = lgf.lgf(n)
    return K


def block_conv_fft(n_b: int, s: int, d, f: np.ndarray) -> np.ndarray:
    """conv(G_{t-src}, f_src) for one block pair by zero-padded FFT (d = target - source)."""
    P = 2 * n_b
    Kh = np.fft.rfftn(kernel_block(n_b, s, d))
    Fh = np.fft.rfftn(f, s=(P, P, P), axes=(0, 1, 2))
    return np.fft.irfftn(Kh * Fh, s=(P, P, P), axes=(0, 1, 2))[:n_b, :n_b, :n_b]


def block_conv_direct(n_b: int, s: int, d, f: np.ndarray) -> np.ndarray:
    """The same block convolution by direct summation (pin of the FFT version)."""
    out = np.zeros((n_b, n_b, n_b))
    idx = np.arange(n_b)
    dx, dy, dz = (int(v) for v in d)
    for z in range(n_b):
        for y in range(n_b):
            for x in range(n_b):
                rz = z - idx[:, None, None]
                ry = y - idx[None, :, None]
                rx = x - idx[None, None, :]
                n = np.stack(np.broadcast_arrays(s * (dx * n_b + rx), s * (dy * n_b + ry),
                                                 s * (dz * n_b + rz)), axis=-1)
                out[z, y, x] = (lgf.lgf(n) * f).sum()
    return out


def flgf(blocks, f, n_b: int, n_i: int, sources=None, targets=None, scale: float = 1.0,
         dtype=np.float64):
    """Algorithm 1 on the block set ``blocks`` ([n, 3]) with sources f ([n, n_b, n_b, n_b]).

    ``sources`` / ``targets`` are optional boolean masks over the base blocks: blocks outside
    ``sources`` carry zero source, outputs are produced for ``targets`` only (others are 0).
    The octree is always that of all ``blocks``.  Returns scale * u as [n, n_b, n_b, n_b].
    ``dtype=np.float32`` emulates a single-precision run (float32 transforms and products; the
    kernel spectra are computed in FP64 and rounded once)."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    f = np.asarray(f, dtype=np.float64).reshape(-1, n_b, n_b, n_b)
    nbase = len(blocks)
    src_mask = np.ones(nbase, bool) if sources is None else np.asarray(sources, bool)
    tgt_mask = np.ones(nbase, bool) if targets is None else np.asarray(targets, bool)
    levels = tree.build_levels(blocks)
    K = len(levels)
    W = interp.child_matrix(n_b, n_i).astype(dtype)
    P = 2 * n_b
    cdt = np.complex64 if dtype == np.float32 else np.complex128

    # parent index and octant of every node
    parent, octant = [], []
    for k in range(K - 1):
        pidx = tree.index_of(levels[k + 1])
        par = tree.parent_of(levels[k])
        parent.append(np.array([pidx[tuple(int(v) for v in p)] for p in par]))
        octant.append(levels[k] - 2 * par)

    # which nodes carry source / need a field (ancestors of source / target base blocks)
    is_src, is_tgt = [src_mask], [tgt_mask]
    for k in range(K - 1):
        s_up = np.zeros(len(levels[k + 1]), bool)
        t_up = np.zeros(len(levels[k + 1]), bool)
        s_up[parent[k][is_src[k]]] = True
        t_up[parent[k][is_tgt[k]]] = True
        is_src.append(s_up)
        is_tgt.append(t_up)

    # 1. upward pass
    src = [np.where(src_mask[:, None, None, None], f, 0.0).astype(dtype)]
    for k in range(K - 1):
        acc = np.zeros((len(levels[k + 1]), n_b, n_b, n_b), dtype)
        for i in np.nonzero(is_src[k])[0]:
            acc[parent[k][i]] += interp.anterp_child(W, octant[k][i], src[k][i])
        src.append(acc)

    # 2. level interaction
    v = []
    for k in range(K):
        s = 2**k
        nodes = levels[k]
        vk = np.zeros((len(nodes), n_b, n_b, n_b), dtype)
        pairs = [(t, j) for (t, j) in tree.interactions(nodes, base=(k == 0))
                 if is_tgt[k][t] and is_src[k][j]]
        if pairs:
            Fh = {j: scipy.fft.rfftn(src[k][j], s=(P, P, P), axes=(0, 1, 2)) for j in {j for _, j in pairs}}
            Kh = {}
            acc = {}
            for t, j in pairs:
                d = tuple(int(v) for v in nodes[t] - nodes[j])
                if d not in Kh:
                    Kh[d] = np.fft.rfftn(kernel_block(n_b, s, d)).astype(cdt)
                acc[t] = acc.get(t, cdt(0)) + Kh[d] * Fh[j]
            for t, a in acc.items():
                vk[t] = scipy.fft.irfftn(a, s=(P, P, P), axes=(0, 1, 2))[:n_b, :n_b, :n_b]
        v.append(vk)

    # 3. downward pass
    for k in range(K - 2, -1, -1):
        for i in np.nonzero(is_tgt[k])[0]:
            v[k][i] += interp.interp_child(W, octant[k][i], v[k + 1][parent[k][i]])
    out = (dtype(scale) * v[0]).astype(dtype)
    out[~tgt_mask] = 0.0
    return out


def count_interactions(blocks):
    """Number of near and far interactions per tree level (for the list pins)."""
    levels = tree.build_levels(blocks)
    res = []
    for k, nodes in enumerate(levels):
        pairs = tree.interactions(nodes, base=(k == 0))
        d = np.array([np.abs(nodes[t] - nodes[j]).max() for t, j in pairs]) if pairs else np.zeros(0)
        near = int((d <= 1).sum()) if k == 0 else 0
        res.append((len(nodes), near, len(pairs) - near))
    return res
