"""Host-only plan builds (no GPU): every kernel work item of every step stays inside the
plan's buffers, and the interaction counts equal the oracle's octree lists (bit-exact
integer bookkeeping).  This runs the same C++ planner the GPU path uses."""
import numpy as np
import pytest

from oracle import fmm, multires
from paper_1911_10228_amd import lgf, workloads


def oracle_interactions(blocks, levels):
    """Sum over refinement levels of near + far pairs, channel T (all -> all) plus channel A
    (leaf sources -> non-leaf targets) where a level has non-leaf blocks."""
    blocks = np.asarray(blocks)
    levels = np.asarray(levels)
    have = {(int(l),) + tuple(int(v) for v in b) for b, l in zip(blocks, levels)}
    leaf = np.array([(int(l) + 1,) + tuple(int(v) for v in 2 * b) not in have
                     for b, l in zip(blocks, levels)])
    total = 0
    from oracle import tree
    for l in range(int(levels.max()) + 1):
        ids = np.nonzero(levels == l)[0]
        lb = blocks[ids]
        tl = tree.build_levels(lb)
        # ancestors of leaf / non-leaf base blocks per tree level
        src = leaf[ids].copy()
        tgt = ~leaf[ids]
        for k, nodes in enumerate(tl):
            pairs = tree.interactions(nodes, base=(k == 0))
            total += len(pairs)
            if tgt.any():
                total += sum(1 for t, s in pairs if tgt[t] and src[s])
            if k + 1 < len(tl):
                pidx = tree.index_of(tl[k + 1])
                par = np.array([pidx[tuple(int(v) for v in p)] for p in tree.parent_of(nodes)])
                s2 = np.zeros(len(tl[k + 1]), bool)
                t2 = np.zeros(len(tl[k + 1]), bool)
                s2[par[src]] = True
                t2[par[tgt]] = True
                src, tgt = s2, t2
    return total


LAYOUTS = {
    "gauss2": lambda: workloads.uniform_gaussian(),
    "box6x8": lambda: workloads.uniform_mixture(nblk=6, n_b=8, n_gauss=3, seed=1),
    "box8x16": lambda: workloads.uniform_mixture(nblk=8, n_b=16, n_gauss=3, seed=2),
    "slab": lambda: workloads.Layout(workloads.box_blocks(13, 3, 1, origin=(-5, 2, 7)),
                                     np.zeros(39, np.int32), 8, None, 6),
    "sparse_neg": lambda: workloads.Layout(
        np.unique(np.random.default_rng(11).integers(-9, 7, size=(70, 3)), axis=0).astype(np.int32),
        None, 8, None, 6),
}


@pytest.mark.parametrize("name", sorted(LAYOUTS))
@pytest.mark.parametrize("precision,dc,tune", [(0, 0, 0), (1, 0, 1), (1, 2, 0), (0, 0, 1)])
def test_uniform_layouts_validate_and_count(name, precision, dc, tune):
    L = LAYOUTS[name]()
    levels = L.levels if L.levels is not None else np.zeros(len(L.blocks), np.int32)
    info = lgf.plan_check(L.blocks, levels, L.n_b, L.interp_order, precision, dc, autotune=tune)
    counts = fmm.count_interactions(L.blocks)
    assert info["interactions"] == sum(a + b for _, a, b in counts)
    assert info["blocks"] == len(L.blocks)


def test_coarse_lds_tiles_take_the_inner_window_only_where_sources_allow():
    """The coarse MAC's LDS form skips the products of a tile's outer window entries only when
    all of the tile's sources lie within its rows' x extent: on the 8^3 layout (level 1 is one
    row of 4 wide) every tile does, on the scattered layout none does, so the GPU parity tests
    of those two layouts run both walks."""
    L = LAYOUTS["box8x16"]()
    info = lgf.plan_check(L.blocks, np.zeros(len(L.blocks), np.int32), L.n_b, L.interp_order)
    assert info["mac_lds_tiles"] == info["mac_lds_inner"] == 4
    L = LAYOUTS["sparse_neg"]()
    info = lgf.plan_check(L.blocks, np.zeros(len(L.blocks), np.int32), L.n_b, L.interp_order)
    assert info["mac_lds_tiles"] > 0 and info["mac_lds_inner"] == 0


def multi_layouts():
    out = []
    base = workloads.box_blocks(4, 4, 4)
    l1 = workloads.box_blocks(4, 4, 4, origin=(2, 2, 2))
    l2 = workloads.box_blocks(2, 4, 2, origin=(6, 4, 6))
    out.append((np.concatenate([base, l1, l2]), np.repeat([0, 1, 2], [64, 64, 16]), 8))
    # refinement touching the domain edge and a negative-coordinate base
    b0 = workloads.box_blocks(3, 3, 3, origin=(-1, -2, 0))
    kids = np.array([[2 * x + i, 2 * y + j, 2 * z + k] for x, y, z in [(-1, -2, 0), (1, 0, 2)]
                     for i in (0, 1) for j in (0, 1) for k in (0, 1)])
    out.append((np.concatenate([b0, kids]), np.repeat([0, 1], [27, 16]), 16))
    return out


@pytest.mark.parametrize("case", range(2))
@pytest.mark.parametrize("precision", [0, 1])
def test_multilevel_layouts_validate_and_count(case, precision):
    blocks, levels, n_b = multi_layouts()[case]
    info = lgf.plan_check(blocks, levels, n_b, 6, precision, 1)
    assert info["refinement_levels"] == int(levels.max()) + 1
    assert info["interactions"] == oracle_interactions(blocks, levels)


def test_batch_generator_layouts_validate():
    rng_layouts = workloads.batch(seed=4, count=6, max_blocks=120)
    for L in rng_layouts:
        for precision in (0, 1):
            info = lgf.plan_check(L.blocks, L.levels, L.n_b, L.interp_order, precision, 1)
            assert info["unknowns"] == L.unknowns


def test_torus_layout_validates():
    L = workloads.torus(nblk=4, n_b=8, n_levels=3)
    for precision in (0, 1):
        info = lgf.plan_check(L.blocks, L.levels, L.n_b, 6, precision, 1, autotune=1)
        assert info["refinement_levels"] == 3


def super_counts(blocks, levels):
    """Base-level super-block bookkeeping written out from the octree lists (oracle.tree): per
    refinement level and channel, the target super-blocks are the parents of target blocks with
    base-level interactions (N(B) + I(B)); each pairs with every neighbouring super-block holding
    a source block.  A source super-block transform is shared where the two channels have the
    same source children."""
    from oracle import tree
    blocks = np.asarray(blocks)
    levels = np.asarray(levels)
    have = {(int(l),) + tuple(int(v) for v in b) for b, l in zip(blocks, levels)}
    leaf = np.array([(int(l) + 1,) + tuple(int(v) for v in 2 * b) not in have
                     for b, l in zip(blocks, levels)])
    nbrs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    n_tgt = pairs = 0
    src_sets = set()
    for l in range(int(levels.max()) + 1):
        ids = np.nonzero(levels == l)[0]
        tl = tree.build_levels(blocks[ids])
        chans = [(np.ones(len(ids), bool), np.ones(len(ids), bool))]
        if not leaf[ids].all():
            chans.append((leaf[ids].copy(), ~leaf[ids]))
        for ch, (src0, tgt0) in enumerate(chans):
            # flags per octree level
            srcs, tgts = [src0], [tgt0]
            pars = []
            for k in range(len(tl) - 1):
                pidx = tree.index_of(tl[k + 1])
                par = np.array([pidx[tuple(int(v) for v in q)] for q in tree.parent_of(tl[k])])
                pars.append(par)
                s2 = np.zeros(len(tl[k + 1]), bool)
                t2 = np.zeros(len(tl[k + 1]), bool)
                s2[par[srcs[k]]] = True
                t2[par[tgts[k]]] = True
                srcs.append(s2)
                tgts.append(t2)
            has_ifft, referenced = [], []
            for k, nodes in enumerate(tl):
                h = np.zeros(len(nodes), bool)
                r = np.zeros(len(nodes), bool)
                for t, s_ in tree.interactions(nodes, base=(k == 0)):
                    if tgts[k][t] and srcs[k][s_]:
                        h[t] = True
                        r[s_] = True
                has_ifft.append(h)
                referenced.append(r)
            need = [None] * len(tl)
            for k in range(len(tl) - 1, -1, -1):
                up = need[k + 1][pars[k]] if k + 1 < len(tl) else np.zeros(len(tl[k]), bool)
                need[k] = srcs[k] & (referenced[k] | up)
            for k, nodes in enumerate(tl):
                if k > 0:                      # coarse levels keep the block-wise lists
                    continue
                use = srcs[k]
                kids = {}
                for i in np.nonzero(use)[0]:
                    b = tuple(int(v) for v in nodes[i])
                    kids.setdefault(tuple(v // 2 for v in b), set()).add(b)
                tsup = {tuple(int(v) // 2 for v in nodes[i]) for i in np.nonzero(has_ifft[k])[0]}
                n_tgt += len(tsup)
                for T in tsup:
                    for D in nbrs:
                        S = tuple(t - d for t, d in zip(T, D))
                        if S in kids:
                            pairs += 1
                            # base sources are shared by the channels; above, each channel
                            # anterpolates its own
                            src_sets.add((l, k, ch if k > 0 else -1, frozenset(kids[S])))
    return n_tgt, pairs, len(src_sets)


@pytest.mark.parametrize("case", ["box6x8", "slab", "sparse_neg", "multi0", "multi1", "torus"])
def test_super_block_bookkeeping(case):
    if case.startswith("multi"):
        blocks, levels, n_b = multi_layouts()[int(case[-1])]
        n_i = 6
    elif case == "torus":
        L = workloads.torus(nblk=4, n_b=8, n_levels=3)
        blocks, levels, n_b, n_i = L.blocks, L.levels, L.n_b, 6
    else:
        L = LAYOUTS[case]()
        blocks, n_b, n_i = L.blocks, L.n_b, L.interp_order
        levels = L.levels if L.levels is not None else np.zeros(len(blocks), np.int32)
    n_tgt, pairs, n_src = super_counts(blocks, levels)
    for precision in (0, 1):
        sup = lgf.plan_check(blocks, levels, n_b, n_i, precision, 1, base_level=lgf.LGF_BASE_SUPER)
        blk = lgf.plan_check(blocks, levels, n_b, n_i, precision, 1, base_level=lgf.LGF_BASE_BLOCK)
        assert (sup["super_inverse"], sup["near_pairs"], sup["super_forward"]) == (n_tgt, pairs, n_src)
        assert sup["interactions"] == blk["interactions"]
        assert blk["super_forward"] == blk["near_rows"] == 0
        # the per-block base transforms are the ones the super-blocks replace
        assert sup["fft_forward"] < blk["fft_forward"] and sup["fft_inverse"] < blk["fft_inverse"]


def test_base_level_option_rejects_unknown():
    L = workloads.uniform_gaussian()
    with pytest.raises(lgf.LgfError):
        lgf.plan_check(L.blocks, None, L.n_b, L.interp_order, 0, 0, base_level=2)
