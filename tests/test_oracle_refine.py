"""Pins of the oracle's adaptation step by the refinement criterion (eq. ref_crit, Sec. 3,
Convergence subsection; reading: exponent L_R - 1 - l, omega = block max |field|): a layout
worked out by hand, reproduction of the workload generator's layouts (independent code that
builds all levels at once from an analytic source) by repeated steps, the fixed point, and the
removal of children whose parent no longer meets the criterion."""
import numpy as np

from oracle import refine
from paper_1911_10228_amd import workloads

ALPHA = 1.0 / 32


def test_hand_worked_layout():
    """Two base blocks of 2^3 cells, L_R = 3.  Step 1: level-0 threshold alpha^2 * 1.0 = 1/1024;
    block (0,0,0) (max 1.0) is refined, block (1,0,0) (max 5e-4) is not.  Step 2: the level-1
    threshold is alpha * 1.0 = 1/32; of the 8 children only (1,1,1) (max 1.0) exceeds it (the
    others have 0.02), so it gets the level-2 children (2..3)^3; level 0 is decided as before."""
    nb = 2
    blocks = np.array([[0, 0, 0], [1, 0, 0]])
    levels = np.array([0, 0])
    f = np.zeros((2, nb, nb, nb))
    f[0, 1, 0, 1] = -1.0                       # |value| counts
    f[1, 0, 0, 0] = 5e-4
    b1, l1 = refine.adapt(blocks, levels, f, 3, ALPHA)
    kids = [[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)]
    assert b1.tolist() == [[0, 0, 0], [1, 0, 0]] + kids
    assert l1.tolist() == [0, 0] + [1] * 8
    f2 = np.zeros((10, nb, nb, nb))
    f2[0, 0, 0, 0] = 1.0
    f2[1, 0, 0, 0] = 5e-4
    f2[2:, 0, 1, 0] = 0.02
    f2[9, 1, 1, 1] = 1.0                       # child (1,1,1) is the last of the 8
    b2, l2 = refine.adapt(b1, l1, f2, 3, ALPHA)
    grand = [[x, y, z] for x in (2, 3) for y in (2, 3) for z in (2, 3)]
    assert b2.tolist() == [[0, 0, 0], [1, 0, 0]] + kids + grand
    assert l2.tolist() == [0, 0] + [1] * 8 + [2] * 8
    # the finest level is never refined, whatever its field
    f3 = np.ones((18, nb, nb, nb))
    b3, l3 = refine.adapt(b2, l2, f3, 3, ALPHA)
    assert int(l3.max()) == 2


def _iterate(base, n_b, n_levels, source):
    blocks, levels = base, np.zeros(len(base), np.int32)
    for _ in range(n_levels - 1):
        blocks, levels = refine.adapt(blocks, levels, source(blocks, levels, n_b), n_levels, ALPHA)
    return blocks, levels


def test_repeated_steps_reproduce_the_generator_on_the_torus():
    L = workloads.torus(nblk=4, n_b=8, n_levels=3)
    m = L.meta
    src = lambda b, lv, nb: workloads.torus_source(workloads.cell_centres(b, lv, nb), m["centre"], m["axis"],
                                                   m["R"], m["sigma"])[0]
    b, l = _iterate(workloads.box_blocks(4, 4, 4), 8, 3, src)
    assert np.array_equal(b, L.blocks) and np.array_equal(l, L.levels)
    # a fixed point: the step on the finished layout returns it unchanged
    b2, l2 = refine.adapt(b, l, src(b, l, 8), 3, ALPHA)
    assert np.array_equal(b2, b) and np.array_equal(l2, l)


def test_repeated_steps_reproduce_the_generator_with_four_levels():
    rng = np.random.default_rng(12)
    mix = workloads.Mixture(rng.uniform(8, 24, size=(3, 3)), rng.uniform(1.0, 2.5, size=3), rng.normal(size=3))
    ref_b, ref_l = workloads.refine_by_criterion(workloads.box_blocks(4, 4, 4), 8, 4, mix)
    b, l = _iterate(workloads.box_blocks(4, 4, 4), 8, 4, mix)
    assert np.array_equal(b, ref_b) and np.array_equal(l, ref_l)
    assert int(l.max()) == 3


def test_children_go_when_the_parent_no_longer_qualifies():
    """Moving the source away removes the refinement that followed it: blocks whose parent fails
    the criterion are not in the new layout, blocks new in this step are not refined further."""
    n_b = 8
    near = workloads.Mixture(np.array([[8.0, 8.0, 8.0]]), np.array([1.5]), np.array([1.0]))
    far = workloads.Mixture(np.array([[56.0, 56.0, 56.0]]), np.array([1.5]), np.array([1.0]))
    b, l = _iterate(workloads.box_blocks(8, 8, 8), n_b, 3, near)
    assert int(l.max()) == 2
    b2, l2 = refine.adapt(b, l, far(b, l, n_b), 3, ALPHA)
    assert int(l2.max()) == 1                  # the new level-1 blocks have no field yet
    assert np.all(b2[l2 == 1].min(axis=0) >= 12)
    # the same as the first two levels of the generator's 3-level layout around the new source
    ref_b, ref_l = workloads.refine_by_criterion(workloads.box_blocks(8, 8, 8), n_b, 3, far)
    keep = ref_l <= 1
    assert np.array_equal(b2, ref_b[keep]) and np.array_equal(l2, ref_l[keep])
