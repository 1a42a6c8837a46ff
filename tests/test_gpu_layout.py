"""The GPU refinement-criterion layout builder (lgf_layout_adapt, eq. ref_crit) against the oracle's
adaptation step and the workload generator, bit for bit (integer output): repeated steps from the
base layout build the torus and vortex-ring layouts, a step on a refined layout with a moved
source drops and adds refinement, and the re-planned layout solves to the oracle's answer."""
import numpy as np
import pytest

from oracle import multires, refine
from paper_1911_10228_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
ALPHA = 1.0 / 32


@pytest.fixture(scope="module")
def lgf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_10228_amd import lgf as m
    m.init()
    return m


def torus_source(L):
    m = L.meta
    return lambda b, lv, nb: workloads.torus_source(workloads.cell_centres(b, lv, nb), m["centre"], m["axis"],
                                                    m["R"], m["sigma"])[0]


def gpu_steps(lgf, base, n_b, n_levels, source, check_oracle=True):
    blocks, levels = base.astype(np.int32), np.zeros(len(base), np.int32)
    for step in range(n_levels - 1):
        f = source(blocks, levels, n_b)
        print(f"step {step}: {len(blocks)} blocks", flush=True)
        nb_, nl_ = lgf.adapt_layout(blocks, levels, n_b, torch.from_numpy(np.ascontiguousarray(f)).cuda(),
                                    n_levels, ALPHA)
        if check_oracle:
            ob, ol = refine.adapt(blocks, levels, f, n_levels, ALPHA)
            assert np.array_equal(nb_, ob) and np.array_equal(nl_, ol), step
        blocks, levels = nb_, nl_
    return blocks, levels


@pytest.mark.parametrize("n_b,nblk", [(16, 8), (8, 4)])
def test_builder_reproduces_the_torus_layout(lgf, n_b, nblk):
    L = workloads.torus(nblk=nblk, n_b=n_b, n_levels=3)
    b, l = gpu_steps(lgf, workloads.box_blocks(nblk, nblk, nblk), n_b, 3, torus_source(L))
    assert np.array_equal(b, L.blocks) and np.array_equal(l, L.levels)
    # the finished layout is a fixed point of the step
    f = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
    b2, l2 = lgf.adapt_layout(b, l, n_b, f, 3, ALPHA)
    assert np.array_equal(b2, b) and np.array_equal(l2, l)


def test_builder_reproduces_the_vortex_ring_layout(lgf):
    """The vortex ring refined by its vorticity magnitude (4 levels)."""
    nblk, n_b, n_levels = 4, 8, 4
    L = workloads.vortex_ring(nblk=nblk, n_b=n_b, n_levels=n_levels)
    h = L.meta["h"]

    def omega(b, lv, nb):
        pos = (workloads.cell_centres(b, lv, nb) + 0.5) * h - 0.25
        _, _, ox, oy = workloads.vortex_ring_field(pos, 0.125, 1e3, 10.0)
        return np.sqrt(ox * ox + oy * oy)

    b, l = gpu_steps(lgf, workloads.box_blocks(nblk, nblk, nblk), n_b, n_levels, omega)
    assert np.array_equal(b, L.blocks) and np.array_equal(l, L.levels)
    assert int(l.max()) == n_levels - 1


def test_step_follows_a_moved_source_and_replans(lgf):
    """Negative block coordinates, a source that moves: the step equals the oracle's, and the
    new layout's plan (the resident kernel spectra reused) solves to the oracle's answer."""
    n_b = 8
    base = workloads.box_blocks(6, 6, 6, origin=(-3, -3, -3))
    near = workloads.Mixture(np.array([[-10.0, -8.0, -9.0]]), np.array([1.6]), np.array([1.0]))
    far = workloads.Mixture(np.array([[12.0, 9.0, 10.0]]), np.array([1.6]), np.array([-1.0]))
    b, l = gpu_steps(lgf, base, n_b, 3, near)
    assert int(l.max()) == 2
    f = far(b, l, n_b)
    b2, l2 = lgf.adapt_layout(b, l, n_b, torch.from_numpy(np.ascontiguousarray(f)).cuda(), 3, ALPHA)
    ob, ol = refine.adapt(b, l, f, 3, ALPHA)
    assert np.array_equal(b2, ob) and np.array_equal(l2, ol)
    assert int(l2.max()) == 1 and len(b2) != len(b)
    fs = far(b2, l2, n_b)
    p = lgf.Plan(b2, l2, n_b, 6)
    src = torch.from_numpy(np.ascontiguousarray(fs)).cuda()
    u = torch.zeros_like(src)
    p.solve(src, u)
    torch.cuda.synchronize()
    ref = multires.solve(b2, l2, fs, n_b, 6)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    p.close()


def test_builder_rejects_a_duplicate_block(lgf):
    blocks = np.array([[0, 0, 0], [1, 0, 0], [0, 0, 0]], np.int32)
    f = torch.ones((3, 8, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(lgf.LgfError) as e:
        lgf.adapt_layout(blocks, np.zeros(3, np.int32), 8, f, 2, ALPHA)
    assert e.value.code == -2
