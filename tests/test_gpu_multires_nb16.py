"""Refined layouts at 16^3 blocks (the block size of the vortex-ring/torus workload) against the
FP64 oracle of Algorithm 2 (Sec. 3): coarsening, the leaf/non-leaf split, the quadratic
refinement J^l, the source correction and the FP64 super-block spectra of FP32 blocks are all
instantiated for N_b = 16 here.

Bars: FP64 within 1e-12 relative L-inf on both base-level paths; FP32 without defect correction
within 1e-6 of the FP64 oracle; FP32 + K defect-correction iterations within 1e-6 of the oracle's
K iterations with FP64 inner solves (the correction moves the answer towards the lattice
solution by the FMM truncation error, so that is the comparison that isolates precision)."""
import numpy as np
import pytest

from oracle import dc as dc_oracle, multires
from paper_1911_10228_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lgf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_10228_amd import lgf as m
    m.init()
    return m


def two_level16():
    base = workloads.box_blocks(4, 4, 4)
    fine = workloads.box_blocks(4, 4, 4, origin=(2, 2, 2))
    blocks = np.concatenate([base, fine]).astype(np.int32)
    levels = np.concatenate([np.zeros(64, np.int32), np.ones(64, np.int32)])
    n_b = 16
    pos = workloads.cell_centres(blocks, levels, n_b)
    f = workloads.gaussian_mixture(pos, [(2.0 * n_b - 0.5,) * 3], [0.3 * n_b], [1.0])
    return workloads.Layout(blocks, levels, n_b, f, 6)


def three_level16():
    """Three levels with a ragged finest level (2 x 4 x 2 blocks off-centre)."""
    base = workloads.box_blocks(4, 4, 4)
    l1 = workloads.box_blocks(4, 4, 4, origin=(2, 2, 2))
    l2 = workloads.box_blocks(2, 4, 2, origin=(6, 4, 6))
    blocks = np.concatenate([base, l1, l2]).astype(np.int32)
    levels = np.concatenate([np.zeros(64), np.ones(64), np.full(16, 2)]).astype(np.int32)
    n_b = 16
    pos = workloads.cell_centres(blocks, levels, n_b)
    f = workloads.gaussian_mixture(pos, [(2.0 * n_b, 2.2 * n_b, 2.0 * n_b)], [0.25 * n_b], [1.0])
    return workloads.Layout(blocks, levels, n_b, f, 6)


def torus16():
    """The tilted Gaussian-core torus on 4^3 base blocks of 16^3 with 3 levels (64 / 192 / 608
    blocks, 3.5 M unknowns), refined by the criterion of eq. ref_crit."""
    return workloads.torus(nblk=4, n_b=16, n_levels=3, interp_order=6)


_cache = {}


def case(name):
    if name not in _cache:
        L = {"two": two_level16, "three": three_level16, "torus": torus16}[name]()
        print(f"oracle: {name} ({len(L.blocks)} blocks of 16^3)", flush=True)
        ref = multires.solve(L.blocks, L.levels, L.f, L.n_b, L.interp_order)
        _cache[name] = (L, ref)
    return _cache[name]


def rel_linf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def solve(lgf, L, precision=0, dc=0, base_level=0, autotune=0, plan=None):
    p = plan or lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, dc,
                         base_level=base_level, autotune=autotune)
    f = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
    u = torch.full_like(f, float("nan"))
    p.solve(f, u)
    torch.cuda.synchronize()
    return u.cpu().numpy(), p


@pytest.mark.parametrize("base_level", [0, 1])
@pytest.mark.parametrize("name", ["two", "three", "torus"])
def test_refined_nb16_fp64(lgf, name, base_level):
    L, ref = case(name)
    print(f"case {name} FP64 base_level {base_level}", flush=True)
    u, p = solve(lgf, L, base_level=base_level)
    assert rel_linf(u, ref) <= 1e-12
    p.close()


@pytest.mark.parametrize("name", ["two", "three", "torus"])
def test_refined_nb16_fp32(lgf, name):
    L, ref = case(name)
    print(f"case {name} FP32 without correction", flush=True)
    u, p = solve(lgf, L, precision=1, dc=0)
    assert rel_linf(u, ref) <= 1e-6
    p.close()


def test_refined_nb16_fp32_defect_correction(lgf):
    L, _ = case("three")
    its = dc_oracle.solve_dc(L.blocks, L.levels, L.f, L.n_b, L.interp_order, iters=2, dtype=np.float64)
    for k in (1, 2):
        print(f"case three FP32 + {k} DC", flush=True)
        u, p = solve(lgf, L, precision=1, dc=k)
        assert rel_linf(u, its[k]) <= 1e-6, k
        p.close()


def test_refined_nb16_every_near_shape(lgf):
    """Every launch shape of the base-level super-block MAC, forced on an autotuned plan of the
    two-level layout: rows of 2, 4 and 8 targets, the pipelined and the fused compact tiles, on
    FP64 spectra (FP64 plans, and FP32 plans of a refined layout, whose super-block spectra are
    FP64)."""
    L, ref = case("two")
    f = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
    for precision, tol in ((0, 1e-12), (1, 1e-6)):
        p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, 0, autotune=1)
        for shape in (2, 4, 8, 21, 23, 42, 44, 0):
            print(f"case two precision {precision} near shape {shape}", flush=True)
            try:
                p.set_near_shape(shape)
            except RuntimeError:
                assert shape in (21, 23, 42, 44), shape   # compact tiles need <= 36 / 48 sources
                continue
            u, _ = solve(lgf, L, plan=p)
            assert rel_linf(u, ref) <= tol, f"precision {precision} shape {shape}"
        p.close()
