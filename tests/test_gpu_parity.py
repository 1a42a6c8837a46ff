"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: FP64 solves within 1e-12 relative L-inf (max |u_gpu - u_oracle| / max |u_oracle|);
FP32 + defect correction within 1e-6; the LGF table within 1e-14 relative; integer bookkeeping
(interaction counts) exact.
"""
import numpy as np
import pytest

from oracle import dc as dc_oracle, direct, fmm, lgf as olgf, multires
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


def rel_linf(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def gpu_solve(lgf, L, precision=0, dc=0, order=None, plan=None, base_level=0):
    p = plan or lgf.Plan(L.blocks, L.levels, L.n_b, order or L.interp_order, precision, dc,
                         base_level=base_level)
    f = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
    u = torch.zeros_like(f)
    p.solve(f, u)
    torch.cuda.synchronize()
    return u.cpu().numpy(), p


# ----------------------------------------------------------------------------- LGF table
def test_green_table_matches_oracle(lgf):
    cube = torch.zeros((101, 101, 101), dtype=torch.float64, device="cuda")
    lgf.green_table(cube)
    torch.cuda.synchronize()
    g = cube.cpu().numpy()
    tri = olgf.sorted_triples()
    ref = olgf.table()[tri[:, 0], tri[:, 1], tri[:, 2]]
    got = g[tri[:, 0], tri[:, 1], tri[:, 2]]
    err = np.abs(got - ref) / np.abs(ref)
    assert err.max() <= 1e-14, (err.max(), tri[err.argmax()])
    # the GPU table satisfies L G = delta by itself
    assert abs(g[1, 0, 0] - g[0, 0, 0] - 1.0 / 6.0) <= 1e-15
    assert abs(g[0, 0, 0] - olgf.watson_g0()) <= 2e-15 * abs(g[0, 0, 0])


def test_green_eval_policy_regions(lgf):
    rng = np.random.default_rng(0)
    pts = np.concatenate([rng.integers(-60, 61, size=(400, 3)), rng.integers(-400, 401, size=(400, 3)),
                          rng.integers(-3000, 3001, size=(200, 3)),
                          np.array([[100, 0, 0], [101, 0, 0], [600, 0, 0], [601, 0, 0], [0, 0, 0],
                                    [36, 48, 80], [360, 480, 0]])]).astype(np.int32)
    nd = torch.from_numpy(pts).cuda()
    out = torch.zeros(len(pts), dtype=torch.float64, device="cuda")
    lgf.green_eval(nd, out)
    torch.cuda.synchronize()
    ref = olgf.lgf(pts)
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max()
    assert (np.abs(out.cpu().numpy() - ref) / np.abs(ref)).max() <= 1e-13


@pytest.mark.parametrize("n_b,s,d", [(8, 1, (0, 0, 0)), (8, 2, (3, -2, 1)), (16, 1, (-1, 2, 0)),
                                     (16, 4, (2, 3, -3)), (16, 16, (-3, 0, 2))])
def test_kernel_spectra_match_oracle(lgf, n_b, s, d):
    P = 2 * n_b
    out = torch.zeros((P, P, n_b + 1, 2), dtype=torch.float64, device="cuda")
    lgf.kernel_spectrum(n_b, s, d, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    ref = np.fft.rfftn(fmm.kernel_block(n_b, s, d))
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("n_b,d", [(8, (0, 0, 0)), (8, (1, -1, 0)), (16, (-1, 1, 1)), (16, (0, 0, 1))])
def test_super_block_kernel_spectra_match_oracle(lgf, n_b, d):
    """Base-level super-block kernels: blocks of 2 N_b cells on the base lattice (FFT size 4 N_b,
    transformed by the long-line DFT path for N_b = 16)."""
    B = 2 * n_b
    out = torch.zeros((2 * B, 2 * B, B + 1, 2), dtype=torch.float64, device="cuda")
    lgf.kernel_spectrum(n_b, 0, d, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    ref = np.fft.rfftn(fmm.kernel_block(B, 1, d))
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


def test_super_block_kernel_spectra_conjugate_pairs(lgf):
    """The near MAC reads the kernels h <= 13 and conjugates them for -d."""
    n_b = 8
    B = 2 * n_b
    spec = {}
    for d in [(1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1)]:
        out = torch.zeros((2 * B, 2 * B, B + 1, 2), dtype=torch.float64, device="cuda")
        lgf.kernel_spectrum(n_b, 0, d, out)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        spec[d] = o[..., 0] + 1j * o[..., 1]
    for d in [(1, 0, -1), (0, 1, 1)]:
        m = tuple(-x for x in d)
        assert np.abs(spec[m] - np.conj(spec[d])).max() <= 1e-14 * np.abs(spec[d]).max()


# ----------------------------------------------------------------------------- uniform FLGF
def test_uniform_gaussian_fp64_matches_oracle_and_brute_force(lgf):
    L = workloads.uniform_gaussian()
    u, p = gpu_solve(lgf, L)
    ref = fmm.flgf(L.blocks, L.f, L.n_b, L.interp_order)
    assert rel_linf(u, ref) <= 1e-12
    brute = direct.direct_sum(L.blocks, L.f, L.n_b).reshape(u.shape)
    assert rel_linf(u, brute) <= 1e-12
    assert p.info()["interactions"] == 64


@pytest.mark.parametrize("base_level", [0, 1])
@pytest.mark.parametrize("nblk,n_b,order", [(6, 8, 4), (5, 8, 8), (3, 16, 6)])
def test_uniform_multilevel_fp64(lgf, nblk, n_b, order, base_level):
    L = workloads.uniform_mixture(nblk=nblk, n_b=n_b, n_gauss=5, seed=nblk + n_b)
    u, p = gpu_solve(lgf, L, order=order, base_level=base_level)
    ref = fmm.flgf(L.blocks, L.f, L.n_b, order)
    assert rel_linf(u, ref) <= 1e-12
    counts = fmm.count_interactions(L.blocks)
    info = p.info()
    assert info["interactions"] == sum(a + b for _, a, b in counts)
    assert info["mac_lds_inner"] == info["mac_lds_tiles"]   # inner-window walk (if any LDS tiles)


@pytest.mark.parametrize("base_level", [0, 1])
def test_sparse_negative_ragged_layout_fp64(lgf, base_level):
    rng = np.random.default_rng(11)
    blocks = np.unique(rng.integers(-9, 7, size=(70, 3)), axis=0).astype(np.int32)
    n_b = 8
    levels = np.zeros(len(blocks), np.int32)
    pos = workloads.cell_centres(blocks, levels, n_b)
    f = workloads.gaussian_mixture(pos, [(-10, 5, 0), (20, -30, 10)], [3.0, 2.0], [1.0, -0.5])
    f = f + 0.01 * rng.normal(size=f.shape)
    L = workloads.Layout(blocks, levels, n_b, f, 6)
    u, p = gpu_solve(lgf, L, base_level=base_level)
    ref = fmm.flgf(blocks, f, n_b, 6)
    assert rel_linf(u, ref) <= 1e-12
    info = p.info()                  # the coarse LDS-form MAC walks its full source window here
    assert info["mac_lds_tiles"] > 0 and info["mac_lds_inner"] == 0


@pytest.mark.parametrize("base_level", [0, 1])
def test_point_source_gives_the_green_function(lgf, base_level):
    """A unit source at one lattice point: on 2x2x2 blocks every pair is in the near field, so
    the result is the lattice Green's function itself (Sec. 2, eq. discretConv), compared with
    the oracle's LGF evaluation, not with its FMM."""
    n_b = 8
    blocks = workloads.box_blocks(2, 2, 2)
    f = np.zeros((len(blocks), n_b, n_b, n_b))
    f[3, 5, 1, 6] = 1.0                                  # block 3, cell (x, y, z) = (6, 1, 5)
    L = workloads.Layout(blocks, np.zeros(len(blocks), np.int32), n_b, f, 4)
    u, _ = gpu_solve(lgf, L, base_level=base_level)
    src = blocks[3] * n_b + np.array([6, 1, 5])
    pos = direct.cell_coords(blocks, n_b).reshape(len(blocks), n_b, n_b, n_b, 3)
    g = olgf.lgf(pos - src)
    assert np.abs(u - g).max() <= 1e-12 * np.abs(g).max()


@pytest.mark.parametrize("precision,dc", [(0, 0), (1, 1)])
def test_zero_source_gives_zero(lgf, precision, dc):
    L = workloads.uniform_mixture(nblk=4, n_b=8, n_gauss=2, seed=3)
    L = workloads.Layout(L.blocks, L.levels, L.n_b, np.zeros_like(L.f), L.interp_order)
    u, _ = gpu_solve(lgf, L, precision=precision, dc=dc)
    assert not np.any(u)


def test_largest_interpolation_order(lgf):
    """n_I = 10, the paper's largest order, on 16^3 blocks with a far field."""
    L = workloads.uniform_mixture(nblk=5, n_b=16, n_gauss=4, seed=41, interp_order=10)
    u, _ = gpu_solve(lgf, L, order=10)
    assert rel_linf(u, fmm.flgf(L.blocks, L.f, L.n_b, 10)) <= 1e-12


def test_single_block(lgf):
    L = workloads.Layout(np.array([[3, -2, 5]], np.int32), np.zeros(1, np.int32), 16,
                         np.random.default_rng(2).normal(size=(1, 16, 16, 16)), 4)
    u, _ = gpu_solve(lgf, L)
    ref = fmm.flgf(L.blocks, L.f, 16, 4)
    assert rel_linf(u, ref) <= 1e-12


@pytest.mark.parametrize("base_level", [0, 1])
def test_uniform_fp32_defect_correction(lgf, base_level):
    """FP32 without DC is compared with the FP64 FLGF oracle; with K DC iterations it is compared
    with the oracle's DC of the same K (FP64 inner solves), which isolates precision: DC moves the
    answer towards the lattice solution L u = f by the FMM truncation error."""
    L = workloads.uniform_mixture(nblk=6, n_b=8, n_gauss=6, seed=3, interp_order=8)
    ref = fmm.flgf(L.blocks, L.f, L.n_b, 8)
    u, _ = gpu_solve(lgf, L, precision=1, dc=0, base_level=base_level)
    assert rel_linf(u, ref) <= 1e-6
    its = dc_oracle.solve_dc(L.blocks, L.levels, L.f, L.n_b, 8, iters=2, dtype=np.float64)
    for k in (1, 2):
        u, _ = gpu_solve(lgf, L, precision=1, dc=k, base_level=base_level)
        assert rel_linf(u, its[k]) <= 1e-6


# ----------------------------------------------------------------------------- multi-resolution
def two_level(n_b):
    base = workloads.box_blocks(4, 4, 4)
    fine = workloads.box_blocks(4, 4, 4, origin=(2, 2, 2))
    blocks = np.concatenate([base, fine]).astype(np.int32)
    levels = np.concatenate([np.zeros(64, np.int32), np.ones(64, np.int32)])
    pos = workloads.cell_centres(blocks, levels, n_b)
    f = workloads.gaussian_mixture(pos, [(2.0 * n_b - 0.5,) * 3], [0.3 * n_b], [1.0])
    return workloads.Layout(blocks, levels, n_b, f, 6)


def three_level(n_b=8):
    base = workloads.box_blocks(4, 4, 4)
    l1 = workloads.box_blocks(4, 4, 4, origin=(2, 2, 2))
    l2 = workloads.box_blocks(2, 4, 2, origin=(6, 4, 6))
    blocks = np.concatenate([base, l1, l2]).astype(np.int32)
    levels = np.concatenate([np.zeros(64), np.ones(64), np.full(16, 2)]).astype(np.int32)
    pos = workloads.cell_centres(blocks, levels, n_b)
    f = workloads.gaussian_mixture(pos, [(2.0 * n_b, 2.2 * n_b, 2.0 * n_b)], [0.25 * n_b], [1.0])
    return workloads.Layout(blocks, levels, n_b, f, 6)


@pytest.mark.parametrize("base_level", [0, 1])
@pytest.mark.parametrize("make", [lambda: two_level(8), three_level])
def test_multires_fp64(lgf, make, base_level):
    L = make()
    u, _ = gpu_solve(lgf, L, base_level=base_level)
    ref = multires.solve(L.blocks, L.levels, L.f, L.n_b, L.interp_order)
    assert rel_linf(u, ref) <= 1e-12


def test_multires_fp32_defect_correction(lgf):
    L = three_level()
    ref = multires.solve(L.blocks, L.levels, L.f, L.n_b, L.interp_order)
    u, _ = gpu_solve(lgf, L, precision=1, dc=0)
    assert rel_linf(u, ref) <= 1e-6
    its = dc_oracle.solve_dc(L.blocks, L.levels, L.f, L.n_b, L.interp_order, iters=2, dtype=np.float64)
    u, _ = gpu_solve(lgf, L, precision=1, dc=2)
    assert rel_linf(u, its[2]) <= 1e-6


# ----------------------------------------------------------------------------- batching
def test_batch_equals_alone(lgf):
    Ls = [workloads.uniform_gaussian(), two_level(8),
          workloads.uniform_mixture(nblk=3, n_b=16, n_gauss=3, seed=9, interp_order=6)]
    alone = [gpu_solve(lgf, L)[0] for L in Ls]
    plans = [lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order) for L in Ls]
    fs = [torch.from_numpy(np.ascontiguousarray(L.f)).cuda() for L in Ls]
    us = [torch.zeros_like(f) for f in fs]
    lgf.solve_batch(plans, fs, us)
    torch.cuda.synchronize()
    for a, u in zip(alone, us):
        assert np.array_equal(a, u.cpu().numpy())


def test_vector_poisson_components(lgf):
    """Three source components through a VectorPlan (one batched solve): each component equals
    its own scalar solve bit for bit and matches the FP64 oracle."""
    L = workloads.uniform_mixture(nblk=3, n_b=8, n_gauss=3, seed=41, interp_order=6)
    comps = [L.f, np.roll(L.f, 5, axis=1), -0.5 * L.f + 0.25]
    vp = lgf.VectorPlan(L.blocks, L.levels, L.n_b, L.interp_order, components=3)
    f = torch.from_numpy(np.ascontiguousarray(np.stack(comps))).cuda()
    u = torch.zeros_like(f)
    vp.solve(f, u)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order)
    for c, fc in enumerate(comps):
        one = torch.zeros_like(f[c])
        p.solve(f[c].clone(), one)
        torch.cuda.synchronize()
        assert np.array_equal(one.cpu().numpy(), got[c]), f"component {c}"
        ref = fmm.flgf(L.blocks, fc, L.n_b, L.interp_order)
        assert np.abs(got[c] - ref).max() <= 1e-12 * np.abs(ref).max(), f"component {c}"
    p.close()
    vp.close()


@pytest.mark.parametrize("make", [three_level, lambda: two_level(16)])
def test_forward_operators_match_oracle(lgf, make):
    """Laplacian, gradient and curl through lgf_apply against the oracle's operators on a refined
    layout: random fields, every cell compared (the output starts as NaN, so a cell the kernel
    leaves unwritten fails), the zeros off the operator's cells included."""
    from oracle import operators
    L = make()
    p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order)
    rng = np.random.default_rng(21)
    shape = L.f.shape
    for op, name in ((lgf.LAPLACIAN, "laplacian"), (lgf.GRADIENT, "gradient"), (lgf.CURL, "curl")):
        u = rng.normal(size=((3,) + shape) if op == lgf.CURL else shape)
        out_shape = shape if op == lgf.LAPLACIAN else (3,) + shape
        out = torch.full(out_shape, float("nan"), dtype=torch.float64, device="cuda")
        p.apply(op, torch.from_numpy(np.ascontiguousarray(u)).cuda(), out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref = operators.apply(L.blocks, L.levels, u, L.n_b, name)
        assert np.all(got[ref == 0.0] == 0.0), name
        assert rel_linf(got, ref) <= 1e-12, name
    u1 = torch.zeros(shape, dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):
        p.apply(7, u1, torch.zeros((3,) + shape, dtype=torch.float64, device="cuda"))
    p.close()
