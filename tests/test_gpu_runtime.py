"""Runtime features on the GPU: captured-graph replays, the launch-shape autotuner, batched solves
and the continuous-batching server.  Every result is compared with an eager single solve of the
same plan (bitwise where the arithmetic is identical) and with the FP64 oracle."""
import numpy as np
import pytest

from oracle import dc as dc_oracle, fmm, multires
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


def field(L):
    return torch.from_numpy(np.ascontiguousarray(L.f)).cuda()


def eager(lgf, plan, f):
    """Solve on the legacy default stream (never captured into a graph)."""
    u = torch.zeros_like(f)
    lgf.load().lgf_solve(plan.handle, lgf._ptr(f), lgf._ptr(u), None)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def small_cases():
    return [workloads.uniform_mixture(nblk=5, n_b=8, n_gauss=4, seed=21, interp_order=6),
            workloads.uniform_mixture(nblk=3, n_b=16, n_gauss=3, seed=22, interp_order=8)]


@pytest.mark.parametrize("precision,dc", [(0, 0), (1, 1)])
def test_graph_replays_equal_eager(lgf, precision, dc):
    L = small_cases()[0]
    p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, dc)
    f = field(L)
    ref = eager(lgf, p, f)
    s = torch.cuda.Stream()
    u = torch.zeros_like(f)
    for rep in range(4):
        with torch.cuda.stream(s):
            u.zero_()                      # a fill kernel, not a memset, between replays
            p.solve(f, u, stream=s)
        s.synchronize()
        junk = torch.randn(1 << 16, device="cuda").sum()   # the program's own eager work
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), ref), f"replay {rep} differs"
        del junk


def test_autotuned_plan_matches(lgf):
    for L in small_cases():
        ref = fmm.flgf(L.blocks, L.f, L.n_b, L.interp_order)
        for precision, tol in ((0, 1e-12), (1, 1e-6)):
            p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, 0)
            a = eager(lgf, p, field(L))
            opt = lgf.Options(precision, 0, 1, 0, 0)
            import ctypes as C
            h = C.c_void_p()
            b = np.ascontiguousarray(L.blocks, dtype=np.int32)
            lv = np.ascontiguousarray(L.levels, dtype=np.int32)
            lgf._check(lgf.load().lgf_plan(b.ctypes.data, lv.ctypes.data, len(b), L.n_b,
                                           L.interp_order, C.byref(opt), C.byref(h)), "lgf_plan")
            q = lgf.Plan.__new__(lgf.Plan)
            q._h, q.n_b, q.nblocks, q.precision = h, L.n_b, len(b), precision
            c = eager(lgf, q, field(L))
            assert np.abs(c - ref).max() <= tol * np.abs(ref).max()
            assert np.abs(c - a).max() <= tol * np.abs(ref).max()
            q.close()


def test_every_mac_shape_matches_oracle(lgf):
    """Every launch shape of the tile MAC, forced on the plan, against the FP64 oracle: FP64
    coarse levels with rows of 8 (level 1 of 16^3 blocks) and of 4 targets (small levels: also the
    LDS form, shape 16), and the FP32 per-block base level."""
    big = workloads.uniform_mixture(nblk=16, n_b=8, n_gauss=6, seed=23, interp_order=6)
    small = small_cases()[0]
    for L, precision, base, tol in ((big, 0, 0, 1e-12), (small, 0, 0, 1e-12), (small, 1, 1, 1e-6)):
        ref = fmm.flgf(L.blocks, L.f, L.n_b, L.interp_order)
        p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, 0, base_level=base)
        f = field(L)
        for shape in (1, 2, 4, 6, 8, 16, 0):
            print(f"case {len(L.blocks)} blocks precision {precision} base {base} shape {shape}", flush=True)
            p.set_mac_shape(shape)
            u = eager(lgf, p, f)
            assert np.abs(u - ref).max() <= tol * np.abs(ref).max(), f"shape {shape}"
        p.close()


def test_every_near_shape_matches_oracle(lgf):
    """Every launch shape of the base-level super-block MAC, forced on an autotuned plan, against
    the FP64 oracle (FP64 spectra: rows of 2, 4 and 8; FP32: also tiles, one chunk per
    workgroup or pipelined over runs of chunks; both: the fused form of compact tiles of 2 x 2
    and 2 x 4 rows, with the super-block transforms switched to line-major planes)."""
    L = workloads.uniform_mixture(nblk=6, n_b=8, n_gauss=4, seed=31, interp_order=6)
    ref = fmm.flgf(L.blocks, L.f, L.n_b, L.interp_order)
    f = field(L)
    for precision, shapes, tol in ((0, (2, 4, 8, 21, 23, 42, 44), 1e-12),
                                   (1, (20, 22, 21, 23, 2, 4, 8, 42, 44), 1e-6)):
        p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, 0, autotune=1)
        for shape in shapes + (0,):
            print(f"case precision {precision} near shape {shape}", flush=True)
            p.set_near_shape(shape)
            u = eager(lgf, p, f)
            assert np.abs(u - ref).max() <= tol * np.abs(ref).max(), f"shape {shape}"
        p.close()


def test_server_results_equal_alone(lgf):
    Ls = small_cases() + [workloads.uniform_gaussian()]
    plans = [lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, 1, 1) for L in Ls]
    fs = [field(L) for L in Ls]
    alone = [eager(lgf, p, f) for p, f in zip(plans, fs)]
    srv = lgf.Server(hbm_budget=0, stream=torch.cuda.Stream())
    outs, ids = [], []
    for rep in range(3):                      # the same plan arrives again while in flight
        for p, f in zip(plans, fs):
            u = torch.zeros_like(f)
            outs.append(u)
            ids.append(srv.submit(p, f, u))
    srv.wait_all()
    st = srv.stats()
    assert st["completed"] == len(ids) and st["p99_us"] >= st["p50_us"] > 0
    for k, u in enumerate(outs):
        assert srv.poll(ids[k])
        assert np.array_equal(u.cpu().numpy(), alone[k % len(plans)])
    srv.close()


def test_server_budget_admission(lgf):
    Ls = small_cases()
    plans = [lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, 0, 0) for L in Ls]
    budget = max(p.info()["workspace_bytes"] for p in plans)   # the larger runs alone
    fs = [field(L) for L in Ls]
    srv = lgf.Server(hbm_budget=budget, stream=torch.cuda.Stream())
    us = [torch.zeros_like(f) for f in fs]
    ids = [srv.submit(p, f, u) for p, f, u in zip(plans, fs, us)]
    srv.wait_all()
    for p, f, u in zip(plans, fs, us):
        assert np.array_equal(u.cpu().numpy(), eager(lgf, p, f))
    srv.close()


def test_multires_torus_reduced_matches_oracle(lgf):
    L = workloads.torus(nblk=4, n_b=8, n_levels=3, interp_order=6)
    p = lgf.Plan(L.blocks, L.levels, L.n_b, 6, 0, 0)
    u = eager(lgf, p, field(L))
    ref = multires.solve(L.blocks, L.levels, L.f, L.n_b, 6)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()
    p32 = lgf.Plan(L.blocks, L.levels, L.n_b, 6, 1, 0)
    u32 = eager(lgf, p32, field(L))
    assert np.abs(u32 - ref).max() <= 1e-6 * np.abs(ref).max()
    its = dc_oracle.solve_dc(L.blocks, L.levels, L.f, L.n_b, 6, iters=1, dtype=np.float64)
    p32 = lgf.Plan(L.blocks, L.levels, L.n_b, 6, 1, 1)
    u32 = eager(lgf, p32, field(L))
    assert np.abs(u32 - its[1]).max() <= 1e-6 * np.abs(its[1]).max()
