"""The benchmark-sized workloads on the GPU, through the C ABI.

* uniform 8^3 blocks of 16^3 (2,097,152 unknowns): FP64 against the FP64 oracle (1e-12), FP32
  against the oracle (1e-6) and FP32 + one defect-correction iteration against the oracle's
  defect correction with FP64 inner solves (1e-6);
* the torus layout (8^3 base blocks of 16^3, two refinement levels): FP64 and FP32 against the
  FP64 oracle's solve at sampled cells (tests/golden/torus_oracle_samples.txt; the oracle's
  multi-level solve at this size takes over a minute on one core), the FP32 forms against the
  FP64 GPU solve and its FP64 defect correction (1e-6), and second-order convergence of the
  FP32 + defect-correction solve to the manufactured solution;
* 64 independent layouts solved in shared launches: equal to each solved alone, and the
  smallest against the oracle;
* a Poisson-arrival request stream through the server: every result equal to its solve alone,
  and the smallest served layouts against the oracle.
"""
import importlib.util
import os
import time

import numpy as np
import pytest

from oracle import dc as dc_oracle, fmm, multires
from paper_1911_10228_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def lgf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_10228_amd import lgf as m
    m.init()
    return m


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def solve(lgf, L, precision, dc, f=None, base_level=0, plan=None):
    p = plan or lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, dc,
                         base_level=base_level)
    fd = torch.from_numpy(np.ascontiguousarray(L.f if f is None else f)).cuda()
    u = torch.zeros_like(fd)
    p.solve(fd, u)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def test_uniform_full_size(lgf):
    L = workloads.uniform_mixture()
    print(f"case: {L.name}", flush=True)
    ref = fmm.flgf(L.blocks, L.f, L.n_b, L.interp_order)
    assert rel(solve(lgf, L, 0, 0), ref) <= 1e-12
    assert rel(solve(lgf, L, 0, 0, base_level=1), ref) <= 1e-12
    assert rel(solve(lgf, L, 1, 0), ref) <= 1e-6
    mask = multires.residual_mask(L.blocks, L.levels, L.n_b)
    r = np.where(mask, L.f - multires.apply_laplace(L.blocks, L.levels, ref, L.n_b), 0.0)
    ref1 = ref + fmm.flgf(L.blocks, r, L.n_b, L.interp_order)
    assert rel(solve(lgf, L, 1, 1), ref1) <= 1e-6
    # the benchmark's configuration: autotuned plans, repeated solves replaying a captured graph
    for precision, dc, want, tol in ((1, 1, ref1, 1e-6), (0, 0, ref, 1e-12)):
        p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, dc, autotune=1)
        fd = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
        for rep in range(3):
            u = torch.zeros_like(fd)
            p.solve(fd, u)
            torch.cuda.synchronize()
            assert rel(u.cpu().numpy(), want) <= tol, f"precision {precision} solve {rep}"
        p.close()


def test_torus_full_size(lgf):
    L = workloads.torus()
    print(f"case: {L.name}, {len(L.blocks)} blocks", flush=True)
    u64 = solve(lgf, L, 0, 0)
    assert rel(solve(lgf, L, 0, 0, base_level=1), u64) <= 1e-12
    assert rel(solve(lgf, L, 1, 0), u64) <= 1e-6
    # one FP64 defect-correction step of the FP64 solve: the FP32 form's fixed point
    mask = multires.residual_mask(L.blocks, L.levels, L.n_b)
    r = np.where(mask, L.f - multires.apply_laplace(L.blocks, L.levels, u64, L.n_b), 0.0)
    u1 = u64 + solve(lgf, L, 0, 0, f=r)
    assert rel(solve(lgf, L, 1, 1), u1) <= 1e-6


def torus_oracle_samples():
    """(input digest, max |u| of the oracle's solve, [(block, cell, u)]) from the fixture written
    by tests/golden/make_torus_samples.py, and that script's input digest function."""
    spec = importlib.util.spec_from_file_location("make_torus_samples", os.path.join(GOLDEN, "make_torus_samples.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    digest, umax, rows = None, None, []
    for line in open(os.path.join(GOLDEN, "torus_oracle_samples.txt")):
        p = line.split()
        if not p or p[0].startswith("#"):
            continue
        if p[0] == "input_sha256":
            digest = p[1]
        elif p[0] == "max_abs_u":
            umax = float(p[1])
        else:
            rows.append((int(p[0]), int(p[1]), float(p[2])))
    return digest, umax, rows, mk.input_digest


def test_torus_full_size_matches_oracle_samples(lgf):
    """The full torus layout against the FP64 oracle's multi-resolution solve (Algorithm 2) at
    510 sampled cells, 170 per refinement level: FP64 to 1e-12 and FP32 without defect
    correction to 1e-6 of max |u|."""
    L = workloads.torus()
    digest, umax, rows, input_digest = torus_oracle_samples()
    assert digest == input_digest(L), "torus input changed: rerun tests/golden/make_torus_samples.py"
    b = np.array([r[0] for r in rows])
    c = np.array([r[1] for r in rows])
    ref = np.array([r[2] for r in rows])
    n3 = L.n_b ** 3
    print(f"case: {L.name} FP64 against {len(rows)} oracle samples", flush=True)
    u64 = solve(lgf, L, 0, 0).reshape(len(L.blocks), n3)
    e64 = np.abs(u64[b, c] - ref).max() / umax
    print(f"FP64: {e64:.2e} of max |u|", flush=True)
    assert e64 <= 1e-12
    print(f"case: {L.name} FP32 against {len(rows)} oracle samples", flush=True)
    u32 = solve(lgf, L, 1, 0).reshape(len(L.blocks), n3)
    e32 = np.abs(u32[b, c] - ref).max() / umax
    print(f"FP32: {e32:.2e} of max |u|", flush=True)
    assert e32 <= 1e-6


def test_torus_second_order_convergence(lgf):
    """Manufactured source (the torus' analytic Laplacian): the error of the FP32 + defect
    correction solve against the torus itself falls by ~4x per halving of the cell size
    (domain 32, 64, 128 base cells)."""
    errs = []
    for nblk, n_b in ((4, 8), (8, 8), (8, 16)):
        L = workloads.torus(nblk=nblk, n_b=n_b, manufactured=True)
        print(f"case: {L.name}", flush=True)
        u = solve(lgf, L, 1, 1)
        errs.append(np.abs(u - L.exact).max() / np.abs(L.exact).max())
    order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("errors", errs, "orders", order, flush=True)
    # the coarsest grid resolves the torus core (0.03 L) with about one cell: pre-asymptotic
    assert errs[-1] < 1e-2 and order[-1] >= 1.8 and order[0] >= 1.5


def test_vortex_ring_vector_second_order(lgf):
    """The paper's manufactured solution (Sec. 3, Convergence subsection: the vortex ring
    R = 0.125, c1 = 1e3, c2 = 10)
    as a vector Poisson problem: both Cartesian streamfunction components through one
    VectorPlan (FP32 + defect correction), on a uniform grid (16^3 blocks) and with one
    refinement level around the ring (8^3 blocks): the errors against psi_x and psi_y fall at
    second order, and the two components (mirror images of each other) have the same error."""
    for n_b, n_levels in ((16, 1), (8, 2)):
        errs = []
        for nblk in (2, 4, 8):
            L = workloads.vortex_ring(nblk=nblk, n_b=n_b, n_levels=n_levels, interp_order=8)
            print(f"case: {L.name}", flush=True)
            vp = lgf.VectorPlan(L.blocks, L.levels, L.n_b, L.interp_order, components=2,
                                precision=1, dc_iters=1)
            f = torch.from_numpy(np.ascontiguousarray(np.stack([L.f, L.meta["f_y"]]))).cuda()
            u = torch.zeros_like(f)
            vp.solve(f, u)
            torch.cuda.synchronize()
            got = u.cpu().numpy()
            vp.close()
            ex = np.abs(got[0] - L.exact).max() / np.abs(L.exact).max()
            ey = np.abs(got[1] - L.meta["exact_y"]).max() / np.abs(L.meta["exact_y"]).max()
            assert abs(ex - ey) <= 1e-3 * ex
            errs.append(ex)
        order = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        print("errors", errs, "orders", order, flush=True)
        assert order[-1] >= 1.8 and errs[-1] < 1e-2


def test_batch_of_64_layouts(lgf):
    Ls = workloads.batch()
    plans = [lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, 1, 1, autotune=1) for L in Ls]
    fs = [torch.from_numpy(np.ascontiguousarray(L.f)).cuda() for L in Ls]
    us = [torch.zeros_like(f) for f in fs]
    lgf.solve_batch(plans, fs, us)
    torch.cuda.synchronize()
    for k, (L, p) in enumerate(zip(Ls, plans)):
        alone = solve(lgf, L, 1, 1, plan=p)
        assert np.array_equal(us[k].cpu().numpy(), alone), f"layout {k}: {L.name}"
    small = sorted(range(len(Ls)), key=lambda k: Ls[k].unknowns)[:3]
    for k in small:
        L = Ls[k]
        its = dc_oracle.solve_dc(L.blocks, L.levels, L.f, L.n_b, L.interp_order, iters=1,
                                 dtype=np.float64)
        assert rel(us[k].cpu().numpy(), its[1]) <= 1e-6, L.name


def test_serving_poisson_stream(lgf):
    pool = workloads.request_pool(count=8, max_unknowns=1 << 21)
    plans = [lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, 1, 1) for L in pool]
    fs = [torch.from_numpy(np.ascontiguousarray(L.f)).cuda() for L in pool]
    alone = [solve(lgf, L, 1, 1, plan=p) for L, p in zip(pool, plans)]
    rng = np.random.default_rng(7)
    times, _ = workloads.arrivals(seed=5, count=48, rate_hz=400.0)
    which = rng.integers(0, len(pool), size=len(times))
    srv = lgf.Server(hbm_budget=sum(p.info()["workspace_bytes"] for p in plans) // 2,
                     stream=torch.cuda.Stream())
    outs, ids = [], []
    t0 = time.perf_counter()
    for t, k in zip(times, which):
        while time.perf_counter() - t0 < t:
            time.sleep(1e-4)
        u = torch.zeros_like(fs[k])
        outs.append(u)
        ids.append(srv.submit(plans[k], fs[k], u))
    srv.wait_all()
    st = srv.stats()
    print("serving", st, flush=True)
    assert st["completed"] == len(ids) and st["p99_us"] >= st["p50_us"] > 0
    for u, k in zip(outs, which):
        assert np.array_equal(u.cpu().numpy(), alone[k])
    srv.close()
    # a sample of the served layouts against the oracle's one-step defect correction
    for k in sorted(set(which.tolist()), key=lambda k: pool[k].unknowns)[:2]:
        L = pool[k]
        its = dc_oracle.solve_dc(L.blocks, L.levels, L.f, L.n_b, L.interp_order, iters=1,
                                 dtype=np.float64)
        assert rel(alone[k], its[1]) <= 1e-6, L.name
