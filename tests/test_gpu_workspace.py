"""Relocatable solve workspaces on the GPU: a plan's work items are placed into any device range
(per-stream workspaces of lgf_solve, server slots), so several solves of one plan run at once,
the server bounds its memory by its budget, and plans can come from the server's layout-keyed
cache.  Every result is compared bit for bit with the same plan solved alone; the poisoned
workspace (NaN bytes wherever the solve does not clear) shows that a solve reads nothing it has
not written."""
import numpy as np
import pytest

from oracle import fmm
from paper_1911_10228_amd import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lgf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1911_10228_amd import lgf as m
    m.init()
    yield m
    m.workspace_poison(False)


def field(L, scale=1.0):
    return torch.from_numpy(np.ascontiguousarray(scale * L.f)).cuda()


def alone(lgf, plan, f):
    """Solve on the legacy default stream (never captured into a graph)."""
    u = torch.zeros_like(f)
    lgf._check(lgf.load().lgf_solve(plan.handle, lgf._ptr(f), lgf._ptr(u), None), "lgf_solve")
    torch.cuda.synchronize()
    return u.cpu().numpy()


def two_level8():
    base = workloads.box_blocks(4, 4, 4)
    fine = workloads.box_blocks(4, 4, 4, origin=(2, 2, 2))
    blocks = np.concatenate([base, fine]).astype(np.int32)
    levels = np.concatenate([np.zeros(64, np.int32), np.ones(64, np.int32)])
    pos = workloads.cell_centres(blocks, levels, 8)
    f = workloads.gaussian_mixture(pos, [(15.5,) * 3], [2.4], [1.0])
    return workloads.Layout(blocks, levels, 8, f, 6)


CASES = [
    ("uniform 5^3 x 8^3 FP64", lambda: workloads.uniform_mixture(nblk=5, n_b=8, n_gauss=4, seed=21, interp_order=6),
     0, 0, 0),
    ("uniform 3^3 x 16^3 FP32 + 1 DC", lambda: workloads.uniform_mixture(nblk=3, n_b=16, n_gauss=3, seed=22,
                                                                        interp_order=8), 1, 1, 0),
    ("two-level 8^3 FP64", two_level8, 0, 0, 0),
    ("two-level 8^3 FP32 + 2 DC", two_level8, 1, 2, 0),
    ("two-level 8^3 FP64 per-block base", two_level8, 0, 0, 1),
]


@pytest.mark.parametrize("name,make,precision,dc,base", CASES, ids=[c[0] for c in CASES])
def test_poisoned_workspace_gives_the_same_result(lgf, name, make, precision, dc, base):
    L = make()
    p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, dc, base_level=base)
    f = field(L)
    ref = alone(lgf, p, f)
    lgf.workspace_poison(True)
    try:
        s = torch.cuda.Stream()              # a new stream: a new workspace, bound poisoned
        u = torch.zeros_like(f)
        p.solve(f, u, stream=s)
        s.synchronize()
    finally:
        lgf.workspace_poison(False)
    got = u.cpu().numpy()
    assert np.all(np.isfinite(got)), name
    assert np.array_equal(got, ref), name
    p.close()


def test_concurrent_solves_of_one_plan(lgf):
    """Two solves of one plan in flight at once on two streams, each on its own workspace."""
    L = workloads.uniform_mixture(nblk=4, n_b=16, n_gauss=4, seed=5, interp_order=8)
    p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, 1, 1)
    fa, fb = field(L), field(L, -0.5)
    ra, rb = alone(lgf, p, fa), alone(lgf, p, fb)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ua, ub = torch.zeros_like(fa), torch.zeros_like(fb)
    for rep in range(3):
        with torch.cuda.stream(sa):
            ua.zero_()
            p.solve(fa, ua, stream=sa)
        with torch.cuda.stream(sb):
            ub.zero_()
            p.solve(fb, ub, stream=sb)
        torch.cuda.synchronize()
        assert np.array_equal(ua.cpu().numpy(), ra), rep
        assert np.array_equal(ub.cpu().numpy(), rb), rep
    p.close()


def test_batch_with_one_plan_several_times(lgf):
    """lgf_solve_batch with one plan three times (a vector field's components): each occurrence
    on its own workspace, each result equal to its solve alone."""
    L = workloads.uniform_mixture(nblk=3, n_b=8, n_gauss=3, seed=41, interp_order=6)
    p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order)
    fs = [field(L), field(L, 2.0), field(L, -1.0) + 0.25]
    refs = [alone(lgf, p, f) for f in fs]
    us = [torch.zeros_like(f) for f in fs]
    lgf.solve_batch([p, p, p], fs, us)
    torch.cuda.synchronize()
    for r, u in zip(refs, us):
        assert np.array_equal(u.cpu().numpy(), r)
    p.close()


def test_server_budget_bounds_the_slots(lgf):
    """With a budget that fits k = 2 workspaces of the plan, at most 2 requests are admitted at
    once (six of one plan arrive together), the server takes no more memory than the budget, and
    every result equals the plan's solve alone."""
    L = workloads.uniform_mixture(nblk=4, n_b=16, n_gauss=4, seed=6, interp_order=8)
    p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, 1, 1)
    need = p.info()["workspace_bytes"]
    k = 2
    budget = k * ((need + 255) // 256 * 256) + 4096
    fs = [field(L, 1.0 + 0.25 * i) for i in range(6)]
    refs = [alone(lgf, p, f) for f in fs]
    srv = lgf.Server(hbm_budget=budget, stream=torch.cuda.Stream())
    us = [torch.zeros_like(f) for f in fs]
    ids = [srv.submit(p, f, u) for f, u in zip(fs, us)]
    srv.wait_all()
    info = srv.info()
    assert all(srv.poll(i) for i in ids)
    assert 1 <= info["peak_slots"] <= k, info
    assert info["reserved_bytes"] <= budget and info["peak_in_use_bytes"] <= budget, info
    assert info["slots"] == 0 and info["in_use_bytes"] == 0, info
    for r, u in zip(refs, us):
        assert np.array_equal(u.cpu().numpy(), r)
    srv.close()
    p.close()


def test_server_reuses_slots_across_plans_and_caches_layouts(lgf):
    """Requests by layout through the server's plan cache, with a budget that makes different
    plans take turns in the same memory (slots re-bound to another plan's items), on poisoned
    workspaces: each layout is planned once, and every result equals a caller-owned plan of the
    same layout solved alone."""
    Ls = [workloads.uniform_mixture(nblk=3, n_b=16, n_gauss=3, seed=22, interp_order=8), two_level8(),
          workloads.uniform_gaussian()]
    plans = [lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, 1, 1) for L in Ls]
    fs = [field(L) for L in Ls]
    refs = [alone(lgf, p, f) for p, f in zip(plans, fs)]
    budget = max(p.info()["workspace_bytes"] for p in plans) + 4096
    lgf.workspace_poison(True)
    try:
        srv = lgf.Server(hbm_budget=budget, stream=torch.cuda.Stream())
        outs, ids = [], []
        for rep in range(3):
            for i, L in enumerate(Ls):
                u = torch.zeros_like(fs[i])
                outs.append((i, u))
                ids.append(srv.submit_layout(L.blocks, L.levels, L.n_b, L.interp_order, fs[i], u, 1, 1))
        srv.wait_all()
        info = srv.info()
    finally:
        lgf.workspace_poison(False)
    assert all(srv.poll(i) for i in ids)
    assert info["plan_misses"] == len(Ls) and info["plan_hits"] == 2 * len(Ls), info
    assert info["plans_cached"] == len(Ls) and info["plan_ms_max"] > 0, info
    assert info["reserved_bytes"] <= budget, info
    for i, u in outs:
        assert np.array_equal(u.cpu().numpy(), refs[i]), i
    st = srv.stats()
    assert st["completed"] == len(ids)
    srv.close()
    for p in plans:
        p.close()


def test_server_rejects_a_request_larger_than_its_budget(lgf):
    L = workloads.uniform_mixture(nblk=3, n_b=8, n_gauss=2, seed=3, interp_order=6)
    p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order)
    srv = lgf.Server(hbm_budget=p.info()["workspace_bytes"] // 2, stream=torch.cuda.Stream())
    f = field(L)
    u = torch.zeros_like(f)
    rid = srv.submit(p, f, u)
    with pytest.raises(lgf.LgfError):
        srv.wait_all()
    with pytest.raises(lgf.LgfError):
        srv.poll(rid)
    srv.close()
    # the plan still solves, and matches the oracle
    ref = fmm.flgf(L.blocks, L.f, L.n_b, L.interp_order)
    got = alone(lgf, p, f)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    p.close()
