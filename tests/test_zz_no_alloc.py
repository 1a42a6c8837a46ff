"""The allocation-free solve (lgf_solve_noalloc): the same plan solved through it and through
lgf_solve gives the same result bit for bit, on two calls in a row on one stream (the second with
a smaller layout, so the static workspace holds the first call's contents when the second
starts), and a plan whose workspace exceeds the static array is refused with LGF_ENOMEM."""
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
    return m


def test_noalloc_equals_solve_on_two_calls(lgf):
    big = workloads.uniform_mixture(nblk=3, n_b=16, n_gauss=3, seed=22, interp_order=8)   # 110592 unknowns
    small = workloads.uniform_mixture(nblk=3, n_b=8, n_gauss=3, seed=9, interp_order=6)   # 13824 unknowns
    cases = []
    for L, precision, dc in ((big, 1, 1), (small, 0, 0)):
        p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, precision, dc)
        assert p.info()["workspace_bytes"] <= lgf.SCRATCH_BYTES
        f = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
        ref = torch.zeros_like(f)
        p.solve(f, ref)
        torch.cuda.synchronize()
        cases.append((L, p, f, ref.cpu().numpy()))
    s = torch.cuda.Stream()
    outs = []
    for L, p, f, _ in cases:                  # two calls in a row, the second smaller
        u = torch.full_like(f, float("nan"))
        p.solve_noalloc(f, u, stream=s)
        outs.append(u)
    s.synchronize()
    for (L, p, f, ref), u in zip(cases, outs):
        got = u.cpu().numpy()
        assert np.array_equal(got, ref)
        oracle = fmm.flgf(L.blocks, L.f, L.n_b, L.interp_order)
        tol = 1e-12 if p.precision == 0 else 1e-6
        assert np.abs(got - oracle).max() <= tol * np.abs(oracle).max()
    for _, p, _, _ in cases:
        p.close()


def test_noalloc_refuses_a_plan_larger_than_the_static_workspace(lgf):
    L = workloads.uniform_mixture(nblk=4, n_b=16, n_gauss=2, seed=3, interp_order=6)
    p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order)
    assert p.info()["workspace_bytes"] > lgf.SCRATCH_BYTES
    f = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
    u = torch.zeros_like(f)
    with pytest.raises(lgf.LgfError) as e:
        p.solve_noalloc(f, u)
    assert e.value.code == -3
    p.close()
