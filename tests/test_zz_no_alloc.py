"""psp_solve_noalloc through the C ABI: the solve whose intermediates live in
the library's fixed device array gives bitwise the result of psp_solve (the
same kernels on the same layout), on consecutive calls where the second is
smaller than the first (the array keeps the first call's contents), in both
tiers; plans whose intermediates exceed the array are refused with
PSP_ENOMEM and leave nothing behind."""
import numpy as np
import pytest

from oracle import psp_oracle as O
from paper_2506_04489_amd import psp as B
from tests.gpu_util import announce, rel_max_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


@pytest.mark.parametrize("dtype,sizes", [("f64", (64, 32)), ("f32", (128, 48)), ("f64", (128, 96))])
def test_noalloc_matches_solve_on_consecutive_calls(dtype, sizes):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    for i, n in enumerate(sizes):
        h = 2.0 / n
        rng = np.random.default_rng(900 + 10 * i + n)
        rho_np = rng.standard_normal((n, n, n))
        rho = to_dev(rho_np, td)
        p = B.Plan(n, h, 40, dtype=dtype).precompute()
        want = p.solve(rho)
        got = torch.full_like(rho, float("nan"))
        torch.cuda.synchronize()
        p.solve_noalloc(rho, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (dtype, n)
        if n <= 64:
            e = rel_max_err(got.double().cpu().numpy(), O.solve(rho_np.astype(np.float32 if dtype == "f32" else
                                                                                np.float64).astype(np.float64),
                                                                 h, 40))
            assert e <= (1e-12 if dtype == "f64" else 1e-5), e
        p.close()


def test_noalloc_grid_plan_matches_solve():
    import torch
    ns, hs = (16, 24, 32), (0.1, 0.08, 0.07)
    rng = np.random.default_rng(7)
    rho = to_dev(rng.standard_normal(ns))
    p = B.Plan(ns, hs, 40).precompute()
    want = p.solve(rho)
    got = torch.empty_like(rho)
    p.solve_noalloc(rho, got)
    torch.cuda.synchronize()
    assert torch.equal(got, want)


def test_noalloc_refuses_plans_beyond_the_array():
    import torch
    n = 192                                   # FP64 intermediates of 359 MB > 128 MiB
    p = B.Plan(n, 2.0 / n, 40).precompute()
    rho = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    u = torch.empty_like(rho)
    with pytest.raises(B.PspError) as ei:
        p.solve_noalloc(rho, u)
    assert ei.value.status == -2              # PSP_ENOMEM
    # the refusal launched nothing: a following small no-alloc solve is exact
    m = 32
    q = B.Plan(m, 2.0 / m, 40).precompute()
    r = to_dev(np.random.default_rng(3).standard_normal((m, m, m)))
    got = torch.empty_like(r)
    q.solve_noalloc(r, got)
    torch.cuda.synchronize()
    assert torch.equal(got, q.solve(r))
