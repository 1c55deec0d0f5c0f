"""Batched launches and captured graphs on the GPU: bitwise equal to single
solves, and parity with the oracle."""
import numpy as np
import pytest

from oracle import psp_oracle as O
from paper_2506_04489_amd import densities as D
from paper_2506_04489_amd import psp as B
from tests.gpu_util import announce, rel_max_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def _setup(count, dtype, seed):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    items = D.batched_workload(count=count, seed=seed)
    plans = {}
    for it in items:
        if it.n not in plans:
            plans[it.n] = B.Plan(it.n, it.h, 40, dtype=dtype).precompute()
    rhos = [it.mixture.sample(it.n, it.h, it.x0, xp=torch, device="cuda").to(td).contiguous() for it in items]
    return items, plans, rhos


@pytest.fixture(params=["grouped", "persistent", "flat"])
def batch_mode(request):
    B.set_batch_mode(request.param)
    yield request.param
    B.set_batch_mode("grouped")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_mixed_sizes_bitwise_equal_to_single(dtype, batch_mode):
    import torch
    items, plans, rhos = _setup(24, dtype, D.BATCH_SEED)
    ps = [plans[it.n] for it in items]
    us = [torch.empty_like(r) for r in rhos]
    B.solve_batched(ps, rhos, us)
    torch.cuda.synchronize()
    for p, r, u in zip(ps, rhos, us):
        alone = p.solve(r)
        torch.cuda.synchronize()
        assert torch.equal(u, alone), p.n


def test_batched_parity_with_oracle(batch_mode):
    import torch
    items, plans, rhos = _setup(6, "f64", 7)
    ps = [plans[it.n] for it in items]
    us = [torch.empty_like(r) for r in rhos]
    B.solve_batched(ps, rhos, us)
    torch.cuda.synchronize()
    for it, r, u in zip(items, rhos, us):
        if it.n > 64:
            continue
        want = O.solve(r.cpu().numpy(), it.h, 40)
        e = rel_max_err(u.cpu().numpy(), want)
        print("batched n=%d E_par=%.3e" % (it.n, e))
        assert e <= 1e-12


def test_batched_repeated_calls_reuse_staging(batch_mode):
    import torch
    items, plans, rhos = _setup(10, "f64", 11)
    ps = [plans[it.n] for it in items]
    outs = []
    for rep in range(3):
        scaled = [r * (rep + 1) for r in rhos]
        us = [torch.empty_like(r) for r in rhos]
        B.solve_batched(ps, scaled, us)
        outs.append(us)
    torch.cuda.synchronize()
    for rep in range(3):
        for p, r, u in zip(ps, rhos, outs[rep]):
            assert torch.equal(u, p.solve(r * (rep + 1)))


def test_batched_more_batches_than_staging_slots(batch_mode):
    """Twelve batches queued back to back on one stream without a host wait:
    their tables go up through a ring of eight staging slots, so slots are
    reused while earlier batches are still queued; each result is bitwise
    that of single solves."""
    import torch
    items, plans, rhos = _setup(12, "f64", 23)
    ps = [plans[it.n] for it in items]
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    outs = []
    for k in range(1, 13):
        us = [torch.empty_like(r) for r in rhos[:k]]
        st.wait_stream(torch.cuda.current_stream())
        B.solve_batched(ps[:k], rhos[:k], us, stream=st)
        outs.append(us)
    st.synchronize()
    for us in outs:
        for p, r, u in zip(ps, rhos, us):
            assert torch.equal(u, p.solve(r))


def test_batched_rejects_mixed_dtypes():
    import torch
    p64 = B.Plan(16, 0.125, 40).precompute()
    p32 = B.Plan(16, 0.125, 40, dtype="f32").precompute()
    r64 = torch.zeros((16,) * 3, dtype=torch.float64, device="cuda")
    r32 = torch.zeros((16,) * 3, dtype=torch.float32, device="cuda")
    with pytest.raises(B.PspError):
        B.solve_batched([p64, p32], [r64, r32], [torch.empty_like(r64), torch.empty_like(r32)])


def test_graph_single_replays_match_eager():
    import torch
    n = 64
    h = 2.0 / n
    p = B.Plan(n, h, 40).precompute()
    rho = D.gaussian(n, h, -1.0, 0.15, xp=torch, device="cuda").contiguous()
    u = torch.empty_like(rho)
    g = B.Graph.capture(p, rho, u)
    for rep in range(4):
        rho.mul_(1.5).add_(0.01 * rep)          # eager work between replays
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        eager = p.solve(rho)
        torch.cuda.synchronize()
        assert torch.equal(u, eager), rep
    g.close()


def test_graph_batched_replays_match_eager(batch_mode):
    import torch
    items, plans, rhos = _setup(12, "f64", 13)
    ps = [plans[it.n] for it in items]
    us = [torch.empty_like(r) for r in rhos]
    g = B.Graph.capture_batched(ps, rhos, us)
    B.set_batch_mode("grouped")       # replays keep the mode of their capture
    for rep in range(3):
        for r in rhos:
            r.mul_(-1.25)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for p, r, u in zip(ps, rhos, us):
            assert torch.equal(u, p.solve(r)), (rep, p.n)
    g.close()


@pytest.mark.parametrize("mode", ["persistent", "flat"])
def test_persistent_batch_covers_every_size_and_large_members(mode):
    """Every padded length up to 256 (radix-2 and radix-3 plans, alternative
    radix plans) in one persistent (or flat) batch, with n = 192 members
    taking the grouped launches in the same call."""
    import torch
    B.set_batch_mode(mode)
    try:
        sizes = [4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192]
        ps, rhos = [], []
        for i, n in enumerate(sizes):
            p = B.Plan(n, 2.0 / n, 40).precompute()
            if n in (64, 128):
                p.set_shape([1] * 5, [0] * 5)
            ps.append(p)
            g = torch.Generator().manual_seed(31 + i)
            rhos.append(torch.randn((n,) * 3, generator=g, dtype=torch.float64).cuda())
        us = [torch.empty_like(r) for r in rhos]
        B.solve_batched(ps, rhos, us)
        torch.cuda.synchronize()
        for p, r, u in zip(ps, rhos, us):
            alone = p.solve(r)
            torch.cuda.synchronize()
            assert torch.equal(u, alone), p.n
    finally:
        B.set_batch_mode("grouped")
