"""Launch shapes and the autotuner on the GPU: every tile choice gives
bitwise the same result, every (radix plan, tile) stays within the parity
tolerance of the oracle's whole-grid solve at every size, the autotuner's pick is valid and used, and batches that mix
shapes give each member its own single-solve result."""
import numpy as np
import pytest

from oracle import psp_oracle as O
from paper_2506_04489_amd import densities as D
from paper_2506_04489_amd import psp as B
from tests.gpu_util import TILES, announce, rel_max_err, shape_rounds

pytestmark = pytest.mark.gpu

@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def _density(n, seed, dtype):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    g = torch.Generator().manual_seed(seed)
    return torch.randn((n,) * 3, generator=g, dtype=torch.float64).to(td).cuda()


@pytest.mark.parametrize("n,dtype", [(48, "f64"), (64, "f64"), (64, "f32"), (96, "f64"), (128, "f64"),
                                     (192, "f64"), (192, "f32"), (384, "f64"), (384, "f32"), (256, "f64")])
def test_every_shape_matches(n, dtype):
    import torch
    h = 2.0 / n
    rho = _density(n, 100 + n, dtype)
    p = B.Plan(n, h, 40, dtype=dtype).precompute()
    p.set_shape([0] * 5, [0] * 5)
    ref = p.solve(rho)
    torch.cuda.synchronize()
    # every shape against the oracle's whole-grid solve (its C naive FFT)
    want = O.solve(rho.double().cpu().numpy(), h, 40)
    tol = 1e-12 if dtype == "f64" else 1e-5
    for plan, tile in shape_rounds(n):
        p.set_shape(plan, tile)
        u = p.solve(rho)
        torch.cuda.synchronize()
        if not any(plan):
            assert torch.equal(u, ref), (plan, tile)
        elif dtype == "f64":
            e_def = rel_max_err(u.cpu().numpy(), ref.cpu().numpy())
            print("n=%d %s plan=%s tile=%s vs default %.2e" % (n, dtype, plan, tile, e_def))
            assert e_def <= 1e-13
        e = rel_max_err(u.double().cpu().numpy(), want)
        print("n=%d %s plan=%s tile=%s vs oracle %.2e" % (n, dtype, plan, tile, e))
        assert e <= tol, (plan, tile, e)


def test_autotune_picks_a_valid_shape_and_uses_it():
    import torch
    n, h = 64, 2.0 / 64
    old = B.tuning_get(n, "f64")
    try:
        p = B.Plan(n, h, 40).precompute()
        res = p.autotune(reps=3)
        print("autotune n=64:", res)
        assert p.shape() == (res["plan"], res["tile"])
        assert B.tuning_get(n, "f64") == (res["plan"], res["tile"])
        assert all(0 <= t < c for t, c in zip(res["tile"], TILES))
        assert all(x > 0 for x in res["pass_ms"])
        q = B.Plan(n, h, 40).precompute()           # new plans start from the table
        assert q.shape() == p.shape()
        rho = D.gaussian(n, h, -1.0, 0.15, xp=torch, device="cuda").contiguous()
        u = p.solve(rho)
        torch.cuda.synchronize()
        want = O.solve(rho.cpu().numpy(), h, 40)
        assert rel_max_err(u.cpu().numpy(), want) <= 1e-12
    finally:
        B.tuning_set(n, "f64", *old)


def test_batch_mixing_shapes_bitwise_equal_to_single():
    import torch
    n, h = 64, 2.0 / 64
    pa = B.Plan(n, h, 40).precompute().set_shape([0] * 5, [0] * 5)
    pb = B.Plan(n, h, 40).precompute().set_shape([1, 0, 1, 0, 1], [1, 1, 1, 1, 2])
    pc = B.Plan(32, 2.0 / 32, 40).precompute().set_shape([0] * 5, [2, 1, 0, 1, 1])
    ps = [pa, pb, pc, pb, pa]
    rhos = [_density(p.n, 7 + i, "f64") for i, p in enumerate(ps)]
    us = [torch.empty_like(r) for r in rhos]
    B.solve_batched(ps, rhos, us)
    torch.cuda.synchronize()
    for p, r, u in zip(ps, rhos, us):
        alone = p.solve(r)
        torch.cuda.synchronize()
        assert torch.equal(u, alone), p.shape()
