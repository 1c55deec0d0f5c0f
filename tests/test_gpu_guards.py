"""Out-of-bounds writes: with guard bands around every workspace buffer,
solves of every launch shape, radix plan, chunking and grouping leave the
bands untouched."""
import pytest

from paper_2506_04489_amd import psp as B
from tests.gpu_util import announce, shape_rounds

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


@pytest.mark.parametrize("n,dtype", [(4, "f64"), (6, "f64"), (24, "f32"), (48, "f64"), (96, "f32"),
                                     (128, "f64"), (192, "f64"), (256, "f32"), (384, "f64")])
def test_passes_stay_inside_their_workspace(n, dtype):
    import torch
    B.debug_guards(True)
    try:
        td = torch.float64 if dtype == "f64" else torch.float32
        g = torch.Generator().manual_seed(n)
        rho = torch.randn((n,) * 3, generator=g, dtype=torch.float64).to(td).cuda()
        p = B.Plan(n, 2.0 / n, 40, dtype=dtype).precompute()
        for plan, tile in shape_rounds(n):
            p.set_shape(plan, tile)
            p.solve(rho)
        torch.cuda.synchronize()
        assert p.guards_intact(), "shapes"
        p.set_shape([0] * 5, [0] * 5)
        if n <= 128:
            p.solve_padded_debug(rho)            # the uncropped passes, same workspace
            assert p.guards_intact(), "uncropped"
        for k3_tiles, group in ((3, 0), (0, max(1, n // 3))):
            p.set_tuning(k3_tiles, group)        # new (guarded) workspaces
            p.solve(rho)
            torch.cuda.synchronize()
            assert p.guards_intact(), (k3_tiles, group)
            # a shrunk workspace cannot hold the uncropped passes
            with pytest.raises(B.PspError, match="default tuning"):
                p.solve_padded_debug(rho)
        p.set_tuning(0, 0)
    finally:
        B.debug_guards(False)
