"""Unequal point counts per axis on the GPU (psp_plan_create_grid): every
pass at its own axis's padded length, the per-axis multiplier octant, and
the solve against the oracle; graph capture; batches mixing grids and
cubes; entry points that need equal counts refuse such plans."""
import numpy as np
import pytest

from oracle import closed_forms as C
from oracle import psp_oracle as O
from paper_2506_04489_amd import psp as B
from tests.gpu_util import announce, rel_max_err, to_dev

pytestmark = pytest.mark.gpu

HS = (0.11, 0.17, 0.29)


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


@pytest.mark.parametrize("ns", [(16, 24, 32), (32, 12, 8), (6, 48, 16)])
def test_grid_multiplier(ns):
    p = B.Plan(ns, HS, 40).precompute()
    m = p.multiplier()
    su = O.setup(ns, HS, 40)
    assert m.shape == su.m.shape
    err = np.max(np.abs(m - su.m)) / np.max(np.abs(su.m))
    print("grid multiplier %s rel err %.2e" % (ns, err))
    assert err < 2e-12


@pytest.mark.parametrize("ns,dtype,tol", [((16, 24, 32), "f64", 1e-12), ((32, 12, 8), "f64", 1e-12),
                                          ((6, 48, 16), "f64", 1e-12), ((48, 32, 64), "f64", 1e-12),
                                          ((16, 24, 32), "f32", 1e-5),
                                          # extreme aspect ratios: the smallest and largest counts together
                                          ((4, 8, 384), "f64", 1e-12), ((384, 4, 6), "f64", 1e-12),
                                          ((8, 384, 4), "f32", 1e-5)])
def test_grid_random_density_parity(ns, dtype, tol):
    import torch
    rho = np.random.default_rng(sum(ns)).standard_normal(ns)
    want = O.solve(rho, HS, 40)
    p = B.Plan(ns, HS, 40, dtype=dtype).precompute()
    td = torch.float64 if dtype == "f64" else torch.float32
    u = p.solve(to_dev(rho, td)).double().cpu().numpy()
    torch.cuda.synchronize()
    e = rel_max_err(u, want)
    print("grid %s %s E_par=%.3e" % (ns, dtype, e))
    assert e <= tol


def test_grid_gaussian_closed_form():
    import torch
    Ns = (48, 64, 96)
    hs = tuple(4.0 / (N - 1) for N in Ns)
    xs = [-2.0 + h * np.arange(N) for h, N in zip(hs, Ns)]
    X, Y, Z = xs[0][:, None, None], xs[1][None, :, None], xs[2][None, None, :]
    rho, u_star = C.gaussian_pair(X, Y, Z, 0.2)
    p = B.Plan(Ns, hs, 461).precompute()
    u = p.solve(to_dev(rho)).cpu().numpy()
    torch.cuda.synchronize()
    E = C.relative_max_error(u, u_star)
    print("grid %s Gaussian E=%.3e" % (Ns, E))
    assert E < 1e-12


def test_grid_graph_and_refusals():
    import torch
    ns = (16, 24, 32)
    p = B.Plan(ns, HS, 40).precompute()
    rho = to_dev(np.random.default_rng(1).standard_normal(ns))
    u = p.solve(rho)
    ug = torch.empty_like(u)
    g = B.Graph.capture(p, rho, ug)
    g.launch()
    torch.cuda.synchronize()
    assert torch.equal(u, ug)
    g.close()
    for call in (lambda: p.solve_padded_debug(rho), lambda: p.autotune(reps=1)):
        with pytest.raises(B.PspError) as ei:
            call()
        assert B.STATUS[ei.value.status] == "PSP_EUNSUPPORTED"


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_grid_batches_match_single_solves(dtype):
    """Grids beside cubes in psp_solve_batched and psp_graph_capture_batched:
    bitwise the single solves (two grids share a shape, so their workspace is
    shared and reused), also on a second batch and on graph replays between
    eager work; the grids alone in a batch too."""
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    rng = np.random.default_rng(7)
    shapes = [(16, 24, 32), 24, (32, 12, 8), 16, (16, 24, 32), (6, 48, 16)]
    plans = [B.Plan(s, HS if isinstance(s, tuple) else 0.1, 40, dtype=dtype).precompute() for s in shapes]
    rhos = [to_dev(rng.standard_normal(p.shape3), td) for p in plans]
    want = [p.solve(r).clone() for p, r in zip(plans, rhos)]
    torch.cuda.synchronize()
    for rep in range(2):
        us = [torch.full_like(r, float("nan")) for r in rhos]
        B.solve_batched(plans, rhos, us)
        torch.cuda.synchronize()
        for i, (u, w) in enumerate(zip(us, want)):
            assert torch.equal(u, w), (rep, i, shapes[i])
    grids = [i for i, s in enumerate(shapes) if isinstance(s, tuple)]
    us = [torch.full_like(rhos[i], float("nan")) for i in grids]
    B.solve_batched([plans[i] for i in grids], [rhos[i] for i in grids], us)
    torch.cuda.synchronize()
    for u, i in zip(us, grids):
        assert torch.equal(u, want[i]), ("grids only", i)
    for members in (list(range(len(shapes))), grids):
        ug = [torch.empty_like(rhos[i]) for i in members]
        g = B.Graph.capture_batched([plans[i] for i in members], [rhos[i] for i in members], ug)
        for rep in range(3):
            for u in ug:
                u.fill_(float("nan"))
            plans[1].solve(rhos[1])               # eager work between replays
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for u, i in zip(ug, members):
                assert torch.equal(u, want[i]), ("graph", rep, i)
        g.close()
