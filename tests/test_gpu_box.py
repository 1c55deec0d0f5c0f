"""Rectangular boxes on the GPU (psp_plan_create_box; Section 3, Tables 4,
6, 8): the multiplier and the solve against the oracle, the paper's rows,
and rectangular plans inside batches."""
import numpy as np
import pytest

from oracle import closed_forms as C
from oracle import psp_oracle as O
from paper_2506_04489_amd import psp as B
from tests.gpu_util import announce, rel_max_err, to_dev
from tests.test_oracle_box import ROWS, R_PAPER

pytestmark = pytest.mark.gpu

HS = (0.11, 0.17, 0.29)


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


@pytest.mark.parametrize("n,hs,R", [(16, HS, 40), (24, (5 / 23, 5.5 / 23, 6 / 23), 461), (12, (0.3, 0.3, 0.05), 40)])
def test_box_multiplier(n, hs, R):
    p = B.Plan(n, hs, R).precompute()
    m = p.multiplier()
    su = O.setup(n, hs, R)
    om, _ = p.gs()
    assert np.max(np.abs(om / su.omega - 1)) < 1e-14
    err = np.max(np.abs(m - su.m)) / np.max(np.abs(su.m))
    print("box multiplier n=%d h=%s R=%d rel err %.2e" % (n, hs, R, err))
    assert err < 2e-12


@pytest.mark.parametrize("n,dtype,tol", [(16, "f64", 1e-12), (32, "f64", 1e-12), (48, "f64", 1e-12), (32, "f32", 1e-5)])
def test_box_random_density_parity(n, dtype, tol):
    import torch
    rho = np.random.default_rng(300 + n).standard_normal((n, n, n))
    want = O.solve(rho, HS, 40)
    p = B.Plan(n, HS, 40, dtype=dtype).precompute()
    td = torch.float64 if dtype == "f64" else torch.float32
    u = p.solve(to_dev(rho, td)).double().cpu().numpy()
    torch.cuda.synchronize()
    e = rel_max_err(u, want)
    print("box n=%d %s E_par=%.3e" % (n, dtype, e))
    assert e <= tol


def _gpu_row(fam, par, box, N):
    import torch
    h, X, Y, Z = C.box_grid(N, box)
    rho, u_star = C.box_pair(fam, par, box, X, Y, Z)
    p = B.Plan(N, h, R_PAPER).precompute()
    u = p.solve(to_dev(rho)).cpu().numpy()
    torch.cuda.synchronize()
    return u, u_star, rho, h


@pytest.mark.parametrize("tab,fam,par,box,N,E_paper", ROWS,
                         ids=["%s-%s-%s-%d" % (r[0].replace(" ", ""), r[1], r[2], r[4]) for r in ROWS])
def test_paper_box_rows_on_gpu(tab, fam, par, box, N, E_paper):
    u, u_star, _, _ = _gpu_row(fam, par, box, N)
    E = C.relative_max_error(u, u_star)
    print("%s %s %s N=%d E=%.4e paper %.4e" % (tab, fam, par, N, E, E_paper))
    if N <= 32:
        # grid-limited: the printed digits
        assert abs(E - E_paper) <= 6e-4 * E_paper
    else:
        # at the Gaussian-sum and rounding floor: the order of magnitude
        assert E < 10 * E_paper + 1e-13


def test_box_row_parity_at_64():
    tab, fam, par, box, N, _ = [r for r in ROWS if r[0] == "Table 8" and r[2] == "32" and r[4] == 64][0]
    u, _, rho, h = _gpu_row(fam, par, box, N)
    want = O.solve(rho, h, R_PAPER)
    e = rel_max_err(u, want)
    print("%s L=32 N=64 parity %.2e" % (tab, e))
    assert e <= 1e-12


def test_box_plans_in_batches_bitwise():
    import torch
    pa = B.Plan(32, HS, 40).precompute()
    pb = B.Plan(32, 2 / 32, 40).precompute()
    pc = B.Plan(16, (0.3, 0.2, 0.1), 40).precompute()
    ps = [pa, pb, pc, pa]
    rhos = [to_dev(np.random.default_rng(40 + i).standard_normal((p.n,) * 3)) for i, p in enumerate(ps)]
    us = [torch.empty_like(r) for r in rhos]
    for mode in ("grouped", "persistent", "flat"):
        B.set_batch_mode(mode)
        try:
            B.solve_batched(ps, rhos, us)
            torch.cuda.synchronize()
        finally:
            B.set_batch_mode("grouped")
        for p, r, u in zip(ps, rhos, us):
            alone = p.solve(r)
            torch.cuda.synchronize()
            assert torch.equal(u, alone), (mode, p.h)
