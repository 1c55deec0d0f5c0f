"""The near-field cutoff on the GPU path (Lemma 1, Theorem 1, Table 3):
plans built with an explicit eps (psp_plan_create_ex) and the paper's
double-precision Gaussian sum (S = 460) match the oracle at every eps of
Table 3, reproduce its error to the order of magnitude, follow the
fourth-order law, and err exactly by the cutoff-defect term
-M0 Lap rho predicted from the Gaussian-sum weights."""
import math

import numpy as np
import pytest

from oracle import closed_forms as C
from oracle import psp_oracle as O
from paper_2506_04489_amd import psp as B
from tests.gpu_util import announce, rel_max_err, to_dev
from tests.test_oracle_eps import R_PAPER, SIGMA, TABLE, cutoff

pytestmark = pytest.mark.gpu

EPS = sorted({e for e, _ in TABLE}, reverse=True)


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def _gpu(N, eps_paper):
    import torch
    h, X, Y, Z = C.paper_grid(N)
    rho, u_star = C.gaussian_pair(X, Y, Z, SIGMA)
    eps = cutoff(eps_paper, N)
    _, delta = O.default_eps_delta(N, h)
    p = B.Plan(N, h, R_PAPER, eps=eps, delta=delta).precompute()
    u = p.solve(to_dev(rho)).cpu().numpy()
    torch.cuda.synchronize()
    return u, u_star, rho, h, (X, Y, Z), eps, delta, p


@pytest.mark.parametrize("eps_paper", EPS)
def test_parity_with_oracle_at_each_cutoff(eps_paper):
    u, _, rho, h, _, eps, delta, p = _gpu(32, eps_paper)
    w, a = p.gs()
    wo, ao = O.gs_weights(R_PAPER, eps, delta)
    assert np.allclose(w, wo, rtol=1e-14, atol=0) and np.allclose(a, ao, rtol=1e-14, atol=0)
    want = O.solve(rho, h, R_PAPER, eps=eps, delta=delta)
    e = rel_max_err(u, want)
    print("N=32 eps=%g parity %.2e" % (eps_paper, e))
    assert e <= 1e-12


@pytest.mark.parametrize("N", [64, 128])
def test_cutoff_law_on_the_gpu(N):
    Es, lines = [], []
    for eps_paper in EPS:
        u, u_star, _, _, (X, Y, Z), eps, _, p = _gpu(N, eps_paper)
        E = rel_max_err(u, u_star)
        w, a = p.gs()
        pred = -C.gs_cutoff_moment(w, a, 8 * eps) * C.gaussian_laplacian(X, Y, Z, SIGMA)
        dev = float(np.max(np.abs((u - u_star) - pred)) / np.max(np.abs(pred)))
        E_pred = float(np.max(np.abs(pred)) / np.max(np.abs(u_star)))
        E_paper = TABLE[(eps_paper, N)]
        lines.append("N=%d eps=%.1e E=%.3e paper %.3e predicted %.3e (field deviation %.1e)"
                     % (N, eps_paper, E, E_paper, E_pred, dev))
        Es.append(E)
        # the paper's construction differs in its sinc step: order of magnitude
        assert E_paper / 10 < E < 10 * E_paper, lines[-1]
        # the defect term is the error once the eps-ball is small against the
        # Gaussian's width (its next term is O((eps/sigma)^2) smaller) and
        # the error is well above rounding
        if E_pred > 1e-11 and eps < SIGMA / 2:
            assert dev <= (2e-3 if eps < SIGMA / 4 else 2e-2), lines[-1]
    print("\n".join(lines))
    # fourth order over the rows the cutoff limits
    k = [i for i, e in enumerate(EPS) if 4e-4 < e < 3e-2]
    slope = np.polyfit(np.log([EPS[i] for i in k]), np.log([Es[i] for i in k]), 1)[0]
    print("N=%d slope of log E against log eps: %.3f" % (N, slope))
    assert abs(slope - 4.0) < 0.15
