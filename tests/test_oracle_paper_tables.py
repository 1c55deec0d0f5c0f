"""Pin the oracle to the error tables the paper prints (Section 3).

At 16^3 and 32^3 the errors are set by the grid (the paper's Table 2 shows a
different method printing the same digits), so they pin the grid convention,
padding, normalisation, sign and multiplier independently of the
Gaussian-sum details: the oracle must reproduce them to the printed 4 digits.
At 64^3, rows limited by the grid must again match; rows at the
double-precision floor must agree to within a small factor.
"""
import csv
import os

import pytest
import sympy as sp

from oracle import closed_forms as C
from oracle import psp_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
R_PAPER = 461          # the paper's S = 460 plus one


def _rows():
    with open(os.path.join(HERE, "golden", "paper_tables.csv")) as f:
        for row in csv.reader(l for l in f if not l.startswith("#")):
            fam, par, N, E, src = row
            yield fam, par, int(N), float(E), src


def _pair(fam, par, X, Y, Z):
    if fam == "gauss":
        return C.gaussian_pair(X, Y, Z, float(par))
    if fam == "two_gauss":
        return C.two_gaussians_pair(X, Y, Z)
    if fam == "anis":
        return C.anisotropic_pair(X, Y, Z)
    if fam == "osc":
        return C.oscillating_pair(X, Y, Z)
    raise KeyError(fam)


# rows whose 64^3 error sits at the double-precision floor (set by the GS fit
# and rounding, not the grid): order-of-magnitude agreement only
_FLOOR = {("gauss", "0.20", 64), ("gauss", "0.15", 64), ("anis", "0.30/0.20/0.28", 64)}

ROWS = list(_rows())


@pytest.mark.parametrize("fam,par,N,E_paper,src", ROWS,
                         ids=["%s-%s-%d" % (r[0], r[1], r[2]) for r in ROWS])
def test_paper_error(fam, par, N, E_paper, src):
    h, X, Y, Z = C.paper_grid(N)
    rho, u_star = _pair(fam, par, X, Y, Z)
    u = O.solve(rho, h, R_PAPER)
    E = C.relative_max_error(u, u_star)
    if (fam, par, N) in _FLOOR:
        assert E_paper / 3 < E < E_paper * 3, (src, E, E_paper)
    else:
        assert abs(E - E_paper) <= 6e-4 * E_paper, (src, E, E_paper)


def test_printed_oscillating_density_is_inconsistent():
    # eq. osci as printed does not reproduce the paper's own Table 9 value,
    # the corrected -Lap u* does (test above): the printed sign is a typo
    h, X, Y, Z = C.paper_grid(32)
    _, u_star = C.oscillating_pair(X, Y, Z)
    u = O.solve(C.oscillating_rho_as_printed(X, Y, Z), h, R_PAPER)
    assert C.relative_max_error(u, u_star) > 100 * 7.921e-3


def test_densities_are_minus_laplacian_of_potentials():
    x, y, z, d, R, s, w = sp.symbols("x y z d R sigma omega", positive=True)
    r2 = x ** 2 + y ** 2 + z ** 2

    def lap(f):
        return sum(sp.diff(f, v, 2) for v in (x, y, z))

    ub = sp.exp(-d * R ** 2 / (R ** 2 - r2))
    fb = (2 * d * R ** 2 * (3 * R ** 4 - 2 * R ** 2 * r2 - r2 ** 2 - 2 * d * R ** 2 * r2)
          / (R ** 2 - r2) ** 4 * sp.exp(-d * R ** 2 / (R ** 2 - r2)))
    assert sp.simplify(-lap(ub) - fb) == 0
    uo = sp.exp(-r2 / s ** 2) * sp.cos(w * r2)
    fo = (sp.exp(-r2 / s ** 2) * (6 * w * sp.sin(w * r2) + 4 * w ** 2 * r2 * sp.cos(w * r2))
          - (4 * r2 / s ** 4 - 6 / s ** 2) * sp.exp(-r2 / s ** 2) * sp.cos(w * r2)
          - 8 * w * r2 / s ** 2 * sp.exp(-r2 / s ** 2) * sp.sin(w * r2))
    assert sp.simplify(-lap(uo) - fo) == 0
    # the numeric helpers evaluate those same formulas
    import numpy as np
    X = np.array([[[0.3]]]); Y = np.array([[[-0.2]]]); Z = np.array([[[0.1]]])
    rho, _ = C.oscillating_pair(X, Y, Z)
    val = float(fo.subs({x: 0.3, y: -0.2, z: 0.1, s: 0.3, w: 20.0}))
    assert abs(rho[0, 0, 0] - val) < 1e-12 * abs(val)
    rho, _ = C.bump_pair(X, Y, Z)
    val = float(fb.subs({x: 0.3, y: -0.2, z: 0.1, d: 10.0, R: 2.0}))
    assert abs(rho[0, 0, 0] - val) < 1e-12 * abs(val)
