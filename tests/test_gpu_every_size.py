"""Both tiers at every supported size n (every even n from 4 to 384 with
2n = 2^a 3^b), each against the oracle's whole-grid solve of the same
seeded white-noise density, in the launch shape the tuning table gives that
size: FP64 <= 1e-12, FP32 <= 1e-5 (eq. error_infty over every grid point).
The measured errors are printed as a table."""
import numpy as np
import pytest

from oracle import psp_oracle as O
from paper_2506_04489_amd import psp as B
from tests.gpu_util import announce, rel_max_err, to_dev

pytestmark = pytest.mark.gpu


def _sizes():
    out = []
    for n in range(4, 385, 2):
        m = 2 * n
        while m % 2 == 0:
            m //= 2
        while m % 3 == 0:
            m //= 3
        if m == 1:
            out.append(n)
    return out


SIZES = _sizes()


def test_sizes_are_the_2a3b_family():
    assert SIZES[:6] == [4, 6, 8, 12, 16, 18] and SIZES[-1] == 384 and len(SIZES) == 24


@pytest.mark.parametrize("n", SIZES)
def test_both_tiers_against_the_oracle(n):
    import torch
    announce("every-size parity n=%d" % n)
    h = 2.0 / n
    rho = np.random.default_rng(7000 + n).standard_normal((n, n, n))
    want = O.solve(rho, h, 40)
    errs = {}
    for dtype, td, tol in (("f64", torch.float64, 1e-12), ("f32", torch.float32, 1e-5)):
        p = B.Plan(n, h, 40, dtype=dtype).precompute()
        u = p.solve(to_dev(rho, td))
        torch.cuda.synchronize()
        errs[dtype] = rel_max_err(u.double().cpu().numpy(), want)
        p.close()
        assert errs[dtype] <= tol, (n, dtype, errs[dtype])
    print("n=%3d (2n=%3d)  E_par FP64 %.2e  FP32 %.2e" % (n, 2 * n, errs["f64"], errs["f32"]))
