"""GPU: the FP64 exponential of the pair kernels (e^{-kappa rho} in K1..K4,
Section 2.1 eq. (Eq_Ls); gfx950 has no FP64 exponential instruction, so the
kernels evaluate their own: a two-constant ln 2 reduction and a degree-10
minimax polynomial).  Checked through the C ABI against the host's 64-bit
mantissa exponential (numpy longdouble) to a bound of 4 ulp over the range
of kappa rho the workloads reach, plus the special values."""
import numpy as np
import pytest

from paper_1301_5885_amd import gabi

pytestmark = pytest.mark.gpu


def ulp_error(got, t):
    ref = np.exp(-t.astype(np.longdouble))
    r64 = ref.astype(np.float64)
    ulp = np.spacing(np.abs(r64))
    return np.abs(got.astype(np.longdouble) - ref) / ulp.astype(np.longdouble)


def test_exp_neg_within_4_ulp():
    rng = np.random.default_rng(0)
    t = np.concatenate([rng.uniform(0.0, 60.0, 400000), rng.uniform(0.0, 1e-3, 50000),
                        np.linspace(0.0, 2.0, 20001)])
    got = gabi.selftest_exp_neg(t)
    err = ulp_error(got, t)
    print(f"max {float(err.max()):.3f} ulp, mean {float(err.mean()):.3f} ulp")
    assert float(err.max()) <= 4.0


def test_exp_neg_special_values():
    t = np.array([0.0, 5e-324, 1e-300, 700.0, 744.0, 745.0, 746.0, 1e6, 1e300])
    got = gabi.selftest_exp_neg(t)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0
    assert 0.0 < got[3] < 1e-300 and 0.0 <= got[4] < 1e-320
    assert np.all(got[6:] == 0.0)
    with pytest.raises(gabi.GabiError):
        gabi.selftest_exp_neg(np.array([-1.0]))
