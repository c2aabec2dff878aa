"""The host FP64 control-variate estimator of the library (no GPU needed)
against the oracle's, including the fallback to the plain mean."""
import os

import numpy as np
import pytest

from oracle import cv

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2601_21005_amd", "libsgw.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


@pytest.mark.parametrize("bias", [0.0, 0.4])
def test_cv_estimate_matches_oracle(bias):
    from paper_2601_21005_amd import sgw
    rs = np.random.default_rng(50)
    u = rs.standard_normal(333)
    y = 0.7 + 1.5 * u + 0.5 * rs.standard_normal(333)
    g = np.tanh(u) + 0.05 * rs.standard_normal(333)
    args = (y[:150], g[:150], y[150:], g[150:], bias + np.tanh(0.0), 0.6, 50000)
    got = sgw.sgw_cv_estimate(*args)
    ref = cv.cv_estimate(*args)
    assert got["fallback"] == ref["fallback"] == (bias > 0)
    for k in ("estimate", "sigma", "c", "rho2", "plain", "sigma_plain", "sigma_cv"):
        assert abs(got[k] - ref[k]) <= 1e-12 * max(1.0, abs(ref[k])), k


def test_cv_estimate_rejects_bad_input():
    from paper_2601_21005_amd import sgw
    y = np.ones(5)
    with pytest.raises(sgw.SgwError):
        sgw.sgw_cv_estimate(y[:1], y[:1], y, y, 0.0, 1.0, 10)
    with pytest.raises(sgw.SgwError):
        sgw.sgw_cv_estimate(y, y, y, y, 0.0, -1.0, 10)
