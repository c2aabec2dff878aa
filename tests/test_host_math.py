"""Host FP64 mathematics of the library (no GPU needed) against the oracle:
the Fermi, gapped-filter and propagator coefficients and the QP solve."""
import os

import numpy as np
import pytest

from oracle import chebyshev as cheb
from oracle import qp as oqp

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2601_21005_amd", "libsgw.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


@pytest.mark.parametrize("eps", [1e-7, 1e-4])
def test_gapped_coefficients_match_oracle(eps):
    from paper_2601_21005_amd import sgw
    emin, emax, eh, el = -9.0, 75.0, -4.9, -4.4
    got = sgw.sgw_gapped_coefficients(eh, el, eps, emin, emax, 3000)
    ref = cheb.gapped_coefficients(eh, el, eps, emin, emax, 3000)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_fermi_coefficients_match_oracle():
    from paper_2601_21005_amd import sgw
    got = sgw.sgw_fermi_coefficients(-4.65, 40.0, -9.0, 75.0, 2000)
    ref = cheb.fermi_coefficients(-4.65, 40.0, -9.0, 75.0, 2000)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_gapped_coefficients_reject_bad_gap():
    from paper_2601_21005_amd import sgw
    with pytest.raises(sgw.SgwError):
        sgw.sgw_gapped_coefficients(-4.0, -4.5, 1e-7, -9.0, 75.0, 10)
    with pytest.raises(sgw.SgwError):
        sgw.sgw_gapped_coefficients(-4.5, -4.0, 0.7, -9.0, 75.0, 10)


def test_host_coefficients_match_oracle():
    from paper_2601_21005_amd import sgw
    for mu, beta, lo, hi, n in ((-0.3, 50.0, -5.0, 60.0, 4000), (0.1, 6.0, -5.7, 61.0, 300)):
        a = sgw.sgw_fermi_coefficients(mu, beta, lo, hi, n)
        assert np.max(np.abs(a - cheb.fermi_coefficients(mu, beta, lo, hi, n))) < 1e-13
    for tau in (0.05, 0.2, -0.2, 1.5):
        b = sgw.sgw_propagator_coefficients(-14.8, 28.4, tau)
        ob = cheb.propagator_coefficients(-14.8, 28.4, tau)
        assert b.size == ob.size and np.max(np.abs(b - ob)) < 1e-14


def test_host_qp_solve_matches_oracle():
    from paper_2601_21005_amd import sgw
    nt, dt = 80, 0.1
    t = dt * np.arange(-nt, nt + 1)
    sig = (np.where(t > 0, -0.08j * np.exp(0.4j * t), 0)
           + np.where(t < 0, 0.05j * np.exp(1.3j * t), 0))
    sig[nt] = 0.5 * (-0.08j + 0.05j)
    for eks, x in ((-0.6, -0.2), (0.1, -0.05)):
        got = sgw.sgw_qp_solve(sig, dt, 0.2, eks, x)
        ref = oqp.qp_solve(sig, dt, 0.2, eks, x)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
