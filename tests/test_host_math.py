"""Host FP64 mathematics of the library (no GPU needed) against the oracle:
the Fermi and gapped filter coefficients."""
import os

import numpy as np
import pytest

from oracle import chebyshev as cheb

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
