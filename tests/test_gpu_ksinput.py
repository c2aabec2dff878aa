"""GPU check of the KS-input stand-in (Chebyshev-filtered subspace
iteration over sgw_apply_H) against the oracle's Lanczos eigenpairs."""
import numpy as np
import pytest

from conftest import make_ctx
from oracle import eigen
from paper_2601_21005_amd import ksinput, sgw

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,tol", [(sgw.SGW_C128, 1e-8), (sgw.SGW_C64, 2e-5)])
def test_lowest_states_gaussian_wells(cfg1, prec, tol):
    s, H = cfg1
    ctx = make_ctx(s, prec)
    lo, hi = ctx.bounds()
    e, phi, res = ksinput.lowest_states(ctx, 9, lo, hi, H.grid.dV)
    eo, Vo = eigen.lowest_states(H, 9)
    assert np.max(np.abs(e - eo)) < tol
    # the HOMO orbital agrees up to sign
    p = phi[7].cpu().numpy()
    ov = abs(H.grid.dV * np.dot(p, Vo[7]))
    assert ov > 1 - 1e3 * tol
    ctx.close()
