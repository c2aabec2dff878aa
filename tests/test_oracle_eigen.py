"""Pins for the oracle's iterative eigensolvers (the stand-in for the
preliminary DFT run that supplies phi and the band edges, Sec. 2.1) against
dense diagonalisation of the same H."""
import numpy as np
import pytest

from oracle import eigen


@pytest.mark.parametrize("which,k,offset", [("tiny8", 6, 0.0), ("tiny12", 8, 0.0),
                                              ("tiny8", 6, 6.0), ("tiny12", 8, 6.0)])
def test_lowest_states_match_dense_eigh(which, k, offset, request):
    """The k lowest eigenpairs from Lanczos on the shifted operator equal the
    dense ones: energies to 1e-9 Ha, orbitals up to sign (|<a|b>| = 1 to
    1e-6 for non-degenerate levels), all normalised to <phi|phi> = 1.  A
    constant offset of the potential makes the whole spectrum positive, where
    only a shift at the top of the spectrum makes the lowest states the
    largest in magnitude."""
    from conftest import build_oracle_h
    s, H = request.getfixturevalue(which)
    e_d, V_d = request.getfixturevalue(which + "_eig")
    if offset:
        from dataclasses import replace
        H = build_oracle_h(replace(s, v_loc=s.v_loc + offset))
        e_d = e_d + offset
        assert e_d[0] > 0
    e, V = eigen.lowest_states(H, k)
    assert np.max(np.abs(e - e_d[:k])) < 1e-9
    dV = H.grid.dV
    assert np.allclose(dV * np.sum(V * V, axis=1), 1.0, atol=1e-10)
    ov = dV * V @ V_d[:k].T
    for a in range(k):
        gap = min(abs(e_d[a] - e_d[b]) for b in range(k + 1) if b != a)
        if gap > 1e-6:
            assert abs(abs(ov[a, a]) - 1.0) < 1e-6, a
    # the orbitals are eigenvectors of this H
    r = H.apply(V) - e[:, None] * V
    assert np.max(np.linalg.norm(r, axis=1) * np.sqrt(dV)) < 1e-6


@pytest.mark.parametrize("which", ["tiny8", "tiny12"])
def test_highest_eigenvalue_matches_dense_eigh(which, request):
    s, H = request.getfixturevalue(which)
    e_d, _ = request.getfixturevalue(which + "_eig")
    assert abs(eigen.highest_eigenvalue(H) - e_d[-1]) < 1e-8 * max(1.0, abs(e_d[-1]))
