"""Pin for the FFT-Poisson Hartree potential (periodic, G = 0 dropped)."""
import numpy as np
from scipy.special import erf

from oracle.grid import Grid
from oracle.tdh import hartree


def gauss3(d2, s):
    return np.exp(-d2 / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5


def test_neutral_gaussian_pair_potential():
    """rho = q (g_s1 - g_s2): V = q [erf(r/sqrt2 s1) - erf(r/sqrt2 s2)] / r
    + 2 pi q (s1^2 - s2^2) / Omega exactly for the zero-mean periodic
    solution (the image sum of a compact neutral spherical charge differs
    from the free-space potential by -V~_free(k=0)/Omega)."""
    g = Grid(48, h=0.5)
    r = g.coords()
    c = np.array(g.L) / 2 + np.array([0.1, 0.2, -0.15])
    d = g.min_image(r - c)
    d2 = np.sum(d * d, axis=1)
    q, s1, s2 = 1.7, 1.5, 1.1
    rho = q * (gauss3(d2, s1) - gauss3(d2, s2))
    v = hartree(g, rho)
    rr = np.sqrt(d2)
    omega = np.prod(g.L)
    with np.errstate(invalid="ignore", divide="ignore"):
        ve = q * (erf(rr / (np.sqrt(2) * s1)) - erf(rr / (np.sqrt(2) * s2))) / rr
    r0 = rr < 1e-12
    ve[r0] = q * np.sqrt(2 / np.pi) * (1 / s1 - 1 / s2)
    ve += 2 * np.pi * q * (s1 ** 2 - s2 ** 2) / omega
    assert np.max(np.abs(v - ve)) < 1e-7
    assert abs(np.mean(v)) < 1e-12


def test_uniform_charge_drops_out():
    """With G = 0 dropped (a neutralising background), a uniform charge adds
    nothing to v_H and a charged density's potential has zero mean: the
    potentials of a single Gaussian and of that Gaussian plus a constant are
    the same."""
    g = Grid(24, h=0.5)
    d = g.min_image(g.coords() - np.array(g.L) / 2)
    rho = gauss3(np.sum(d * d, axis=1), 1.2)
    v1 = hartree(g, rho)
    v2 = hartree(g, rho + 0.37)
    assert abs(np.mean(v1)) < 1e-12
    assert np.max(np.abs(v1 - v2)) < 1e-12 * np.max(np.abs(v1))
