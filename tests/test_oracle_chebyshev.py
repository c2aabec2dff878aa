"""Pins for the Chebyshev filter (Eq. 3) and the Chebyshev propagator."""
import numpy as np
import scipy.linalg as sla

from oracle import chebyshev as cheb
from oracle.grid import Grid
from oracle.hamiltonian import Hamiltonian


def test_scalar_fermi_reconstruction():
    emin, emax, mu, beta = -5.0, 60.0, -0.3, 50.0
    tol = 1e-10
    N = cheb.suggested_ncoef(mu, beta, emin, emax, tol=tol, nmax=16384)
    a = cheb.fermi_coefficients(mu, beta, emin, emax, N)
    c, R = cheb.cheb_map(emin, emax)
    x = np.linspace(-1, 1, 100001)
    err = np.max(np.abs(cheb.cheb_series_scalar(a, x) - cheb.fermi(c + R * x, mu, beta)))
    assert err < 2 * tol
    # the truncation error is bounded by the discarded tail
    a_long = cheb.fermi_coefficients(mu, beta, emin, emax, 4 * N)
    assert np.sum(np.abs(a_long[N:])) < tol
    # the Fermi step is smooth: coefficients decay monotonically far out
    assert abs(a[-1]) < 1e-11


def test_filter_matches_eigendecomposition(tiny12, tiny12_eig):
    s, H = tiny12
    e, V = tiny12_eig
    emin, emax = H.bounds()
    mu, beta = 0.5 * (e[1] + e[2]), 6.0
    N = cheb.suggested_ncoef(mu, beta, emin, emax, tol=1e-12, nmax=8192)
    a = cheb.fermi_coefficients(mu, beta, emin, emax, N)
    x = np.random.default_rng(3).standard_normal((2, H.grid.N))
    out = cheb.apply_series(H, a, emin, emax, x)
    dV = H.grid.dV
    f = cheb.fermi(e, mu, beta)
    exact = ((x @ V.T) * dV * f[None, :]) @ V        # sum_k f_k phi_k <phi_k|x>
    bound = np.sum(np.abs(cheb.fermi_coefficients(mu, beta, emin, emax, 4 * N)[N:]))
    assert np.max(np.abs(out - exact)) <= (bound + 1e-11) * np.max(np.abs(x)) * 10


def test_jacobi_anger_scalar():
    emin, emax = -4.0, 40.0
    c, R = cheb.cheb_map(emin, emax)
    x = np.linspace(-1, 1, 2001)
    for tau in (0.05, 0.2, -0.2, 1.3):
        b = cheb.propagator_coefficients(emin, emax, tau)
        series = cheb.cheb_series_scalar(b.real, x) + 1j * cheb.cheb_series_scalar(b.imag, x)
        assert np.max(np.abs(series - np.exp(-1j * (c + R * x) * tau))) < 1e-13


def test_propagator_matches_expm_and_is_unitary(tiny8, tiny8_eig):
    s, H = tiny8
    e, V = tiny8_eig
    emin, emax = H.bounds()
    g = H.grid
    psi = np.random.default_rng(2).standard_normal(g.N) + 0j
    psi /= np.sqrt(g.norm2(psi))
    tau = 0.2
    out = cheb.propagate(H, emin, emax, tau, psi)
    exact = V.T @ (np.exp(-1j * e * tau) * (g.dV * V @ psi))
    assert np.max(np.abs(out - exact)) < 1e-12
    # unitarity and time reversal over 100 steps
    p = psi.copy()
    for _ in range(100):
        p = cheb.propagate(H, emin, emax, tau, p)
    assert abs(g.norm2(p) - 1.0) < 1e-11
    for _ in range(100):
        p = cheb.propagate(H, emin, emax, -tau, p)
    assert np.max(np.abs(p - psi)) * np.sqrt(g.dV) < 1e-11


def test_free_particle_packet():
    """V = 0: a Gaussian packet drifts by k0 t and spreads as
    sigma(t)^2 = sigma0^2 + (t / (2 sigma0))^2 (per axis)."""
    g = Grid(32, h=0.5)
    H = Hamiltonian(g, np.zeros(g.N))
    emin, emax = H.bounds()
    r = g.coords()
    L = np.array(g.L)
    r0 = L / 2
    k0 = 2 * np.pi * np.array([2, -1, 0]) / L
    s0 = 1.2
    d = g.min_image(r - r0)
    psi = np.exp(-np.sum(d * d, axis=1) / (4 * s0 * s0) + 1j * (r @ k0))
    psi /= np.sqrt(g.norm2(psi))
    t, tau = 0.0, 0.25
    for _ in range(8):
        psi = cheb.propagate(H, emin, emax, tau, psi)
        t += tau
        rho = g.dV * np.abs(psi) ** 2
        centre = r0 + k0 * t
        dd = g.min_image(r - centre)
        mean = rho @ dd
        var = rho @ (dd * dd)
        assert np.max(np.abs(mean)) < 1e-5
        assert np.allclose(var, s0 ** 2 + (t / (2 * s0)) ** 2, rtol=1e-6)


def test_gapped_step_edges_and_symmetry():
    """G(E_HOMO) = 1 - eps, G(E_LUMO) = eps, G(mu + x) = 1 - G(mu - x), and
    G stays within eps of the step outside the gap."""
    eh, el, eps = -0.7, -0.2, 1e-7
    assert abs(cheb.gapped_step(eh, eh, el, eps) - (1 - eps)) < 1e-15
    assert abs(cheb.gapped_step(el, eh, el, eps) - eps) < 1e-20
    x = np.linspace(0, 3, 301)
    mu = 0.5 * (eh + el)
    assert np.allclose(cheb.gapped_step(mu + x, eh, el, eps),
                       1 - cheb.gapped_step(mu - x, eh, el, eps), rtol=0, atol=1e-15)
    E = np.concatenate([np.linspace(-10, eh, 500), np.linspace(el, 10, 500)])
    step = (E < mu).astype(float)
    assert np.max(np.abs(cheb.gapped_step(E, eh, el, eps) - step)) <= eps * (1 + 1e-12)


def test_gapped_reconstruction_and_shorter_than_fermi():
    """The series reproduces G to its discarded tail, and for the same edge
    accuracy (1e-7 at the gap edges) it is shorter than the Fermi series."""
    emin, emax, eh, el, eps = -5.0, 60.0, -0.7, -0.2, 1e-7
    a = cheb.gapped_coefficients(eh, el, eps, emin, emax, 8192)
    N = cheb.tail_length(a, 1e-9)
    c, R = cheb.cheb_map(emin, emax)
    x = np.linspace(-1, 1, 50001)
    err = np.max(np.abs(cheb.cheb_series_scalar(a[:N], x) - cheb.gapped_step(c + R * x, eh, el, eps)))
    assert err < 2e-9
    beta = 2 * np.log((1 - eps) / eps) / (el - eh)       # Fermi with the same edge values
    assert abs(cheb.fermi(el, 0.5 * (eh + el), beta) - eps) < 1e-12
    nf = cheb.suggested_ncoef(0.5 * (eh + el), beta, emin, emax, tol=1e-9, nmax=16384)
    assert N < 0.6 * nf, (N, nf)


def test_gapped_filter_matches_eigendecomposition(tiny12, tiny12_eig):
    s, H = tiny12
    e, V = tiny12_eig
    emin, emax = H.bounds()
    eh, el = e[1], e[2]
    a = cheb.gapped_coefficients(eh, el, 1e-6, emin, emax, 4096)
    N = cheb.tail_length(a, 1e-12)
    x = np.random.default_rng(4).standard_normal((2, H.grid.N))
    out = cheb.apply_series(H, a[:N], emin, emax, x)
    f = cheb.gapped_step(e, eh, el, 1e-6)
    exact = ((x @ V.T) * H.grid.dV * f[None, :]) @ V
    assert np.max(np.abs(out - exact)) <= 1e-11 * np.max(np.abs(x)) * 10
