"""Chebyshev expansions of functions of H (oracle side).

* Occupied-space filter, Eq. (3): Theta(mu - H) ~ sum_{n=0}^{N} a_n T_n(H~),
  with H~ = (H - c)/R mapping the spectral interval [E_min, E_max] onto
  [-1, 1] (Sec. 2.1).  Applied to the white-noise orbitals to obtain random
  combinations of occupied states (Sec. 2.1, Sec. 2.3).
* Propagator e^{-i H tau} used to evolve the zeta orbitals (Sec. 2.1, second
  phase).

Readings:
* Filter function: a Fermi function F(E) = 1 / (1 + exp(beta (E - mu))) with
  mu mid-gap stands in for the Heaviside step (the sharp limit beta -> inf).
* Gapped filter (Sec. 2.1: the cutoff is spread over the band gap
  E_HOMO <= mu <= E_LUMO instead of sitting at one mu; the coefficient
  construction itself is in a reference the paper cites and does not
  restate).  Reading: the Gaussian-smoothed step
      G(E) = erfc((E - mu) / sigma) / 2,  mu = (E_HOMO + E_LUMO) / 2,
      sigma = (E_LUMO - E_HOMO) / (2 erfcinv(2 eps)),
  which is 1 - eps at E_HOMO and eps at E_LUMO and within eps of the step
  everywhere outside the gap; being entire, its Chebyshev coefficients decay
  faster than those of a Fermi function with the same edge values.
* Coefficients by Chebyshev-Gauss quadrature with M = 4 * ncoef nodes:
      a_n = (2 - delta_n0) / M  sum_j F(c + R cos theta_j) cos(n theta_j),
      theta_j = pi (j + 1/2) / M.
  No damping kernel (none is mentioned in the paper).
* Propagator: e^{-i H tau} = e^{-i c tau} sum_n (2 - delta_n0) (-i)^n
  J_n(R tau) T_n(H~)  (the Jacobi-Anger expansion), truncated at the first
  order n > R|tau| with |J_n(R|tau|)| < tol.
"""
import numpy as np
from scipy.fft import dct
from scipy.special import erfc, erfcinv, expit, jv


def fermi(E, mu, beta):
    return expit(-beta * (np.asarray(E, dtype=np.float64) - mu))


def cheb_map(emin, emax):
    c = 0.5 * (emax + emin)
    R = 0.5 * (emax - emin)
    return c, R


def fermi_coefficients(mu, beta, emin, emax, ncoef):
    """a_0 .. a_{ncoef-1} of the Fermi filter on [emin, emax]."""
    c, R = cheb_map(emin, emax)
    M = 4 * int(ncoef)
    j = np.arange(M)
    theta = np.pi * (j + 0.5) / M
    f = fermi(c + R * np.cos(theta), mu, beta)
    # DCT-II: y_n = 2 sum_j f_j cos(n theta_j)  (a library primitive)
    y = dct(f, type=2)
    a = y[:ncoef] / M
    a[0] *= 0.5
    return a


def gapped_step(E, e_homo, e_lumo, eps):
    """G(E): 1 - eps at e_homo, eps at e_lumo, erfc-shaped in between."""
    mu = 0.5 * (e_homo + e_lumo)
    sigma = (e_lumo - e_homo) / (2.0 * erfcinv(2.0 * eps))
    return 0.5 * erfc((np.asarray(E, dtype=np.float64) - mu) / sigma)


def gapped_coefficients(e_homo, e_lumo, eps, emin, emax, ncoef):
    """a_0 .. a_{ncoef-1} of the gapped filter, same quadrature as the Fermi
    filter."""
    c, R = cheb_map(emin, emax)
    M = 4 * int(ncoef)
    theta = np.pi * (np.arange(M) + 0.5) / M
    y = dct(gapped_step(c + R * np.cos(theta), e_homo, e_lumo, eps), type=2)
    a = y[:ncoef] / M
    a[0] *= 0.5
    return a


def tail_length(a, tol):
    """Smallest N with sum_{n >= N} |a_n| < tol."""
    tail = np.cumsum(np.abs(a[::-1]))[::-1]
    ok = np.nonzero(tail < tol)[0]
    if ok.size == 0:
        raise ValueError("coefficients too short for the requested tolerance")
    return int(ok[0])


def suggested_ncoef(mu, beta, emin, emax, tol=1e-10, nmax=65536):
    """Smallest N whose discarded tail sum_{n>=N} |a_n| is below ``tol``
    (tail measured on coefficients computed to ``nmax``)."""
    a = fermi_coefficients(mu, beta, emin, emax, nmax)
    tail = np.cumsum(np.abs(a[::-1]))[::-1]  # tail[n] = sum_{k>=n} |a_k|
    ok = np.nonzero(tail < tol)[0]
    if ok.size == 0:
        raise ValueError("nmax too small for the requested tolerance")
    return int(ok[0])


def cheb_series_scalar(coef, x):
    """sum_n coef_n T_n(x) for scalar/array x (three-term recurrence)."""
    x = np.asarray(x, dtype=np.float64)
    t0 = np.ones_like(x)
    out = coef[0] * t0
    if len(coef) == 1:
        return out
    t1 = x.copy()
    out = out + coef[1] * t1
    for n in range(2, len(coef)):
        t0, t1 = t1, 2.0 * x * t1 - t0
        out = out + coef[n] * t1
    return out


def apply_series(H, coef, emin, emax, x):
    """sum_n coef_n T_n(H~) x via v_{n+1} = 2 H~ v_n - v_{n-1}  (Eq. 3)."""
    c, R = cheb_map(emin, emax)

    def Ht(v):
        return (H.apply(v) - c * v) / R

    v0 = np.array(x, copy=True)
    out = coef[0] * v0
    if len(coef) == 1:
        return out
    v1 = Ht(v0)
    out = out + coef[1] * v1
    for n in range(2, len(coef)):
        v0, v1 = v1, 2.0 * Ht(v1) - v0
        out = out + coef[n] * v1
    return out


def fermi_filter(H, mu, beta, emin, emax, ncoef, x):
    """F(H) x with the Chebyshev-Gauss Fermi coefficients."""
    a = fermi_coefficients(mu, beta, emin, emax, ncoef)
    return apply_series(H, a, emin, emax, x)


def propagator_nterms(R, tau, tol=1e-14):
    """Number of Jacobi-Anger terms kept: the first n > R|tau| (n >= 1) with
    |J_n(R |tau|)| < tol, terms 0..n-1 being kept."""
    x = abs(R * tau)
    n = max(1, int(np.floor(x)) + 1)
    while abs(jv(n, x)) >= tol:
        n += 1
    return n


def propagator_coefficients(emin, emax, tau, tol=1e-14):
    """Complex b_n with e^{-i H tau} = sum_n b_n T_n(H~)."""
    c, R = cheb_map(emin, emax)
    nt = propagator_nterms(R, tau, tol)
    n = np.arange(nt)
    b = (2.0 - (n == 0)) * (-1j) ** n * jv(n, R * tau) * np.exp(-1j * c * tau)
    return b


def propagate(H, emin, emax, tau, psi, tol=1e-14):
    """e^{-i H tau} psi by the Chebyshev expansion (one step)."""
    b = propagator_coefficients(emin, emax, tau, tol)
    return apply_series(H, b, emin, emax, np.asarray(psi, dtype=np.complex128))
