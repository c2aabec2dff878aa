"""Frequency-resolved self-energy and the quasi-particle equation.

* Eq. (7): <phi|Sigma(omega)|phi> = int Sigma(t) exp(-gamma^2 t^2 / 2)
  exp(i omega t) dt.  Reading: trapezoid rule on t_j = j dt,
  j = -N_tau..N_tau.  Sec. 3: N_tau ~ 3 / (gamma dt).
* Eq. (6): eps_QP = eps_KS + <phi|X + Sigma(eps_QP) - V_xc|phi>, using the
  real part of Sigma (the QP energy is real).
Readings:
* linearised solution: Z = 1 / (1 - d Re Sigma / d omega) at eps_KS,
  eps_lin = eps_KS + Z (X + Re Sigma(eps_KS) - v_xc);
* graphical solution: the root of
  f(omega) = eps_KS + X + Re Sigma(omega) - v_xc - omega
  nearest eps_lin: intervals of 1 mHa are scanned outwards from eps_lin
  (right then left at each distance) up to +-``search`` Ha, the first one
  with a sign change is bisected to 1e-10 Ha.
* error bar of the mean of per-sample values: std (ddof = 1) / sqrt(N).
"""
import numpy as np


def trapezoid_weights(n_tau):
    w = np.ones(2 * n_tau + 1)
    w[0] = w[-1] = 0.5
    return w


def sigma_omega(sig_t, dt, gamma, omega):
    """Sigma(omega) for Sigma(t_j), j = -N_tau..N_tau (last axis)."""
    sig_t = np.asarray(sig_t)
    n_tau = (sig_t.shape[-1] - 1) // 2
    t = dt * np.arange(-n_tau, n_tau + 1)
    wt = dt * trapezoid_weights(n_tau) * np.exp(-0.5 * gamma ** 2 * t ** 2)
    om = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    E = np.exp(1j * np.outer(om, t))                   # (n_omega, n_t)
    out = (sig_t * wt) @ E.T
    return out if np.ndim(omega) else out[..., 0]


def dsigma_domega(sig_t, dt, gamma, omega):
    sig_t = np.asarray(sig_t)
    n_tau = (sig_t.shape[-1] - 1) // 2
    t = dt * np.arange(-n_tau, n_tau + 1)
    wt = dt * trapezoid_weights(n_tau) * np.exp(-0.5 * gamma ** 2 * t ** 2)
    return np.sum(sig_t * wt * 1j * t * np.exp(1j * omega * t), axis=-1)


def default_gamma(n_tau, dt):
    """gamma = 3 / (N_tau dt), inverting N_tau ~ 3 / (gamma dt) (Sec. 3)."""
    return 3.0 / (n_tau * dt)


class NoRoot(RuntimeError):
    pass


def solve_root(f, x0, step=1e-3, tol=1e-10, search=2.0):
    """Root of f nearest x0 (scan outwards, then bisection)."""
    f0 = f(x0)
    if f0 == 0.0:
        return x0
    nsteps = int(np.ceil(search / step))
    for k in range(nsteps):
        for a, b in ((x0 + k * step, x0 + (k + 1) * step),
                     (x0 - (k + 1) * step, x0 - k * step)):
            fa, fb = f(a), f(b)
            if fa == 0.0:
                return a
            if fa * fb < 0.0:
                while b - a > tol:
                    m = 0.5 * (a + b)
                    fm = f(m)
                    if fa * fm <= 0.0:
                        b = m
                    else:
                        a, fa = m, fm
                return 0.5 * (a + b)
    raise NoRoot("no root of the QP equation within the search window")


def qp_from_sigma_w(sigma_w, dsigma_w, eps_ks, x, vxc, **kw):
    """Graphical and linearised QP energies for a callable Re/complex
    Sigma(omega) and its derivative."""
    d = float(np.real(dsigma_w(eps_ks)))
    Z = 1.0 / (1.0 - d)
    eps_lin = eps_ks + Z * (x + float(np.real(sigma_w(eps_ks))) - vxc)

    def f(w):
        return eps_ks + x + float(np.real(sigma_w(w))) - vxc - w

    eps_g = solve_root(f, eps_lin, **kw)
    return eps_g, eps_lin, Z


def qp_solve(sig_t, dt, gamma, eps_ks, x, vxc=0.0, **kw):
    """QP energies from the time series Sigma(t_j) (Eq. 6, Eq. 7)."""
    return qp_from_sigma_w(lambda w: sigma_omega(sig_t, dt, gamma, w),
                           lambda w: dsigma_domega(sig_t, dt, gamma, w),
                           eps_ks, x, vxc, **kw)


def mean_and_error(values):
    v = np.asarray(values, dtype=np.float64)
    return float(np.mean(v)), float(np.std(v, ddof=1) / np.sqrt(v.size))
