"""Stochastic estimate of <phi|Sigma_c(t)|phi> and of the exchange X.

Follows Sec. 2.1 step by step for each Monte Carlo sample i:
 1. white-noise zeta-bar_i and eta-bar_{i,l} (l = 1..N_eta)            [rng]
 2. filter both sets with the Chebyshev occupied-space filter, Eq. (3):
    zeta_i = F(H) zeta-bar_i,  eta_{i,l} = F(H) eta-bar_{i,l}
 3. first phase: TDH linear response to dv_i = v_H[phi zeta-bar_i] gives
    u^R_i(r, t); it is accumulated in the sparse xi basis (or kept on the
    full grid in "exact" mode) and time-ordered to u_i(r, t)
 4. second phase: the occupied part zeta_i is propagated backwards in time
    and its complement zeta-bar_i - zeta_i forwards (Sec. 2.1, Sec. 2.3),
    the stochastic Green's function of Eq. (4)
 5. Eq. (5): Sigma_i(t) = int phi(r) zeta_i(r, t) u_i(r, t) dr
 6. exchange X_i in the eta basis (Sec. 2.1, after Eq. 6)

Readings:
* iG(t) = theta(t) (1 - P) e^{-iHt} - theta(-t) P e^{-iHt}, with P -> F(H):
  zeta^+(t) = U(t) (zeta-bar - zeta),  zeta^-(-t) = -U(-t) zeta  (t >= 0).
  Sigma(t = 0) is the mean of the two one-sided limits.
* xi mode: u_i(r, t) ~ sum_m xi_m(r) c_m(t), c_m = time-ordered <xi_m|u^R_i>,
  so Sigma_i(t_j) = sum_m c_m(t_|j|) d^{sgn j}_m(t_j),
  d^{+-}_m(t_j) = <xi_m| phi zeta^{+-}(t_j)>  (xi real).
* X_i = -(1/N_eta) sum_l <phi eta_l| v_H[phi eta_l]>, no spin factor
  (exchange acts within one spin channel).
* Time axis: N_tau output steps of dt each side; the TDH output steps are
  split into m_sub Strang substeps of dt / m_sub.
"""
from dataclasses import dataclass

import numpy as np

from . import chebyshev as cheb
from . import rng
from .sroi import XiBasis
from .tdh import TDH, hartree
from .timeorder import time_order


@dataclass
class SGWParams:
    seed: int
    n_zeta: int
    n_eta: int
    n_tau: int
    dt: float
    m_sub: int
    mu: float
    beta: float
    ncoef: int
    emin: float
    emax: float
    n_xi: int = 10000
    f_g: float = 0.003
    mode: str = "xi"          # "xi" or "exact"
    prop_tol: float = 1e-14
    n_ft: int = None
    first_sample: int = 0
    filter: str = "fermi"     # "fermi" (mu, beta) or "gapped" (e_homo, e_lumo, eps)
    e_homo: float = 0.0
    e_lumo: float = 0.0
    filter_eps: float = 1e-7


def white_noise_sets(grid, p: SGWParams, i):
    zb = rng.white_noise(p.seed, rng.ZETA, i, 0, grid.N, grid.dV)
    eb = np.stack([rng.white_noise(p.seed, rng.ETA, i, l, grid.N, grid.dV)
                   for l in range(p.n_eta)])
    return zb, eb


def exchange(grid, phi, eta):
    """X = -(1/N_eta) sum_l <phi eta_l | v_H[phi eta_l]> for real eta."""
    pe = phi[None, :] * np.atleast_2d(eta)
    return -np.mean(grid.dV * np.sum(pe * hartree(grid, pe), axis=1))


def sample_sigma(H, phi, p: SGWParams, i, return_parts=False,
                 zb=None, eta_det=None, eta_weight=None):
    """Sigma_i(t_j), j = -N_tau..N_tau (complex, length 2 N_tau + 1), and
    X_i for Monte Carlo sample number i.

    Test hooks: ``zb`` replaces the white-noise zeta-bar_i; ``eta_det``
    replaces the filtered eta set by given orbitals with density weight
    ``eta_weight`` (deterministic limits)."""
    grid = H.grid
    phi = np.asarray(phi, dtype=np.float64)
    zb_rng, eb = white_noise_sets(grid, p, i)
    zb = zb_rng if zb is None else np.asarray(zb, dtype=np.float64)

    # 2. filter (both sets with the same F, Sec. 2.1)
    if p.filter == "gapped":
        a = cheb.gapped_coefficients(p.e_homo, p.e_lumo, p.filter_eps, p.emin, p.emax, p.ncoef)
    else:
        a = cheb.fermi_coefficients(p.mu, p.beta, p.emin, p.emax, p.ncoef)
    if eta_det is None:
        filt = cheb.apply_series(H, a, p.emin, p.emax, np.vstack([zb[None], eb]))
        z_occ, eta = filt[0], filt[1:]
        weight = 2.0 / p.n_eta
    else:
        z_occ = cheb.apply_series(H, a, p.emin, p.emax, zb[None])[0]
        eta = np.asarray(eta_det)
        weight = float(eta_weight)
    z_un = zb - z_occ

    # 6. exchange
    X = exchange(grid, phi, eta)

    # 3. first phase: TDH
    dv = hartree(grid, phi * zb)
    tau = p.dt / p.m_sub
    tdh = TDH(H, tau, weight)
    uR = tdh.run(eta, dv, p.n_tau, p.m_sub)          # (n_tau+1, N)

    # 4. second phase: G
    bp = cheb.propagator_coefficients(p.emin, p.emax, p.dt, p.prop_tol)
    bm = cheb.propagator_coefficients(p.emin, p.emax, -p.dt, p.prop_tol)
    zp = z_un.astype(np.complex128)
    zm = -z_occ.astype(np.complex128)
    zps, zms = [zp], [zm]
    for _ in range(p.n_tau):
        zp = cheb.apply_series(H, bp, p.emin, p.emax, zp)
        zm = cheb.apply_series(H, bm, p.emin, p.emax, zm)
        zps.append(zp)
        zms.append(zm)
    zps, zms = np.array(zps), np.array(zms)          # (n_tau+1, N)

    # 5. contraction
    if p.mode == "exact":
        u = time_order(uR.T, p.n_ft).T                # (n_tau+1, N)
        sp = grid.dV * np.sum(phi[None] * zps * u, axis=1)
        sm = grid.dV * np.sum(phi[None] * zms * u, axis=1)
        parts = dict(u=u, uR=uR)
    else:
        xi = XiBasis(p.seed, i, grid.N, p.n_xi, p.f_g, grid.dV)
        cR = np.array([xi.overlaps(uR[j]) for j in range(p.n_tau + 1)]).T
        c = time_order(cR, p.n_ft)                    # (n_xi, n_tau+1)
        dp = np.array([xi.overlaps(phi * zps[j]) for j in range(p.n_tau + 1)]).T
        dm = np.array([xi.overlaps(phi * zms[j]) for j in range(p.n_tau + 1)]).T
        sp = np.sum(c * dp, axis=0)
        sm = np.sum(c * dm, axis=0)
        parts = dict(cR=cR, c=c, dp=dp, dm=dm, uR=uR)
    sig = np.empty(2 * p.n_tau + 1, dtype=np.complex128)
    sig[p.n_tau + 1:] = sp[1:]
    sig[:p.n_tau] = sm[1:][::-1]
    sig[p.n_tau] = 0.5 * (sp[0] + sm[0])
    if return_parts:
        parts.update(z_occ=z_occ, eta=eta, zps=zps, zms=zms, dv=dv, zb=zb, eb=eb)
        return sig, X, parts
    return sig, X


def estimate(H, phi, p: SGWParams):
    """Per-sample Sigma_i(t) (n_zeta, 2 N_tau + 1) and X_i (n_zeta,)."""
    sig = np.empty((p.n_zeta, 2 * p.n_tau + 1), dtype=np.complex128)
    X = np.empty(p.n_zeta)
    for s in range(p.n_zeta):
        sig[s], X[s] = sample_sigma(H, phi, p, p.first_sample + s)
    return sig, X
