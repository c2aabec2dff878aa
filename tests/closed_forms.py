"""Closed forms used to pin the oracle (test helpers, not part of either side).

Everything here is computed from the eigenpairs of a small dense H, so it is
independent of the oracle's time stepping, Chebyshev expansions and sparse
projections.

* Casida / RPA.  For real KS orbitals (closed shell) the retarded RPA
  response is chi(t) = -2 theta(t) sum_n |rho_n><rho_n| sin(Omega_n t), where
  Omega_n^2 and F_n are the eigenpairs of C = D^2 + 4 D^1/2 K D^1/2
  (D_ja = e_a - e_j, K_{ja,kb} = <phi_j phi_a | v | phi_k phi_b>) and
  rho_n = sum_ja phi_j phi_a (D^1/2 F_n)_ja sqrt(2 / Omega_n).
* Stochastic single-sample forms: the response of the TDH with the exact
  occupied orbitals to the kick dv = v[phi zeta-bar] is
      u^R(r, t) = -2 sum_n sin(Omega_n t) V_n(r) <V_n|phi zeta-bar>,
  V_n = v rho_n, and the Green's-function orbitals are
      zeta^+(t)  = sum_a e^{-i e_a t} (1 - f_a) phi_a <phi_a|zeta-bar>
      zeta^-(-t) = -sum_a e^{+i e_a t} f_a phi_a <phi_a|zeta-bar>.
"""
import numpy as np

from oracle.tdh import hartree


def casida(grid, e, phi, n_occ):
    """Returns Omega (n,), V_n (n, N) = v rho_n."""
    occ, vir = phi[:n_occ], phi[n_occ:]
    no, nv = occ.shape[0], vir.shape[0]
    pairs = (occ[:, None, :] * vir[None, :, :]).reshape(no * nv, grid.N)
    D = (e[n_occ:][None, :] - e[:n_occ][:, None]).ravel()
    vp = hartree(grid, pairs)
    K = grid.dV * pairs @ vp.T
    K = 0.5 * (K + K.T)
    sD = np.sqrt(D)
    C = np.diag(D ** 2) + 4.0 * (sD[:, None] * K * sD[None, :])
    w2, F = np.linalg.eigh(C)
    Om = np.sqrt(w2)
    coef = (sD[:, None] * F) * np.sqrt(2.0 / Om)[None, :]   # (npair, n)
    Vn = (vp.T @ coef).T                                    # v rho_n
    return Om, Vn


def uR_closed(grid, Om, Vn, phi_k, zb, t):
    """u^R(r, t_j) for the kick v[phi_k zb] (rows: t_j)."""
    amp = grid.dV * Vn @ (phi_k * zb)                  # <V_n|phi zb>
    return -2.0 * (np.sin(np.outer(t, Om)) * amp[None, :]) @ Vn


def zeta_closed(grid, e, phi, f, zb, t):
    """zeta^+(t_j) and zeta^-(-t_j) for t_j >= 0 (rows: t_j)."""
    c = grid.dV * phi @ zb                              # <phi_a|zb>
    ph = np.exp(-1j * np.outer(t, e))
    zp = (ph * ((1.0 - f) * c)[None, :]) @ phi
    zm = -(np.conj(ph) * (f * c)[None, :]) @ phi
    return zp, zm
