"""Time-dependent Hartree (TDH) linear response for W (oracle side).

Sec. 2.1 (first phase): a perturbed copy eta^lambda of every filtered
stochastic occupied orbital eta_l is propagated together with the unperturbed
copy under the time-dependent Hamiltonian; the causal response u^R(r, t) is
the difference of the two time-dependent potentials.  Sec. 2.3 packs the two
copies side by side; the density rho(r, t) is needed at every step.  The
propagation uses the split-operator scheme with dt = 0.05 a.u. (Sec. 3).

Readings (the paper defers the equations to its references):
* H^c(t) = H_0 + v_H[n^c(t)] - v_H[n(0)] for either copy c, with
  n^c(t) = w sum_l |eta^c_l(r, t)|^2, w = 2 / N_eta (closed shell).
* The perturbation is an impulsive kick eta^lambda(0) = exp(-i lambda dv) eta
  with dv = v_H[phi * zeta-bar] (Sec. 2.1 perturbs with a potential built
  from the random vector zeta-bar).
* u^R(t) = (v_H[n^lambda(t)] - v_H[n(t)]) / lambda.  The canonical form used
  by the library is its lambda -> 0 limit: the exact tangent map of the
  Strang step, carried by delta-eta with delta-eta(0) = -i dv eta(0) and
  u^R(t) = v_H[delta n(t)], delta n = w sum_l 2 Re(conj(eta_l) delta-eta_l).
  ``finite_lambda_response`` keeps the paper's finite-difference form.
* v_H[rho] = F^{-1}[ 4 pi / |k|^2 F[rho] ] with the k = 0 term dropped
  (periodic box, neutralising background).
* One Strang substep of length tau:
      local half step  exp(-i V(t) tau/2)
      KB half step     exp(-i V_NL tau/2)
      kinetic step     F^{-1} exp(-i T tau) F
      KB half step     exp(-i V_NL tau/2)
      density n(t+tau), delta n(t+tau)  ->  V(t+tau), u^R(t+tau)
      local half step  exp(-i V(t+tau) tau/2)
  The last local half step changes neither n nor delta n, so the potentials
  of step 5 are those of the state at t + tau.
"""
import numpy as np
import scipy.linalg as sla

from .grid import Grid


def coulomb_kernel(grid: Grid):
    k2 = grid.k2()
    vk = np.zeros_like(k2)
    nz = k2 > 0
    vk[nz] = 4.0 * np.pi / k2[nz]
    return vk


def hartree(grid: Grid, rho):
    """v_H[rho] for real rho of shape (..., N) (returns the real part)."""
    return np.real(grid.ifft(coulomb_kernel(grid) * grid.fft(rho)))


def kb_exponential_matrix(kb, tau):
    """K with exp(-i tau V_NL) = I + dV B K B^T  (exact for the separable
    V_NL = dV B E B^T):  K = (-i tau) E phi1(-i tau S E),
    phi1(X) = sum_k X^k / (k+1)!, evaluated with the block-matrix
    exponential expm([[X, I], [0, 0]]) = [[e^X, phi1(X)], [0, I]]."""
    S = kb.gram()
    E = np.diag(kb.ekb)
    n = S.shape[0]
    X = -1j * tau * (S @ E)
    Z = np.zeros((2 * n, 2 * n), dtype=np.complex128)
    Z[:n, :n] = X
    Z[:n, n:] = np.eye(n)
    phi1 = sla.expm(Z)[:n, n:]
    return (-1j * tau) * (E @ phi1)


def apply_kb_exponential(kb, K, psi):
    if kb is None:
        return psi
    C = kb.project(psi)            # (nvec, Np), includes dV
    return psi + kb.expand(C @ K.T)


class TDH:
    """Linear-response TDH propagation for one Monte Carlo sample."""

    def __init__(self, H, tau, weight):
        self.H = H
        self.grid = H.grid
        self.tau = float(tau)
        self.w = float(weight)
        self.prop_T = np.exp(-1j * H.T * self.tau)
        self.K = None
        if H.kb is not None:
            self.K = kb_exponential_matrix(H.kb, 0.5 * self.tau)

    def kb_half(self, psi):
        return apply_kb_exponential(self.H.kb, self.K, psi) if self.K is not None else psi

    def kinetic(self, psi):
        return self.grid.ifft(self.prop_T * self.grid.fft(psi))

    def densities(self, eta, deta):
        n = self.w * np.sum(np.abs(eta) ** 2, axis=0)
        dn = self.w * np.sum(2.0 * np.real(np.conj(eta) * deta), axis=0)
        return n, dn

    def start(self, eta, dv):
        """Initial state: eta(0), delta-eta(0) = -i dv eta(0)."""
        eta = np.array(eta, dtype=np.complex128)
        deta = -1j * dv[None, :] * eta
        n0, dn0 = self.densities(eta, deta)
        self.vh_n0 = hartree(self.grid, n0)
        v = self.H.v.copy()
        u = hartree(self.grid, dn0)
        return eta, deta, v, u

    def local_half(self, eta, deta, v, u):
        ph = np.exp(-0.5j * self.tau * v)[None, :]
        deta = ph * (deta - 0.5j * self.tau * u[None, :] * eta)
        eta = ph * eta
        return eta, deta

    def substep(self, eta, deta, v, u):
        eta, deta = self.local_half(eta, deta, v, u)
        eta, deta = self.kb_half(eta), self.kb_half(deta)
        eta, deta = self.kinetic(eta), self.kinetic(deta)
        eta, deta = self.kb_half(eta), self.kb_half(deta)
        n, dn = self.densities(eta, deta)
        v = self.H.v + hartree(self.grid, n) - self.vh_n0
        u = hartree(self.grid, dn)
        eta, deta = self.local_half(eta, deta, v, u)
        return eta, deta, v, u

    def run(self, eta, dv, n_out, m_sub, store_field=False):
        """u^R at t_j = j * m_sub * tau, j = 0..n_out.  Returns an
        (n_out+1, N) array of u^R(r, t_j)."""
        eta, deta, v, u = self.start(eta, dv)
        out = np.empty((n_out + 1, self.grid.N))
        out[0] = u
        for j in range(1, n_out + 1):
            for _ in range(m_sub):
                eta, deta, v, u = self.substep(eta, deta, v, u)
            out[j] = u
        return out


def finite_lambda_response(H, tau, weight, eta, dv, lam, n_out, m_sub,
                           central=False):
    """The paper's form: propagate the unperturbed copy and the kicked copy
    exp(-i lam dv) eta with the non-linear TDH Strang step and return
    (v_H[n^lam] - v_H[n^0]) / lam  (or the central difference)."""
    grid = H.grid
    K = kb_exponential_matrix(H.kb, 0.5 * tau) if H.kb is not None else None
    pT = np.exp(-1j * H.T * tau)
    eta = np.array(eta, dtype=np.complex128)
    n0 = weight * np.sum(np.abs(eta) ** 2, axis=0)
    vh0 = hartree(grid, n0)

    def step(psi, v):
        psi = np.exp(-0.5j * tau * v)[None, :] * psi
        if K is not None:
            psi = apply_kb_exponential(H.kb, K, psi)
        psi = grid.ifft(pT * grid.fft(psi))
        if K is not None:
            psi = apply_kb_exponential(H.kb, K, psi)
        n = weight * np.sum(np.abs(psi) ** 2, axis=0)
        vh = hartree(grid, n)
        v = H.v + vh - vh0
        psi = np.exp(-0.5j * tau * v)[None, :] * psi
        return psi, v, vh

    def trajectory(psi):
        v = H.v.copy()
        vhs = [vh0.copy()]
        for _ in range(n_out):
            for _ in range(m_sub):
                psi, v, vh = step(psi, v)
            vhs.append(vh)
        return np.array(vhs)

    base = trajectory(eta)
    plus = trajectory(np.exp(-1j * lam * dv)[None, :] * eta)
    if central:
        minus = trajectory(np.exp(1j * lam * dv)[None, :] * eta)
        return (plus - minus) / (2 * lam)
    return (plus - base) / lam
