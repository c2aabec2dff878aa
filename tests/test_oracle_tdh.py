"""Pins for the TDH linear-response propagation (first phase, Sec. 2.1)."""
import numpy as np
import scipy.linalg as sla

from closed_forms import casida, uR_closed
from oracle.tdh import TDH, apply_kb_exponential, finite_lambda_response, hartree, \
    kb_exponential_matrix


def test_kb_exponential_is_exact(tiny8):
    s, H = tiny8
    g = H.grid
    B = H.kb.B.toarray()
    A = g.dV * B @ np.diag(H.kb.ekb) @ B.T
    for tau in (0.025, 0.3):
        K = kb_exponential_matrix(H.kb, tau)
        psi = np.random.default_rng(4).standard_normal((2, g.N)) + 0j
        out = apply_kb_exponential(H.kb, K, psi)
        exact = psi @ sla.expm(-1j * tau * A).T
        assert np.max(np.abs(out - exact)) < 1e-12


def _setup_det(tiny8, tiny8_eig):
    s, H = tiny8
    e, V = tiny8_eig
    g = H.grid
    n_occ = s.n_occ
    phi_k = V[n_occ - 1]
    zb = np.random.default_rng(5).choice([-1.0, 1.0], g.N) / np.sqrt(g.dV)
    dv = hartree(g, phi_k * zb)
    return s, H, e, V, g, n_occ, phi_k, zb, dv


def test_tdh_matches_casida(tiny8, tiny8_eig):
    """TDH with the exact occupied orbitals (weight 2) reproduces the RPA
    response u^R(t) = -2 sum_n sin(Omega_n t) V_n <V_n|phi zeta-bar>, with a
    splitting error that falls as dt^2."""
    s, H, e, V, g, n_occ, phi_k, zb, dv = _setup_det(tiny8, tiny8_eig)
    Om, Vn = casida(g, e, V, n_occ)
    n_out, dt = 8, 0.2
    t = dt * np.arange(n_out + 1)
    exact = uR_closed(g, Om, Vn, phi_k, zb, t)
    errs = []
    for m_sub in (4, 8, 16):
        tdh = TDH(H, dt / m_sub, 2.0)
        uR = tdh.run(V[:n_occ], dv, n_out, m_sub)
        errs.append(np.max(np.abs(uR - exact)) / np.max(np.abs(exact)))
    assert errs[-1] < 1e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0
    assert np.max(np.abs(uR[0])) == 0.0


def test_tdh_norm_conservation(tiny8, tiny8_eig):
    s, H, e, V, g, n_occ, phi_k, zb, dv = _setup_det(tiny8, tiny8_eig)
    eta = np.random.default_rng(6).standard_normal((3, g.N))
    tdh = TDH(H, 0.05, 2.0 / 3)
    st = tdh.start(eta, dv)
    n0 = g.norm2(st[0])
    for _ in range(40):
        st = tdh.substep(*st)
    assert np.allclose(g.norm2(st[0]), n0, rtol=1e-12)


def test_finite_lambda_converges_to_linearised(tiny8, tiny8_eig):
    """The paper's finite-difference response approaches the tangent form:
    one-sided at O(lambda), central at O(lambda^2)."""
    s, H, e, V, g, n_occ, phi_k, zb, dv = _setup_det(tiny8, tiny8_eig)
    eta = np.random.default_rng(7).standard_normal((4, g.N)) * 0.5
    tau, n_out, m_sub = 0.05, 6, 2
    lin = TDH(H, tau, 2.0 / 4).run(eta, dv, n_out, m_sub)
    scale = np.max(np.abs(lin))
    d = []
    for lam in (1e-2, 5e-3):
        fd = finite_lambda_response(H, tau, 2.0 / 4, eta, dv, lam, n_out, m_sub)
        cd = finite_lambda_response(H, tau, 2.0 / 4, eta, dv, lam, n_out, m_sub,
                                    central=True)
        d.append((np.max(np.abs(fd - lin)) / scale, np.max(np.abs(cd - lin)) / scale))
    assert 1.7 < d[0][0] / d[1][0] < 2.3          # O(lambda)
    assert 3.4 < d[0][1] / d[1][1] < 4.6          # O(lambda^2)
    assert d[1][1] < 1e-4
