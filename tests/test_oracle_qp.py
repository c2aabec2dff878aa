"""Pins for Sigma(omega) (Eq. 7) and the QP equation (Eq. 6)."""
import numpy as np
from scipy.special import wofz

from oracle import qp


def test_single_pole_roots():
    a, p = 0.3, -0.8
    for eks, x in ((-0.4, -0.1), (0.5, 0.2), (-2.0, 0.3)):
        e0 = eks + x
        sw = lambda w: a * a / (w - p)
        dsw = lambda w: -a * a / (w - p) ** 2
        eg, el, Z = qp.qp_from_sigma_w(sw, dsw, eks, x, 0.0)
        roots = [(e0 + p + s * np.sqrt((e0 - p) ** 2 + 4 * a * a)) / 2 for s in (1, -1)]
        best = min(roots, key=lambda r: abs(r - el))
        assert abs(eg - best) < 1e-9
        assert np.isclose(Z, 1 / (1 + a * a / (eks - p) ** 2))



def test_linear_sigma_solved_exactly():
    """For Sigma(w) = s0 + s1 (w - eps_KS) the QP equation (Eq. 6) is linear:
    eps = eps_KS + (X + s0 - v_xc) / (1 - s1).  One Newton step from eps_KS
    solves it, so the linearised energy equals it, as does the root, and
    Z = 1 / (1 - s1)."""
    for eks, x, vxc, s0, s1 in ((-0.4, -0.1, 0.05, 0.2, -0.3), (0.5, 0.2, -0.1, -0.15, 0.4)):
        sw = lambda w: s0 + s1 * (w - eks)
        eg, el, Z = qp.qp_from_sigma_w(sw, lambda w: s1, eks, x, vxc)
        exact = eks + (x + s0 - vxc) / (1.0 - s1)
        assert abs(el - exact) < 1e-14 and abs(eg - exact) < 1e-9
        assert np.isclose(Z, 1.0 / (1.0 - s1))


def test_quadrature_exact_for_linear_sigma():
    """Eq. 7 is integrated by the trapezoid rule on t_j = j dt,
    j = -N_tau..N_tau, which is exact for a linear integrand: with no damping
    (gamma = 0) and omega = 0, Sigma(t) = a + b t integrates to 2 a T,
    T = N_tau dt, whatever b."""
    dt, n_tau = 0.05, 40
    t = dt * np.arange(-n_tau, n_tau + 1)
    for a, b in ((1.0, 0.0), (0.3 - 0.2j, 1.7)):
        val = qp.sigma_omega(a + b * t, dt, 0.0, 0.0)
        assert abs(val - 2.0 * a * n_tau * dt) < 1e-12

def test_damped_transform_of_single_pole():
    """Sigma(t) = -i a^2 e^{-i p t} theta(t) (Sigma(0) = half the limit):
    int_0^inf Sigma(t) e^{-g^2 t^2/2} e^{i w t} dt
      = -i a^2 sqrt(pi/2)/g w((w - p) / (sqrt(2) g)),  w = Faddeeva."""
    a, p, gam, dt, nt = 0.4, -0.5, 0.15, 0.01, 3000
    t = dt * np.arange(-nt, nt + 1)
    sig = np.where(t > 0, -1j * a * a * np.exp(-1j * p * t), 0.0)
    sig[nt] = -0.5j * a * a
    om = np.linspace(-1.5, 0.5, 9)
    num = qp.sigma_omega(sig, dt, gam, om)
    ref = -1j * a * a * np.sqrt(np.pi / 2) / gam * wofz((om - p) / (np.sqrt(2) * gam))
    assert np.max(np.abs(num - ref)) < 1e-5
    # derivative of the damped transform vs centred differences of itself
    h = 1e-5
    for w in om[:3]:
        fd = (qp.sigma_omega(sig, dt, gam, w + h) - qp.sigma_omega(sig, dt, gam, w - h)) / (2 * h)
        assert abs(qp.dsigma_domega(sig, dt, gam, w) - fd) < 1e-6


def test_default_gamma_inverts_tau_count():
    # N_tau = 3 / (gamma dt): gamma = 0.06, dt = 0.05 gives 1000 (Sec. 3)
    assert np.isclose(qp.default_gamma(1000, 0.05), 0.06)


def test_no_root_raises():
    # f(w) = 1 + Sigma(w) - w = 6 + w^2/2 never vanishes
    sw = lambda w: w + 5.0 + 0.5 * w * w
    try:
        qp.qp_from_sigma_w(sw, lambda w: 1.0 + w, 1.0, 0.0, 0.0, search=1.0)
    except qp.NoRoot:
        return
    raise AssertionError("expected NoRoot")
