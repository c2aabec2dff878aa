"""Pins for the retarded -> time-ordered conversion (Sec. 2.1, Sec. 2.3)."""
import numpy as np
from scipy.integrate import quad

from oracle.timeorder import default_nft, time_order


def test_real_part_is_half_the_causal_signal():
    rs = np.random.default_rng(0)
    f = rs.standard_normal((3, 51))
    g = time_order(f)
    assert np.allclose(g[:, 1:].real, 0.5 * f[:, 1:], atol=1e-13)
    assert np.allclose(g[:, 0].real, f[:, 0], atol=1e-13)


def test_even_in_time():
    f = np.random.default_rng(1).standard_normal(40)
    N = default_nft(39)
    buf = np.zeros(N)
    buf[:40] = f
    F = N * np.fft.ifft(buf)
    k = np.fft.fftfreq(N) * N
    F[k < 0] = np.conj(F[k < 0])
    full = np.fft.fft(F) / N
    assert np.allclose(full[1:40], full[::-1][:39], atol=1e-13)   # g(-t) = g(t)


def test_damped_mode_against_continuous_transform():
    """u^R(t) = -2 sin(W t) e^{-k t} theta(t): the time-ordered function is
    g(t) = (1/pi) int_0^inf F(w) cos(w t) dw with
    F(w) = 1/(w - W + ik) - 1/(w + W + ik)  (Im part by quadrature)."""
    W, kap, dt, nt = 1.0, 0.3, 0.02, 2000
    t = dt * np.arange(nt + 1)
    f = -2 * np.sin(W * t) * np.exp(-kap * t)
    g = time_order(f, n_ft=8 * 2048)

    def imF(w):
        return -kap / ((w - W) ** 2 + kap ** 2) + kap / ((w + W) ** 2 + kap ** 2)

    for j in (25, 50, 100, 200, 400):
        ref, _ = quad(imF, 0, np.inf, weight="cos", wvar=t[j], limlst=200)
        assert abs(g[j].imag - ref / np.pi) < 2e-3 * np.max(np.abs(f))
    # undamped limit: single RPA mode -> -i e^{-i W |t|}  (|err| ~ kappa)
