"""Retarded -> time-ordered conversion (oracle side).

Sec. 2.1 time-orders the accumulated causal response u^R(r, t) into u(r, t);
Sec. 2.3 does so with an FFT along t, a complex conjugation, and an inverse
FFT.  With the convention F(omega) = int f(t) e^{i omega t} dt, the
time-ordered response equals the retarded one for omega > 0 and its complex
conjugate for omega < 0.

Discrete reading (the paper gives no discretisation):
* f_j = u^R(t_j), t_j = j dt, j = 0..N_tau, zero for t < 0 and beyond
  N_tau, placed in a periodic buffer of N_FT >= 4 (N_tau + 1) points
  (the smallest power of two, by default);
* F_k = sum_j f_j e^{+i omega_k t_j},  omega_k = 2 pi k / (N_FT dt),
  k in (-N_FT/2, N_FT/2];
* G_k = conj(F_k) for omega_k < 0, G_k = F_k otherwise;
* g_j = (1/N_FT) sum_k G_k e^{-i omega_k t_j}, kept for j = 0..N_tau.
For real f the result is even in t (G_k = G_{-k}), so the negative-time half
is g_{-j} = g_j, and Re g_j = f_j / 2 for j > 0.
"""
import numpy as np


def default_nft(n_tau):
    n = 1
    while n < 4 * (n_tau + 1):
        n *= 2
    return n


def time_order(f, n_ft=None):
    """Time-order causal samples f[..., 0..N_tau] along the last axis."""
    f = np.asarray(f)
    nt1 = f.shape[-1]
    N = default_nft(nt1 - 1) if n_ft is None else int(n_ft)
    if N < 2 * nt1:
        raise ValueError("N_FT too small")
    buf = np.zeros(f.shape[:-1] + (N,), dtype=np.complex128)
    buf[..., :nt1] = f
    k = np.fft.fftfreq(N) * N            # signed integer frequencies
    # F_k = sum_j f_j exp(+2 pi i k j / N)  ==  N * ifft(f)
    F = N * np.fft.ifft(buf, axis=-1)
    neg = k < 0
    F[..., neg] = np.conj(F[..., neg])
    # g_j = (1/N) sum_k G_k exp(-2 pi i k j / N)  ==  fft(G) / N
    g = np.fft.fft(F, axis=-1) / N
    return g[..., :nt1]
