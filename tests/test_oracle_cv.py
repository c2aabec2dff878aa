"""Pins of the control-variate oracle (features, network, Adam, estimator)
against closed forms, finite differences and known distributions."""
import numpy as np

from oracle import cv
from oracle.grid import Grid


def small_theta(rs, din, h1, h2, scale=0.5):
    n = h1 * din + h1 + h2 * h1 + h2 + h2 + 1
    return scale * rs.standard_normal(n)


def test_backprop_matches_central_differences():
    """dL/dtheta by the chain rule against central differences in FP64
    (step 1e-5: truncation ~1e-10, rounding ~1e-11): relative 1e-6."""
    rs = np.random.default_rng(0)
    din, h1, h2, n = 5, 7, 6, 11
    th = small_theta(rs, din, h1, h2)
    x = rs.standard_normal((n, din))
    y = rs.standard_normal(n)
    L, g = cv.loss_and_gradient(th, x, y, din, h1, h2)
    fd = np.empty_like(th)
    h = 1e-5
    for i in range(th.size):
        e = np.zeros_like(th)
        e[i] = h
        fd[i] = (cv.loss_and_gradient(th + e, x, y, din, h1, h2)[0]
                 - cv.loss_and_gradient(th - e, x, y, din, h1, h2)[0]) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-6 * np.max(np.abs(fd))
    assert abs(L - np.mean((cv.forward(th, x, din, h1, h2)[0] - y) ** 2)) < 1e-15 * max(L, 1)


def test_backprop_full_size_sampled_coordinates():
    """The 64 -> 256 -> 256 -> 1 network: 40 sampled coordinates of every
    parameter block against central differences."""
    rs = np.random.default_rng(1)
    th = small_theta(rs, 64, 256, 256, scale=0.05)
    x = rs.standard_normal((9, 64))
    y = rs.standard_normal(9)
    _, g = cv.loss_and_gradient(th, x, y)
    idx = np.unique(np.concatenate([rs.integers(0, th.size, 34), [0, 16384, 16640, 82176,
                                                                  82432, th.size - 1]]))
    h = 1e-5
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (cv.loss_and_gradient(th + e, x, y)[0] - cv.loss_and_gradient(th - e, x, y)[0]) / (2 * h)
        assert abs(g[i] - fd) < 1e-6 * max(abs(fd), 1e-3), i


def test_adam_closed_form_constant_gradient():
    """With a constant gradient the bias-corrected moments are exactly g and
    g^2 at every step, so each step moves theta by -lr g / (|g| + eps)."""
    rs = np.random.default_rng(2)
    th0 = rs.standard_normal(50)
    g = rs.standard_normal(50) * np.logspace(-6, 2, 50)
    opt = cv.Adam(50, lr=0.01)
    th = th0.copy()
    for t in range(1, 6):
        th = opt.step(th, g)
        expect = th0 - t * 0.01 * g / (np.abs(g) + 1e-8)
        assert np.allclose(th, expect, rtol=0, atol=1e-12), t


def test_adam_two_gradients_by_hand():
    """Two steps with gradients g1, g2 written out from the moment recursions."""
    g1, g2 = np.array([0.3, -2.0]), np.array([-0.1, 1.0])
    b1, b2, lr, eps = 0.9, 0.999, 0.05, 1e-8
    opt = cv.Adam(2, lr=lr, b1=b1, b2=b2, eps=eps)
    th = opt.step(np.zeros(2), g1)
    th = opt.step(th, g2)
    m2 = (1 - b1) * (b1 * g1 + g2)
    v2 = (1 - b2) * (b2 * g1 ** 2 + g2 ** 2)
    step1 = lr * g1 / (np.abs(g1) + eps)
    step2 = lr * (m2 / (1 - b1 ** 2)) / (np.sqrt(v2 / (1 - b2 ** 2)) + eps)
    assert np.allclose(th, -step1 - step2, rtol=1e-14, atol=0)


def test_features_parseval_complete_basis():
    """Over a complete dV-orthonormal basis, sum_k |<phi_k|zeta>|^2 = <zeta|zeta>
    = N (zeta = +-1/sqrt(dV)): exact for every sample."""
    g = Grid(4, h=0.6)
    rs = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rs.standard_normal((g.N, g.N)))
    phis = Q.T / np.sqrt(g.dV)
    x = cv.features(g, phis, seed=99, samples=[0, 1, 5, 77])
    assert np.allclose(x.sum(axis=1), g.N, rtol=1e-12)


def test_features_mean_is_norm():
    """E|<phi|zeta>|^2 = dV^2 sum phi^2 / dV = <phi|phi> = 1 for normalised phi
    (independent +-1 signs); variance 2 - 2 dV^2 sum phi^4 < 2."""
    g = Grid(8, h=0.5)
    rs = np.random.default_rng(4)
    phi = rs.standard_normal((3, g.N))
    phi /= np.sqrt(g.dV * np.sum(phi * phi, axis=1))[:, None]
    x = cv.features(g, phi, seed=5, samples=range(3000))
    assert np.all(np.abs(x.mean(axis=0) - 1.0) < 5 * np.sqrt(2.0 / 3000))


def test_features_eta_parseval_and_mean():
    """Occupied-orbital noise features: over a complete dV-orthonormal basis
    the mean over l of sum_k |<phi_k|eta_l>|^2 is <eta|eta> = N exactly; for a
    normalised phi the sample mean over 1500 samples x 4 vectors is 1 within
    5 standard errors (variance below 2 / 4 per sample)."""
    g = Grid(4, h=0.6)
    rs = np.random.default_rng(13)
    Q, _ = np.linalg.qr(rs.standard_normal((g.N, g.N)))
    x = cv.features_eta(g, Q.T / np.sqrt(g.dV), seed=99, samples=[0, 3, 70], n_eta=3)
    assert np.allclose(x.sum(axis=1), g.N, rtol=1e-12)
    g = Grid(8, h=0.5)
    phi = rs.standard_normal((2, g.N))
    phi /= np.sqrt(g.dV * np.sum(phi * phi, axis=1))[:, None]
    x = cv.features_eta(g, phi, seed=5, samples=range(1500), n_eta=4)
    assert np.all(np.abs(x.mean(axis=0) - 1.0) < 5 * np.sqrt(0.5 / 1500))


def test_features_eta_use_the_estimators_draws():
    """The eta-bar features of sample i are those of the white-noise set that
    the estimator filters for sample i (and not of another stream): against
    the projections of sigma.white_noise_sets' eta set."""
    from oracle.sigma import SGWParams, white_noise_sets
    g = Grid(8, h=0.5)
    rs = np.random.default_rng(14)
    phi = rs.standard_normal((3, g.N))
    p = SGWParams(seed=21, n_zeta=1, n_eta=6, n_tau=1, dt=0.1, m_sub=1, mu=0.0, beta=1.0,
                  ncoef=2, emin=-1.0, emax=1.0)
    for i in (0, 9):
        zb, eb = white_noise_sets(g, p, i)
        ref = np.mean((g.dV * eb @ phi.T) ** 2, axis=0)
        got = cv.features_eta(g, phi, 21, [i], 6)[0]
        assert np.allclose(got, ref, rtol=1e-13)
        assert not np.allclose(got, (g.dV * phi @ zb) ** 2, rtol=1e-3)


def test_cv_unbiased_and_variance_ratio():
    """y = 2 + 3 u + e (u, e standard normal), g = u with E[g] = 0: over 400
    repetitions the estimator's mean is 2 within 4 standard errors and its
    variance is (1 - rho^2) = 0.1 of the plain one."""
    rs = np.random.default_rng(6)
    nA, nB, reps = 200, 200, 400
    ests, plains = [], []
    for _ in range(reps):
        u = rs.standard_normal(nA + nB)
        y = 2.0 + 3.0 * u + rs.standard_normal(nA + nB)
        r = cv.cv_estimate(y[:nA], u[:nA], y[nA:], u[nA:], 0.0, 1.0, 10 ** 9)
        assert not r["fallback"]
        ests.append(r["estimate"])
        plains.append(np.mean(y[nA:]))
    ests, plains = np.array(ests), np.array(plains)
    assert abs(ests.mean() - 2.0) < 4 * ests.std(ddof=1) / np.sqrt(reps)
    ratio = ests.var(ddof=1) / plains.var(ddof=1)
    assert 0.07 < ratio < 0.14, ratio



def test_cv_exact_for_a_linear_relation():
    """If y = a + b g holds exactly, the fit gives c = b, every residual
    y - c g on B equals a, and the estimate is a + b mean_M(g) with the
    variance of that term alone, b^2 Var_M(g) / M."""
    rs = np.random.default_rng(8)
    g = rs.standard_normal(300)
    a, b = 1.25, -2.5
    y = a + b * g
    gm, gvar, M = 0.04, 0.9, 5000
    r = cv.cv_estimate(y[:150], g[:150], y[150:], g[150:], gm, gvar, M)
    assert np.isclose(r["c"], b, rtol=1e-12)
    assert not r["fallback"]
    assert abs(r["estimate"] - (a + b * gm)) < 1e-12
    assert abs(r["sigma_cv"] - abs(b) * np.sqrt(gvar / M)) < 1e-9

def test_cv_falls_back_on_a_biased_control_mean():
    rs = np.random.default_rng(7)
    u = rs.standard_normal(400)
    y = 1.0 + u + 0.1 * rs.standard_normal(400)
    ok = cv.cv_estimate(y[:200], u[:200], y[200:], u[200:], 0.0, 1.0, 10 ** 6)
    bad = cv.cv_estimate(y[:200], u[:200], y[200:], u[200:], 0.5, 1.0, 10 ** 6)
    assert not ok["fallback"] and bad["fallback"]
    assert bad["estimate"] == bad["plain"] == np.mean(y)
    assert ok["sigma"] < 0.2 * ok["sigma_plain"]


def test_training_fits_a_learnable_target():
    """Full-batch Adam lowers the loss of a smooth target of the features by
    more than 20x in 300 steps."""
    rs = np.random.default_rng(8)
    din, h1, h2 = 8, 32, 32
    x = rs.standard_normal((256, din))
    y = np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2]
    th = small_theta(rs, din, h1, h2, scale=0.3)
    th, hist = cv.train(th, x, y, 300, lr=3e-3, din=din, h1=h1, h2=h2)
    assert hist[-1] < hist[0] / 20
    assert np.all(np.isfinite(hist))


def test_forward_designed_values():
    """Weights chosen so every activation is a round number: tanh(atanh(0.6))
    = 0.6, tanh(atanh(0.8)) = 0.8, g = 2.5 * 0.8 - 1 = 1 (one unit per
    layer), and with two identical units per layer g = 2 (2.5 * 0.8) - 1 = 3."""
    th = np.array([np.arctanh(0.6), 0.0, np.arctanh(0.8) / 0.6, 0.0, 2.5, -1.0])
    g, (a1, a2) = cv.forward(th, np.array([[1.0]]), 1, 1, 1)
    assert np.allclose([a1[0, 0], a2[0, 0], g[0]], [0.6, 0.8, 1.0], rtol=1e-14)
    W1 = [np.arctanh(0.6)] * 2
    W2 = [np.arctanh(0.8) / 1.2] * 4
    th2 = np.array(W1 + [0.0, 0.0] + W2 + [0.0, 0.0] + [2.5, 2.5] + [-1.0])
    g2, _ = cv.forward(th2, np.array([[1.0]]), 1, 2, 2)
    assert abs(g2[0] - 3.0) < 1e-14
