"""Learned control variate for the per-sample self-energy (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is an addition to the paper's estimator, not part of it.  The paper
averages independent Monte Carlo samples until the statistical error of the
QP energies is below 0.03 eV (Sec. 3, 1024 samples); per sample, y_i = X_i +
Re Sigma_c,i(omega) enters the QP equation (Eq. 6) linearly, so the spread of
y_i sets that error.  A control
variate g(x_i), computed from cheap features x_i of the same random vector,
lowers that spread without bias when E[g] is known well:

  features   x_{i,k} = |<phi_k|zeta_i>|^2, k = 1..K, zeta_i the white noise of
             sample i (+-1/sqrt(dV), the same draw the sample's filter uses),
             and the same over the sample's occupied-orbital noise eta-bar_{i,l},
             averaged over l (features_eta);
  network    g(x) = w3 . tanh(W2 tanh(W1 xh + b1) + b2) + b3,
             xh = (x - mean) / std with training-set statistics;
  training   mean squared error (1/n) sum (g(x_i) - y_i)^2, full-batch Adam;
  estimator  c = Cov_A(y, g) / Var_A(g) on the fit set A,
             S_cv = mean_B(y - c g) + c mean_M(g)  over an evaluation set B and
             M cheap samples (features only), with variance
             Var_B(y - c g) / n_B + c^2 Var_M(g) / M;  the plain mean of y over
             A and B serves as a check: when |S_cv - S_plain| exceeds three
             combined standard deviations the plain estimate is returned.

Readings (the method has no source for these details): tanh activation (so
finite differences are clean); Glorot-uniform initial weights supplied as an
input; Adam with the bias-corrected moments of Kingma & Ba (ICLR 2015); ddof
= 1 in every sample variance; the fallback threshold uses
sqrt(sigma_cv^2 + sigma_plain^2).
"""
import numpy as np

from . import rng


# ------------------------------------------------------------------ features
def features(grid, phis, seed, samples):
    """x[i, k] = |<phi_k|zeta_i>|^2 with <f|g> = dV sum f g, zeta_i the white
    noise of sample ``samples[i]`` (stream kind ZETA, l = 0)."""
    phis = np.atleast_2d(np.asarray(phis, dtype=np.float64))
    out = np.empty((len(samples), phis.shape[0]))
    for j, s in enumerate(samples):
        z = rng.white_noise(seed, rng.ZETA, int(s), 0, grid.N, grid.dV)
        a = grid.dV * (phis @ z)
        out[j] = a * a
    return out


def features_eta(grid, phis, seed, samples, n_eta):
    """x[i, k] = (1/n_eta) sum_l |<phi_k|eta-bar_{i,l}>|^2 over the occupied-
    orbital white noise of sample ``samples[i]`` (stream kind ETA, l = 0 ..
    n_eta - 1): the draws whose filtered images give the sample's density and
    its exchange X_i (Sec. 2.1)."""
    phis = np.atleast_2d(np.asarray(phis, dtype=np.float64))
    out = np.zeros((len(samples), phis.shape[0]))
    for j, s in enumerate(samples):
        for l in range(n_eta):
            e = rng.white_noise(seed, rng.ETA, int(s), l, grid.N, grid.dV)
            a = grid.dV * (phis @ e)
            out[j] += a * a
    return out / n_eta


def standardization(x):
    """Per-feature mean and standard deviation (ddof = 0) of the training
    features; a constant feature gets std 1."""
    m = x.mean(axis=0)
    s = x.std(axis=0)
    s[s == 0] = 1.0
    return m, s


# ------------------------------------------------------------------ network
def unpack(theta, din=64, h1=256, h2=256):
    """Views W1 [h1][din], b1, W2 [h2][h1], b2, w3 [h2], b3 of the packed
    parameter vector."""
    o = 0
    W1 = theta[o:o + h1 * din].reshape(h1, din); o += h1 * din
    b1 = theta[o:o + h1]; o += h1
    W2 = theta[o:o + h2 * h1].reshape(h2, h1); o += h2 * h1
    b2 = theta[o:o + h2]; o += h2
    w3 = theta[o:o + h2]; o += h2
    b3 = theta[o:o + 1]; o += 1
    assert o == theta.size
    return W1, b1, W2, b2, w3, b3


def forward(theta, xh, din=64, h1=256, h2=256):
    """g for standardized features xh [n][din]; returns g and the hidden
    activations."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, din, h1, h2)
    a1 = np.tanh(xh @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    g = a2 @ w3 + b3[0]
    return g, (a1, a2)


def loss_and_gradient(theta, xh, y, din=64, h1=256, h2=256):
    """L = (1/n) sum (g_i - y_i)^2 and dL/dtheta (packed like theta) by the
    chain rule through the two tanh layers."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, din, h1, h2)
    g, (a1, a2) = forward(theta, xh, din, h1, h2)
    n = xh.shape[0]
    r = g - y
    L = float(np.mean(r * r))
    dg = 2.0 * r / n                       # dL/dg_i
    dw3 = a2.T @ dg
    db3 = np.array([dg.sum()])
    d2 = np.outer(dg, w3) * (1.0 - a2 * a2)   # dL/d(pre-activation 2)
    dW2 = d2.T @ a1
    db2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1.0 - a1 * a1)
    dW1 = d1.T @ xh
    db1 = d1.sum(axis=0)
    grad = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, db3])
    return L, grad


class Adam:
    """Adam with bias-corrected moments: m = b1 m + (1 - b1) g,
    v = b2 v + (1 - b2) g^2, theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, size, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(size)
        self.v = np.zeros(size)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, grad):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * grad
        self.v = self.b2 * self.v + (1.0 - self.b2) * grad * grad
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def train(theta, xh, y, steps, lr=1e-3, din=64, h1=256, h2=256):
    """Full-batch Adam on the mean squared error; returns the parameters and
    the loss before each step."""
    opt = Adam(theta.size, lr=lr)
    hist = []
    for _ in range(steps):
        L, gr = loss_and_gradient(theta, xh, y, din, h1, h2)
        hist.append(L)
        theta = opt.step(theta, gr)
    return theta, np.array(hist)


# ------------------------------------------------------------------ estimator
def cv_estimate(yA, gA, yB, gB, gM_mean, gM_var, M):
    """Control-variate estimate of E[y] with the plain mean as fallback."""
    yA, gA, yB, gB = (np.asarray(a, dtype=np.float64) for a in (yA, gA, yB, gB))
    vg = np.var(gA, ddof=1)
    c = float(np.cov(yA, gA, ddof=1)[0, 1] / vg) if vg > 0 else 0.0
    rB = yB - c * gB
    est = float(rB.mean() + c * gM_mean)
    var_cv = float(np.var(rB, ddof=1) / yB.size + c * c * gM_var / M)
    yall = np.concatenate([yA, yB])
    plain = float(yall.mean())
    var_plain = float(np.var(yall, ddof=1) / yall.size)
    fallback = abs(est - plain) > 3.0 * np.sqrt(var_cv + var_plain)
    rho = float(np.corrcoef(yA, gA)[0, 1]) if vg > 0 else 0.0
    if fallback:
        return dict(estimate=plain, sigma=np.sqrt(var_plain), c=c, rho2=rho * rho,
                    plain=plain, sigma_plain=np.sqrt(var_plain), fallback=True,
                    sigma_cv=np.sqrt(var_cv))
    return dict(estimate=est, sigma=np.sqrt(var_cv), c=c, rho2=rho * rho, plain=plain,
                sigma_plain=np.sqrt(var_plain), fallback=False, sigma_cv=np.sqrt(var_cv))
