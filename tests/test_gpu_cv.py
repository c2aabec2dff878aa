"""GPU parity of the learned control variate: features, network forward and
gradient, Adam, training, cheap-sample moments, and the gain over the plain
estimator on real per-sample Sigma values.

Two references: the FP64 oracle (tolerances from BF16 operand rounding,
u = 2^-9) and, for tight checks, a model of the kernels' own arithmetic in
this file: every GEMM operand rounded to BF16 (nearest even), everything else
in FP64."""
import numpy as np
import pytest
import torch

from conftest import build_oracle_h
from oracle import cv
from oracle import eigen
from oracle import qp as oqp
from oracle.grid import Grid
from paper_2601_21005_amd import sgw, systems

pytestmark = pytest.mark.gpu
U_BF16 = 2.0 ** -9


def bf16(a):
    """Round to BF16 (nearest even) through FP32, returned as float64."""
    u = np.ascontiguousarray(np.asarray(a, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def model_forward(theta, xh, din, h1, h2):
    W1, b1, W2, b2, w3, b3 = cv.unpack(theta, din, h1, h2)
    a1 = np.tanh(bf16(xh) @ bf16(W1).T + b1)
    a2 = np.tanh(bf16(a1) @ bf16(W2).T + b2)
    return a2 @ w3 + b3[0], a1, a2


def model_gradient(theta, xh, y, din, h1, h2):
    W1, b1, W2, b2, w3, b3 = cv.unpack(theta, din, h1, h2)
    g, a1, a2 = model_forward(theta, xh, din, h1, h2)
    n = xh.shape[0]
    dg = 2.0 * (g - y) / n
    d2 = np.outer(dg, w3) * (1 - a2 * a2)
    d1 = (bf16(d2) @ bf16(W2)) * (1 - a1 * a1)
    return np.concatenate([(bf16(d1).T @ bf16(xh)).ravel(), d1.sum(0),
                           (bf16(d2).T @ bf16(a1)).ravel(), d2.sum(0), a2.T @ dg, [dg.sum()]])


def f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def blocks(v, din, h1, h2):
    return [b.ravel() for b in cv.unpack(v, din, h1, h2)]


# ------------------------------------------------------------------ features
@pytest.mark.parametrize("which,K,first,nsamp", [("tiny8", 16, 0, 300), ("cfg1", 64, 1000, 70)])
def test_features_match_oracle(which, K, first, nsamp, request):
    """a = sqrt(dV) sum_r phi(r) s(r) with phi rounded to BF16 and FP32 sums:
    |a_gpu - a| <= sqrt(dV) sum|phi| (u + N 2^-24), x = a^2."""
    s, H = request.getfixturevalue(which)
    g = H.grid
    rs = np.random.default_rng(31)
    phi = rs.standard_normal((K, g.N))
    phi /= np.sqrt(g.dV * np.sum(phi * phi, axis=1))[:, None]
    phi = phi.astype(np.float32).astype(np.float64)
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, None, precision=sgw.SGW_C64, max_nvec=4)
    x = sgw.cv_features(ctx, f32(phi), seed=77, first_sample=first, nsamp=nsamp)
    got = x.cpu().numpy().astype(np.float64)
    ctx.close()
    ref = cv.features(g, phi, 77, range(first, first + nsamp))
    a = np.sqrt(ref)
    da = np.sqrt(g.dV) * np.sum(np.abs(phi), axis=1) * (U_BF16 + g.N * 2.0 ** -24)
    assert np.all(np.abs(got - ref) <= 2 * a * da[None] + da[None] ** 2)
    # the BF16 rounding model of the kernel: only FP32 summation differs
    model = g.dV * (bf16(phi) @ np.stack([cv.rng.white_noise_signs(
        77, cv.rng.stream_id(cv.rng.ZETA, i, 0), g.N) for i in range(first, first + nsamp)]).T).T ** 2
    assert np.max(np.abs(got - model)) < 1e-4 * np.max(model)


def test_features_160_grid_sampled():
    """The control-variate configuration's grid (160^3 points, h = 0.6 bohr)
    with its 64 states and a ragged last block of samples (600 = 2 x 256 + 88):
    sampled rows (block edges and the tail) against the oracle computed one
    sample at a time.  The states are random normalised stand-ins for the
    near-gap KS states (the kernel sees only their values).  Bounds: the
    rigorous one of test_features_match_oracle, and against the BF16 rounding
    model the FP32 accumulation over N = 4.1e6 points, whose rounding errors
    add like a random walk: 2^-24 sqrt(N) sum|phi| sqrt(dV) per amplitude, with
    a factor 16 of margin."""
    n, h, K, nsamp, first = 160, 0.6, 64, 600, 3000
    g = Grid(n, h=h)
    rs = np.random.default_rng(35)
    phi = rs.standard_normal((K, g.N)).astype(np.float32).astype(np.float64)
    phi /= np.sqrt(g.dV * np.sum(phi * phi, axis=1))[:, None]
    phi = phi.astype(np.float32).astype(np.float64)
    ctx = sgw.Context(n, h, np.zeros(g.N), None, precision=sgw.SGW_C64, max_nvec=2)
    x = sgw.cv_features(ctx, f32(phi), seed=91, first_sample=first, nsamp=nsamp)
    got = x.cpu().numpy().astype(np.float64)
    ctx.close()
    rows = [0, 1, 255, 256, 511, 512, 599]
    ref = cv.features(g, phi, 91, [first + i for i in rows])
    a = np.sqrt(ref)
    l1 = np.sqrt(g.dV) * np.sum(np.abs(phi), axis=1)
    da = l1 * (U_BF16 + g.N * 2.0 ** -24)
    assert np.all(np.abs(got[rows] - ref) <= 2 * a * da[None] + da[None] ** 2)
    signs = np.stack([cv.rng.white_noise_signs(91, cv.rng.stream_id(cv.rng.ZETA, first + i, 0),
                                               g.N) for i in rows])
    am = np.sqrt(g.dV) * (bf16(phi) @ signs.T).T
    e = 16 * 2.0 ** -24 * np.sqrt(g.N) * l1
    assert np.all(np.abs(got[rows] - am ** 2) <= 2 * np.abs(am) * e[None] + e[None] ** 2)
    assert np.all(np.isfinite(got)) and np.all(got >= 0)


def test_features_reject_bad_sizes(tiny8):
    s, _ = tiny8
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, None, precision=sgw.SGW_C64, max_nvec=4)
    phi = torch.zeros((65, s.grid.N), dtype=torch.float32, device="cuda")
    with pytest.raises(sgw.SgwError) as e:
        sgw.cv_features(ctx, phi, 1, 0, 4)
    assert e.value.code == sgw.SGW_EINVAL
    with pytest.raises(sgw.SgwError):
        sgw.cv_features(ctx, phi[:4], 1, (1 << 20) - 2, 4)
    ctx.close()


@pytest.mark.parametrize("which,K,first,nsamp,neta", [("tiny8", 16, 0, 120, 5),
                                                       ("cfg1", 32, 700, 40, 8)])
def test_features_eta_match_oracle(which, K, first, nsamp, neta, request):
    """Occupied-orbital noise features: the mean over l of a_l^2 with each
    a_l bounded as in the zeta-bar features (BF16 phi, FP32 sums), written
    into columns 7 .. 7 + K - 1 of wider rows; against the FP64 oracle and,
    tightly, the BF16 rounding model."""
    s, H = request.getfixturevalue(which)
    g = H.grid
    rs = np.random.default_rng(32)
    phi = rs.standard_normal((K, g.N))
    phi /= np.sqrt(g.dV * np.sum(phi * phi, axis=1))[:, None]
    phi = phi.astype(np.float32).astype(np.float64)
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, None, precision=sgw.SGW_C64, max_nvec=4)
    out = torch.full((nsamp, K + 9), -1.0, dtype=torch.float32, device="cuda")
    sgw.cv_features_eta(ctx, f32(phi), 78, first, nsamp, neta, out=out, col0=7)
    got_all = out.cpu().numpy().astype(np.float64)
    ctx.close()
    assert np.all(got_all[:, :7] == -1.0) and np.all(got_all[:, 7 + K:] == -1.0)
    got = got_all[:, 7:7 + K]
    ref = cv.features_eta(g, phi, 78, range(first, first + nsamp), neta)
    da = np.sqrt(g.dV) * np.sum(np.abs(phi), axis=1) * (U_BF16 + g.N * 2.0 ** -24)
    # |mean_l a_l^2 - mean_l b_l^2| <= mean_l (2 |b_l| da + da^2) <= 2 sqrt(mean b^2) da + da^2
    assert np.all(np.abs(got - ref) <= 2 * np.sqrt(ref) * da[None] + da[None] ** 2)
    signs = np.stack([[cv.rng.white_noise_signs(78, cv.rng.stream_id(cv.rng.ETA, i, l), g.N)
                       for l in range(neta)] for i in range(first, first + nsamp)])
    model = np.mean(g.dV * np.einsum("kn,iln->ilk", bf16(phi), signs) ** 2, axis=1)
    assert np.max(np.abs(got - model)) < 1e-4 * np.max(model)


# ------------------------------------------------------------------ network
@pytest.fixture(scope="module")
def net_case():
    rs = np.random.default_rng(32)
    din, h1, h2, n = 64, 256, 256, 700
    theta = systems.mlp_init(5, din, h1, h2)
    theta[din * h1:din * h1 + h1] = 0.1 * rs.standard_normal(h1)    # non-zero biases
    x = rs.gamma(1.0, 1.0, size=(n, din)).astype(np.float32).astype(np.float64)
    mean, std = cv.standardization(x)
    y = np.tanh(x[:, 0] - 1) + 0.3 * x[:, 1] + 0.1 * rs.standard_normal(n)
    y = y.astype(np.float32).astype(np.float64)
    xh = ((x.astype(np.float32) - mean.astype(np.float32))
          * (1.0 / std).astype(np.float32)).astype(np.float64)
    return dict(theta=theta.astype(np.float32).astype(np.float64), x=x, y=y, mean=mean,
                std=std, xh=xh, din=din, h1=h1, h2=h2)


def make_net(c):
    m = sgw.Mlp(c["theta"], c["din"], c["h1"], c["h2"])
    m.set_standardization(c["mean"], c["std"])
    return m


def test_forward_matches_oracle(net_case):
    c = net_case
    m = make_net(c)
    g = m.forward(f32(c["x"])).cpu().numpy().astype(np.float64)
    m.close()
    ref, _ = cv.forward(c["theta"], c["xh"])
    mod, _, _ = model_forward(c["theta"], c["xh"], 64, 256, 256)
    # BF16 operands: each layer's pre-activation carries ~2u relative noise
    assert np.linalg.norm(g - ref) < 8 * U_BF16 * np.linalg.norm(ref)
    assert np.max(np.abs(g - mod)) < 1e-4 * np.max(np.abs(ref))


def test_gradient_matches_oracle_backprop(net_case):
    """The device gradient against the FP64 chain rule (normwise 4e-2 per
    parameter block from BF16 operands) and against the rounding model
    (5e-4)."""
    c = net_case
    m = make_net(c)
    L, gr = m.gradient(f32(c["x"]), f32(c["y"]))
    m.close()
    Lo, go = cv.loss_and_gradient(c["theta"], c["xh"], c["y"])
    gm = model_gradient(c["theta"], c["xh"], c["y"], 64, 256, 256)
    assert abs(L - Lo) < 4 * U_BF16 * Lo
    for k, (a, b, mdl) in enumerate(zip(blocks(gr, 64, 256, 256), blocks(go, 64, 256, 256),
                                        blocks(gm, 64, 256, 256))):
        nb = np.linalg.norm(b)
        assert np.linalg.norm(a - b) < 4e-2 * nb, k
        assert np.linalg.norm(a - mdl) < 5e-4 * np.linalg.norm(mdl), k
    cos = gr @ go / (np.linalg.norm(gr) * np.linalg.norm(go))
    assert cos > 0.999


def test_adam_steps_match_oracle(net_case):
    """Given gradients (host FP64 inputs), three Adam steps in FP32 against
    the oracle's FP64 Adam: relative 1e-6 of the parameters' scale."""
    c = net_case
    m = make_net(c)
    rs = np.random.default_rng(33)
    opt = cv.Adam(c["theta"].size, lr=2e-3)
    th = c["theta"].copy()
    for _ in range(3):
        gvec = rs.standard_normal(th.size) * np.exp(rs.uniform(-8, 2, th.size))
        m.adam(gvec, lr=2e-3)
        th = opt.step(th, gvec.astype(np.float32).astype(np.float64))
    got = m.params()
    m.close()
    assert np.max(np.abs(got - th)) < 1e-6 * (1 + np.max(np.abs(th)))


def model_train(theta, xh, y, steps, din, h1, h2, lr=1e-3):
    """Full-batch Adam driven by the rounding model's gradient (BF16 GEMM
    operands, FP64 otherwise), parameters kept as FP32 masters like the
    device's; returns the loss before each step."""
    opt = cv.Adam(theta.size, lr=lr)
    hist = []
    W1, b1, W2, b2, w3, b3 = cv.unpack(theta, din, h1, h2)
    for _ in range(steps):
        g, _, _ = model_forward(theta, xh, din, h1, h2)
        hist.append(float(np.mean((g - y) ** 2)))
        theta = opt.step(theta, model_gradient(theta, xh, y, din, h1, h2))
        theta = theta.astype(np.float32).astype(np.float64)
    return np.array(hist)


def test_training_follows_oracle(net_case):
    """200 full-batch Adam steps on the device (BF16 products) against two
    host trajectories from the same start: the FP64 oracle, and the same
    Adam driven by the rounding model of the device's arithmetic (BF16 GEMM
    operands, FP32 parameters).  The first 20 losses agree with the oracle to
    5%.  Late in training the loss falls to the floor that BF16 operands
    leave, where the FP64 oracle keeps descending: the rounding model's own
    final loss differs from the oracle's by about x1.5, so the device is held
    to the rounding model (5% over the first 100 steps, x1.3 at the end) and
    to the oracle only within that model-to-oracle gap times 1.3.  Neither
    host trajectory descends monotonically (full-batch Adam overshoots near
    the floor), so no monotonicity is asserted; both must drop > 3x."""
    c = net_case
    m = make_net(c)
    hist = m.train(f32(c["x"]), f32(c["y"]), 200, lr=1e-3)
    m.close()
    _, ho = cv.train(c["theta"], c["xh"], c["y"], 200, lr=1e-3)
    hm = model_train(c["theta"], c["xh"], c["y"], 200, c["din"], c["h1"], c["h2"])
    assert abs(hist[0] - ho[0]) < 4 * U_BF16 * ho[0]
    assert np.max(np.abs(hist[:20] / ho[:20] - 1)) < 0.05
    assert np.max(np.abs(hist[:100] / hm[:100] - 1)) < 0.05
    assert abs(np.log(hist[-1] / hm[-1])) < np.log(1.3)
    assert abs(np.log(hist[-1] / ho[-1])) < abs(np.log(hm[-1] / ho[-1])) + np.log(1.3)
    assert hist[-1] < hist[0] / 3 and ho[-1] < ho[0] / 3


def test_cheap_moments_match_model(tiny8, net_case):
    """Mean and variance of g over 3000 cheap samples: device chunks of 512
    against the FP64 oracle (features and network)."""
    s, H = tiny8
    c = net_case
    g = H.grid
    rs = np.random.default_rng(34)
    phi = rs.standard_normal((64, g.N))
    phi /= np.sqrt(g.dV * np.sum(phi * phi, axis=1))[:, None]
    phi = phi.astype(np.float32).astype(np.float64)
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, None, precision=sgw.SGW_C64, max_nvec=4)
    m = sgw.Mlp(c["theta"])
    x = cv.features(g, phi, 9, range(5000, 8000))
    mean, std = cv.standardization(x)
    m.set_standardization(mean, std)
    mu, var = sgw.cv_cheap_moments(ctx, m, f32(phi), 9, 5000, 3000, chunk=512)
    m.close()
    ctx.close()
    go, _ = cv.forward(c["theta"], (x - mean) / std)
    assert abs(mu - go.mean()) < 0.02 * go.std()
    assert abs(var / go.var(ddof=1) - 1) < 0.05


def test_cheap_moments_mixed_match_model(tiny8):
    """Mean and variance of g over 3000 cheap samples whose input rows are
    [16 zeta-bar features, 48 eta-bar features (N_eta = 6)], device chunks of
    700, against the FP64 oracle."""
    s, H = tiny8
    g = H.grid
    th = systems.mlp_init(8)
    rs = np.random.default_rng(35)
    phi = rs.standard_normal((64, g.N))
    phi /= np.sqrt(g.dV * np.sum(phi * phi, axis=1))[:, None]
    phi = phi.astype(np.float32).astype(np.float64)
    pz, pe = phi[:16], phi[16:]
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, None, precision=sgw.SGW_C64, max_nvec=4)
    m = sgw.Mlp(th)
    x = np.hstack([cv.features(g, pz, 11, range(2000, 5000)),
                   cv.features_eta(g, pe, 11, range(2000, 5000), 6)])
    mean, std = cv.standardization(x)
    m.set_standardization(mean, std)
    mu, var = sgw.cv_cheap_moments_mixed(ctx, m, f32(pz), f32(pe), 11, 6, 2000, 3000, chunk=700)
    m.close()
    ctx.close()
    go, _ = cv.forward(th, (x - mean) / std)
    assert abs(mu - go.mean()) < 0.02 * go.std()
    assert abs(var / go.var(ddof=1) - 1) < 0.05


# ------------------------------------------------------------------ gain
def test_control_variate_gain_on_sgw_samples(tiny8, tiny8_eig):
    """Plain sGW on the 8^3 system (N_eta = 32, exact mode) gives per-sample
    y_i = X_i + Re Sigma_c,i(omega*) for 4096 samples.  A network on the
    sample's cheap projections -- |<phi_k|zeta-bar_i>|^2 and the mean over l
    of |<phi_k|eta-bar_{i,l}>|^2 over the 32 lowest states -- is trained on
    1536 of them (early-stopped on 512 more), c is fitted on 1024 others (A)
    and the estimate taken on the last 1024 (B) with 50000 cheap samples for
    E[g].  The variance ratio on B (measured 0.24) plus three of its
    jackknife standard errors over the B samples stays below 0.6 (linear fits
    of the same features on the oracle's samples explain 80 % of the
    variance, so a working estimator reaches about 0.2 up to training noise),
    and the estimate agrees with the plain mean (no fallback)."""
    s, H = tiny8
    e, V = tiny8_eig
    ho = s.n_occ - 1
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=sgw.SGW_C64,
                      max_nvec=256)
    lo, hi = ctx.bounds()
    mu = 0.5 * (e[ho] + e[ho + 1])
    p = dict(seed=41, n_eta=32, n_tau=30, dt=0.1, m_sub=2, mu=mu, beta=10.0, ncoef=600,
             emin=lo, emax=hi, n_xi=64, f_g=0.125, mode=1)
    n = 4096
    sig, xs = [], []
    for b in range(0, n, 64):
        si, xi, _ = ctx.sigma_estimate(V[ho], n_zeta=64, first_sample=b, **p)
        sig.append(si)
        xs.append(xi)
    sig, xs = np.concatenate(sig), np.concatenate(xs)
    gam = oqp.default_gamma(p["n_tau"], p["dt"])
    eqp = sgw.sgw_qp_solve(sig.mean(0), p["dt"], gam, e[ho], xs.mean())[0]
    y = xs + np.array([sgw.sgw_sigma_omega(si, p["dt"], gam, eqp)[0].real for si in sig])
    Vn = V[:32] / np.sqrt(H.grid.dV * np.sum(V[:32] ** 2, axis=1))[:, None]
    phi = f32(Vn)
    x = torch.empty((n, 64), dtype=torch.float32, device="cuda")
    x[:, :32] = sgw.cv_features(ctx, phi, p["seed"], 0, n)
    sgw.cv_features_eta(ctx, phi, p["seed"], 0, n, p["n_eta"], out=x, col0=32)
    xn = x.cpu().numpy().astype(np.float64)
    tr, va, A, B = slice(0, 1536), slice(1536, 2048), slice(2048, 3072), slice(3072, 4096)
    mean, std = cv.standardization(xn[tr])
    ym, ysd = y[tr].mean(), y[tr].std()
    yt = f32((y - ym) / ysd)
    m = sgw.Mlp(systems.mlp_init(3))
    m.set_standardization(mean, std)
    best, best_loss = None, np.inf
    for it in range(30):                          # early stopping on the validation set
        m.train(x[tr].contiguous(), yt[tr].contiguous(), 10, lr=1e-3)
        gv = m.forward(x[va].contiguous()).cpu().numpy().astype(np.float64)
        loss = np.mean((gv - (y[va] - ym) / ysd) ** 2)
        if loss < best_loss:
            best, best_loss = m.params(), loss
    m.close()
    m = sgw.Mlp(best)
    m.set_standardization(mean, std)
    g = m.forward(x).cpu().numpy().astype(np.float64)
    gm, gvar = sgw.cv_cheap_moments_mixed(ctx, m, phi, phi, p["seed"], p["n_eta"], 10000, 50000,
                                          chunk=8192)
    m.close()
    ctx.close()
    r = sgw.sgw_cv_estimate(y[A], g[A], y[B], g[B], gm, gvar, 50000)
    plain_B = y[B].std(ddof=1) / np.sqrt(1024)
    ratio = (r["sigma_cv"] / plain_B) ** 2
    se = variance_ratio_jackknife_se(y[B], g[B], r["c"], r["c"] ** 2 * gvar / 50000)
    print(f"\ncontrol variate: rho2(A) {r['rho2']:.3f}  variance ratio {ratio:.3f} "
          f"+- {se:.3f}  cv {r['estimate']:.5f} +- {r['sigma_cv']:.5f}  "
          f"plain {r['plain']:.5f}  fallback {r['fallback']}", flush=True)
    assert not r["fallback"]
    assert ratio + 3.0 * se < 0.6


def variance_ratio_jackknife_se(y, g, c, var_mean_term):
    """Jackknife standard error, over the evaluation samples, of the variance
    ratio (Var(y - c g)/n + var_mean_term) / (Var(y)/n) with c fixed (it is
    fitted on another set)."""
    n = y.size
    r = y - c * g

    def ratio(yy, rr):
        m = yy.size
        return (np.var(rr, ddof=1) / m + var_mean_term) / (np.var(yy, ddof=1) / m)

    loo = np.array([ratio(np.delete(y, i), np.delete(r, i)) for i in range(n)])
    return float(np.sqrt((n - 1) / n * np.sum((loo - loo.mean()) ** 2)))
