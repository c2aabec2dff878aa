"""Batching: HIP-graph replay of the repeated launch sequences gives bitwise
the results of eager launches (filter of odd and even length, the zeta
propagator, the TDH output steps), and concurrent uneven clusters give each
cluster's own results."""
import numpy as np
import pytest
import torch

from conftest import make_ctx
from paper_2601_21005_amd import sgw

pytestmark = pytest.mark.gpu


def ctx_on_stream(system, prec, stream, max_nvec=64):
    return sgw.Context(system.grid.n, system.grid.h, system.v_loc, system.projectors,
                       precision=prec, ecut=system.ecut, max_nvec=max_nvec,
                       stream=stream.cuda_stream)


@pytest.mark.parametrize("ncoef", [70, 71, 200])
def test_filter_graph_bitwise(tiny8, ncoef):
    s, _ = tiny8
    st = torch.cuda.Stream()
    rs = np.random.default_rng(60)
    x = rs.standard_normal((5, s.grid.N)) + 1j * rs.standard_normal((5, s.grid.N))
    out = []
    for graphs in (False, True):
        ctx = ctx_on_stream(s, sgw.SGW_C64, st)
        lo, hi = ctx.bounds()
        coef = sgw.sgw_fermi_coefficients(-0.5, 6.0, lo, hi, ncoef)
        if graphs:
            ctx.use_graphs(True)
        res = []
        for rep in range(3):                 # first call eager, then replays
            with torch.cuda.stream(st):
                xd = torch.from_numpy(x).to(torch.complex64).cuda()
            st.synchronize()
            ctx.fermi_filter(xd, coef, lo, hi)
            st.synchronize()
            res.append(xd.cpu().numpy())
        ctx.close()
        for r in res[1:]:
            assert np.array_equal(r, res[0])
        out.append(res[0])
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("mode", [0, 1])
def test_sigma_graph_bitwise(tiny8, tiny8_eig, mode):
    s, _ = tiny8
    e, V = tiny8_eig
    st = torch.cuda.Stream()
    lo_hi = None
    res = []
    for graphs in (False, True):
        ctx = ctx_on_stream(s, sgw.SGW_C64, st, max_nvec=16)
        lo, hi = ctx.bounds()
        if graphs:
            ctx.use_graphs(True)
        p = dict(seed=61, n_eta=4, n_tau=9, dt=0.1, m_sub=2, mu=0.5 * (e[1] + e[2]),
                 beta=10.0, ncoef=151, emin=lo, emax=hi, n_xi=64, f_g=0.125, mode=mode)
        a = ctx.sigma_estimate(V[s.n_occ - 1], n_zeta=3, first_sample=0, **p)
        b = ctx.sigma_estimate(V[s.n_occ - 1], n_zeta=3, first_sample=0, **p)
        ctx.close()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        res.append(a)
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


def test_graphs_need_a_stream(tiny8):
    s, _ = tiny8
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=sgw.SGW_C64,
                      stream=0)
    with pytest.raises(sgw.SgwError) as e:
        ctx.use_graphs(True)
    assert e.value.code == sgw.SGW_EINVAL
    ctx.close()


def test_uneven_batch_matches_sequential(tiny8, tiny12l, cfg1):
    """Three clusters of different grids (8^3 with KB, 12^3 local, 32^3
    local) and sizes on three streams through the batch call: each result is
    bitwise the one from its own sequential call."""
    cases = []
    for (s, H), neta, nz in ((tiny8, 4, 3), (tiny12l, 8, 2), (cfg1, 4, 2)):
        st = torch.cuda.Stream()
        ctx = ctx_on_stream(s, sgw.SGW_C64, st, max_nvec=16)
        lo, hi = ctx.bounds()
        rs = np.random.default_rng(s.grid.N)
        phi = rs.standard_normal(s.grid.N)
        phi /= np.sqrt(s.grid.h ** 3 * np.sum(phi * phi))
        kw = dict(seed=62, n_zeta=nz, n_eta=neta, n_tau=5, dt=0.1, m_sub=1, mu=-1.0,
                  beta=4.0, ncoef=90, emin=lo, emax=hi, n_xi=32, f_g=0.25, mode=0)
        cases.append((ctx, phi, kw))
    seq = [c[0].sigma_estimate(c[1], **c[2]) for c in cases]
    bat = sgw.batch_sigma_estimate(cases, nworkers=3)
    for (s1, x1, _), (s2, x2, ms) in zip(seq, bat):
        assert np.array_equal(s1, s2) and np.array_equal(x1, x2)
        assert ms > 0
    for c in cases:
        c[0].close()


def test_batch_rejects_a_shared_context(tiny8):
    s, _ = tiny8
    ctx = make_ctx(s, sgw.SGW_C64)
    lo, hi = ctx.bounds()
    kw = dict(seed=1, n_zeta=1, n_eta=2, n_tau=2, dt=0.1, m_sub=1, mu=-1.0, beta=4.0,
              ncoef=10, emin=lo, emax=hi, n_xi=8, f_g=0.25, mode=0)
    phi = np.ones(s.grid.N)
    with pytest.raises(sgw.SgwError):
        sgw.batch_sigma_estimate([(ctx, phi, kw), (ctx, phi, kw)])
    ctx.close()


def test_tune_cache_file(tmp_path):
    """With SGW_TUNE_CACHE set, a fresh process writes its KB kernel choices
    (keyed by arch, kernel, grid, precision and batch width) to the file, and
    a second process reads them back and gives the same result."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = tmp_path / "tune.json"
    code = ("import sys, numpy as np, torch; sys.path.insert(0, %r)\n"
            "from paper_2601_21005_amd import sgw, systems\n"
            "s = systems.tiny_system(8, 0.7)\n"
            "ctx = sgw.Context(8, 0.7, s.v_loc, s.projectors, precision=sgw.SGW_C64)\n"
            "x = torch.ones((24, 512), dtype=torch.complex64, device='cuda')\n"
            "y = torch.empty_like(x); ctx.apply_H(x, y)\n"
            "np.save(sys.argv[1], y.cpu().numpy())\n" % root)
    env = dict(os.environ, SGW_TUNE_CACHE=str(path))
    outs = []
    for k in range(2):
        out = tmp_path / f"y{k}.npy"
        subprocess.run([sys.executable, "-c", code, str(out)], env=env, check=True, timeout=300)
        outs.append(np.load(out))
        entries = json.loads(path.read_text())
        keys = [k for k in entries if "/kb_gather/8x8x8/p1/24" in k or "/kb_scatter/8x8x8/p1/24" in k]
        assert len(keys) == 2, entries
        assert all(k.startswith("gfx") for k in keys)
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("graphs", [False, True])
def test_zeta_overlap_bitwise(tiny8, tiny8_eig, monkeypatch, graphs):
    """The zeta propagation on the context's second stream, beside the TDH
    steps, gives bitwise the results of running it after them (two states,
    so the stored overlaps of every state and step are used)."""
    s, _ = tiny8
    e, V = tiny8_eig
    phis = np.stack([V[s.n_occ - 1], V[s.n_occ]])
    st = torch.cuda.Stream()
    res = []
    for ov in ("1", "0"):
        monkeypatch.setenv("SGW_ZETA_OVERLAP", ov)
        ctx = ctx_on_stream(s, sgw.SGW_C64, st, max_nvec=16)
        lo, hi = ctx.bounds()
        if graphs:
            ctx.use_graphs(True)
        p = dict(seed=63, n_eta=4, n_tau=11, dt=0.1, m_sub=2, mu=0.5 * (e[1] + e[2]),
                 beta=10.0, ncoef=151, emin=lo, emax=hi, n_xi=64, f_g=0.125, mode=0)
        a = ctx.sigma_estimate_states(phis, n_zeta=3, **p)
        b = ctx.sigma_estimate_states(phis, n_zeta=3, **p)
        ctx.close()
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        res.append(a)
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
