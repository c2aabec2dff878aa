"""GPU parity: the linear-response TDH Strang step (Sec. 2.1 first phase)."""
import numpy as np
import pytest
import torch

from conftest import make_ctx, norm_err, rel_err, row_max_err
from oracle.tdh import TDH
from paper_2601_21005_amd import sgw

pytestmark = pytest.mark.gpu


def run(system, H, prec, S, neta, nsub, tau, seed=0):
    ctx = make_ctx(system, prec)
    N = system.grid.N
    rs = np.random.default_rng(seed)
    eta = 0.3 * rs.standard_normal((S, neta, N))
    dv = 0.5 * np.sin(np.linspace(0, 7, N))[None, :] * (1 + rs.standard_normal((S, 1)))
    psi = torch.zeros((S, 2, neta, N), dtype=ctx.cdtype, device="cuda")
    psi[:, 0] = torch.from_numpy(eta).to(ctx.cdtype)
    v, u, vh0 = ctx.fields(S), ctx.fields(S), ctx.fields(S)
    dvd = torch.from_numpy(dv).to(ctx.rdtype).cuda()
    w = 2.0 / neta
    st = ctx.tdh_state(psi, v, u, vh0, S, neta, w)
    ctx.tdh_init(st, dvd)
    ctx.tdh_step(st, nsub, tau)
    torch.cuda.synchronize()
    dv_in = dvd.cpu().numpy().astype(np.float64)
    out = []
    for s in range(S):
        o = TDH(H, tau, w)
        e0 = torch.from_numpy(eta[s]).to(ctx.cdtype).numpy().astype(np.complex128)
        st_o = o.start(e0, dv_in[s])
        for _ in range(nsub):
            st_o = o.substep(*st_o)
        out.append(st_o)
    got = psi.cpu().numpy().astype(np.complex128)
    res = dict(eta=(got[:, 0], np.array([o[0] for o in out])),
               deta=(got[:, 1], np.array([o[1] for o in out])),
               v=(v.cpu().numpy(), np.array([o[2] for o in out])),
               u=(u.cpu().numpy(), np.array([o[3] for o in out])))
    ctx.close()
    return res


@pytest.mark.parametrize("prec,tol", [(sgw.SGW_C128, 1e-11), (sgw.SGW_C64, 1e-5)])
def test_tdh_tiny8_kb(tiny8, prec, tol):
    s, H = tiny8
    r = run(s, H, prec, S=2, neta=4, nsub=6, tau=0.05)
    for k in ("eta", "deta"):
        assert norm_err(r[k][0].reshape(-1, s.grid.N), r[k][1].reshape(-1, s.grid.N)) < tol, k
        assert row_max_err(r[k][0].reshape(-1, s.grid.N), r[k][1].reshape(-1, s.grid.N)) < 10 * tol, k
    assert rel_err(r["u"][0], r["u"][1]) < 10 * tol
    assert rel_err(r["v"][0], r["v"][1]) < 10 * tol


@pytest.mark.parametrize("prec,tol", [(sgw.SGW_C128, 1e-11), (sgw.SGW_C64, 2e-5)])
def test_tdh_gaussian_wells(cfg1, prec, tol):
    s, H = cfg1
    r = run(s, H, prec, S=3, neta=8, nsub=8, tau=0.05, seed=1)
    for k in ("eta", "deta"):
        assert norm_err(r[k][0].reshape(-1, s.grid.N), r[k][1].reshape(-1, s.grid.N)) < tol, k
        assert row_max_err(r[k][0].reshape(-1, s.grid.N), r[k][1].reshape(-1, s.grid.N)) < 10 * tol, k
    assert rel_err(r["u"][0], r["u"][1]) < 20 * tol


def test_tdh_si35h36_fp32_per_step(si35):
    """One substep on the 64^3 cluster in complex FP32: 1e-6 relative."""
    s, H = si35
    r = run(s, H, sgw.SGW_C64, S=1, neta=8, nsub=1, tau=0.05, seed=2)
    for k in ("eta", "deta"):
        assert norm_err(r[k][0].reshape(-1, s.grid.N), r[k][1].reshape(-1, s.grid.N)) < 1e-6, k
        assert row_max_err(r[k][0].reshape(-1, s.grid.N), r[k][1].reshape(-1, s.grid.N)) < 10 * 1e-6, k
