"""GPU parity: H|psi> through the C ABI against the FP64 oracle (Eq. 1)."""
import numpy as np
import pytest
import torch

from conftest import make_ctx, norm_err, rel_err, row_max_err
from paper_2601_21005_amd import sgw

pytestmark = pytest.mark.gpu

# FP32 paths: inputs are exact FP32 values on both sides, so the error is the
# kernels' own rounding: ~log2(N_g) FFT stages of unit roundoff 6e-8 in each
# direction plus the potential and projector terms -> 3e-6 normwise (the
# largest entries of H psi come from T(k) up to 60 Ha).
TOL = {sgw.SGW_C128: 1e-12, sgw.SGW_C64: 3e-6}


def run_hpsi(system, H, prec, nvec=5, pad=0, seed=0):
    ctx = make_ctx(system, prec, max_nvec=4)        # forces chunking (5 > 4)
    N = system.grid.N
    rs = np.random.default_rng(seed)
    x = rs.standard_normal((nvec, N)) + 1j * rs.standard_normal((nvec, N))
    dt = ctx.cdtype
    xin = torch.zeros((nvec, N + pad), dtype=dt, device="cuda")
    xin[:, :N] = torch.from_numpy(x).to(dt)
    out = torch.zeros_like(xin)
    ctx.apply_H(xin, out)
    torch.cuda.synchronize()
    xin_h = xin[:, :N].cpu().numpy().astype(np.complex128)
    ref = H.apply(xin_h)
    got = out[:, :N].cpu().numpy().astype(np.complex128)
    if pad:
        assert torch.all(out[:, N:] == 0)
    ctx.close()
    return got, ref


@pytest.mark.parametrize("prec", [sgw.SGW_C128, sgw.SGW_C64])
def test_hpsi_tiny_with_kb(tiny8, prec):
    s, H = tiny8
    got, ref = run_hpsi(s, H, prec)
    assert norm_err(got, ref) < TOL[prec]
    assert row_max_err(got, ref) < 10 * TOL[prec]


@pytest.mark.parametrize("prec", [sgw.SGW_C128, sgw.SGW_C64])
def test_hpsi_tiny12_padded_ld(tiny12l, prec):
    s, H = tiny12l
    got, ref = run_hpsi(s, H, prec, nvec=3, pad=40)
    assert norm_err(got, ref) < TOL[prec]
    assert row_max_err(got, ref) < 10 * TOL[prec]


@pytest.mark.parametrize("prec", [sgw.SGW_C128, sgw.SGW_C64])
def test_hpsi_gaussian_wells_32(cfg1, prec):
    s, H = cfg1
    got, ref = run_hpsi(s, H, prec, nvec=7)
    assert norm_err(got, ref) < TOL[prec]
    assert row_max_err(got, ref) < 10 * TOL[prec]


def test_hpsi_gaussian_wells_160():
    """The control-variate configuration's grid, 160^3 at h = 0.6 bohr (x
    lines and pencils with radix 8, 5 and 4 stages; the planes do not fit in
    LDS): local H psi on two vectors against the oracle."""
    from conftest import build_oracle_h
    from paper_2601_21005_amd import systems
    s = systems.gaussian_wells(seed=1011, n=160, h=0.6, nwell=24)
    H = build_oracle_h(s, workers=8)
    for prec in (sgw.SGW_C128, sgw.SGW_C64):
        got, ref = run_hpsi(s, H, prec, nvec=2)
        assert norm_err(got, ref) < TOL[prec], prec
        assert row_max_err(got, ref) < 10 * TOL[prec], prec


@pytest.mark.parametrize("prec", [sgw.SGW_C128, sgw.SGW_C64])
def test_hpsi_si35h36_64(si35, prec):
    # C128 at 64^3 runs the x-line / y-pencil fallback (plane too big for LDS)
    s, H = si35
    got, ref = run_hpsi(s, H, prec, nvec=9)
    assert norm_err(got, ref) < TOL[prec]
    assert row_max_err(got, ref) < 10 * TOL[prec]
    assert rel_err(got, ref) < 10 * TOL[prec]


def test_hpsi_errors_and_empty(tiny8):
    s, H = tiny8
    ctx = make_ctx(s, sgw.SGW_C128)
    x = torch.zeros((2, s.grid.N), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    ctx.apply_H(x[:0], y[:0])                         # nvec = 0: no-op
    with pytest.raises(sgw.SgwError) as e:          # ld < N
        sgw._check(sgw.load().sgw_apply_H(ctx.ctx, x.data_ptr(), y.data_ptr(), 2,
                                          s.grid.N - 1), ctx.ctx)
    assert e.value.code == sgw.SGW_EINVAL
    with pytest.raises(sgw.SgwError) as e:          # in place is refused
        sgw._check(sgw.load().sgw_apply_H(ctx.ctx, x.data_ptr(), x.data_ptr(), 2, s.grid.N),
                   ctx.ctx)
    assert e.value.code == sgw.SGW_EINVAL
    ctx.close()


def test_create_rejects_bad_input(tiny8):
    s, _ = tiny8
    v = s.v_loc.copy()
    v[3] = np.nan
    with pytest.raises(sgw.SgwError) as e:
        sgw.Context(8, 0.7, v, None, precision=sgw.SGW_C128)
    assert e.value.code == sgw.SGW_EINVAL
    with pytest.raises(sgw.SgwError) as e:
        sgw.Context(10, 0.7, np.zeros(1000), None, precision=sgw.SGW_C128)
    assert e.value.code == sgw.SGW_EUNSUPPORTED


def test_bounds_match_oracle(si35, tiny8):
    for s, H in (si35, tiny8):
        ctx = make_ctx(s, sgw.SGW_C64)
        a, b = ctx.bounds(0.01)
        ea, eb = H.bounds(0.01)
        assert abs(a - ea) < 1e-10 * abs(ea) and abs(b - eb) < 1e-10 * abs(eb)
        ctx.close()


@pytest.mark.parametrize("prec,names", [(sgw.SGW_C64, ("kb_gather", "kb_scatter")),
                                         (sgw.SGW_C64_BF16KB, ("kb_gather_bf16", "kb_scatter_bf16")),
                                         (sgw.SGW_C64_BF16X2KB,
                                          ("kb_gather_bf16x2", "kb_scatter_bf16x2"))])
def test_kb_variants_bit_identical(si35, monkeypatch, prec, names):
    """Every autotuned KB kernel variant adds the same products in the same
    order: H psi is bitwise the same whichever variant runs, on a batch of 20
    vectors and on one of 100 (six full blocks of 16 and a ragged one)."""
    s, H = si35
    rs = np.random.default_rng(9)
    x = rs.standard_normal((100, s.grid.N)) + 1j * rs.standard_normal((100, s.grid.N))
    xd = torch.from_numpy(x).to(torch.complex64).cuda()
    ref = {}
    for g, sc in [(g, 0) for g in range(4)] + [(0, sc) for sc in range(1, 9)]:
        monkeypatch.setenv("SGW_FORCE_VARIANT", f"{names[0]}={g},{names[1]}={sc}")
        ctx = make_ctx(s, prec, max_nvec=128)
        for nv in (20, 100):
            yd = torch.empty_like(xd[:nv])
            ctx.apply_H(xd[:nv], yd)
            out = yd.cpu().numpy()
            if nv not in ref:
                ref[nv] = out
            else:
                assert np.array_equal(out, ref[nv]), (g, sc, nv)
        ctx.close()
    assert np.array_equal(ref[20], ref[100][:20])


@pytest.mark.parametrize("prec", [sgw.SGW_C64, sgw.SGW_C64_BF16KB, sgw.SGW_C64_BF16X2KB])
def test_kb_support_masks_change_no_value(si35, monkeypatch, prec):
    """The KB kernels skip the 16-point rows (gather: K groups) that no
    projector reaches; the products skipped are exact zeros, so H psi equals
    the one with every row live (SGW_KB_MASK=0) -- on the 64^3 cluster (16 x
    8 x 4 tiles) and on a 17-Si cluster at 40^3 (8 x 8 x 8 tiles)."""
    from paper_2601_21005_amd import systems
    species, pos = systems.si_cluster(17, seed=3)
    s40 = systems.cluster_model(species, pos, n=40, h=0.6, ecut=28.0)
    for s in (si35[0], s40):
        rs = np.random.default_rng(12)
        x = rs.standard_normal((36, s.grid.N)) + 1j * rs.standard_normal((36, s.grid.N))
        xd = torch.from_numpy(x).to(torch.complex64).cuda()
        out = {}
        for m in ("1", "0"):
            monkeypatch.setenv("SGW_KB_MASK", m)
            ctx = make_ctx(s, prec, max_nvec=64)
            st = ctx.kb_stats()
            yd = torch.empty_like(xd)
            ctx.apply_H(xd, yd)
            out[m] = yd.cpu().numpy()
            ctx.close()
        print(f"{s.grid.n}^3: support points {st['support_points']} of {st['tile_points']} "
              "tile points", flush=True)
        assert st["support_points"] < st["tile_points"]
        assert np.array_equal(out["1"], out["0"])


def test_lanczos_bounds_match_oracle(tiny8, tiny8_eig):
    """40 Lanczos steps from the same start vector on the device (C128) and
    in the oracle give the same interval, and it encloses the spectrum."""
    from oracle import eigen
    s, H = tiny8
    e, _ = tiny8_eig
    ctx = make_ctx(s, sgw.SGW_C128)
    lo, hi = ctx.lanczos_bounds(40, seed=3, pad=0.01)
    ctx.close()
    lo_o, hi_o = eigen.lanczos_bounds(H, 40, seed=3, pad=0.01)
    w = e[-1] - e[0]
    assert abs(lo - lo_o) < 1e-6 * w and abs(hi - hi_o) < 1e-6 * w
    assert lo <= e[0] and hi >= e[-1]


def test_lanczos_bounds_si35h36_fp32(si35):
    """On the 64^3 cluster in complex FP32 the Lanczos interval encloses the
    extreme eigenvalues that the oracle's ARPACK eigensolvers give
    (tests/golden/si35h36_64_extremes.json, written by
    make_si35h36_extremes.py) and is at least 10% narrower than the rigorous
    one."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "si35h36_64_extremes.json")) as f:
        ext = json.load(f)
    s, H = si35
    ctx = make_ctx(s, sgw.SGW_C64)
    lo, hi = ctx.lanczos_bounds(60, seed=1, pad=0.01)
    lw, hw = ctx.bounds(0.0)
    ctx.close()
    # a Ritz value lies inside the spectrum: the true lowest eigenvalue is at
    # most 1e-10 relative below the stored one, the true highest at most 1e-6
    # relative above it, and never above the rigorous bound hw
    assert lo <= ext["e_min"] - 1e-8
    assert hi >= min(ext["e_max"] + 3e-5, hw)
    assert lw <= lo and hi <= hw
    assert hi - lo < 0.9 * (hw - lw)


def test_kernel_timers(tiny8, monkeypatch):
    """The launch timers of the Chebyshev plane pass and the KB scatter and
    gather count one launch of each per filter term and the points they cover
    (the 8^3 grid is one 512-point tile, which the projectors touch); the
    projector layout sizes match that tile.  The gathers are timed on the
    context's own stream: with SGW_KB_OVERLAP=0 the filter issues them there
    (by default they run on the second stream, untimed, beside the FFT
    passes)."""
    s, _ = tiny8
    monkeypatch.setenv("SGW_KB_OVERLAP", "0")
    ctx = make_ctx(s, sgw.SGW_C64, max_nvec=32)
    N, nvec = s.grid.N, 5
    g = torch.Generator(device="cuda").manual_seed(3)
    x = torch.randn((nvec, N), generator=g, device="cuda", dtype=torch.complex64)
    lo, hi = ctx.bounds()
    coef = sgw.sgw_fermi_coefficients(-0.5, 6.0, lo, hi, 40)
    ctx.kernel_timer(sgw.SGW_TIMER_CHEB_PLANE | sgw.SGW_TIMER_KB_SCATTER |
                     sgw.SGW_TIMER_KB_GATHER)
    ctx.fermi_filter(x, coef, lo, hi)
    ctx.kernel_timer(0)
    ms, n, pts = ctx.kernel_timer_read(sgw.SGW_TIMER_CHEB_PLANE)
    assert n == 39 and pts == 39 * nvec * N and ms > 0
    ms, n, pts = ctx.kernel_timer_read(sgw.SGW_TIMER_KB_SCATTER)
    assert n == 39 and pts == 39 * nvec * 512 and ms > 0
    assert ctx.kernel_timer_read(sgw.SGW_TIMER_KB_SCATTER)[:2] == (0.0, 0)   # read resets
    ms, n, pts = ctx.kernel_timer_read(sgw.SGW_TIMER_KB_GATHER)
    assert n == 39 and pts == 39 * nvec * 512 and ms > 0
    # the oracle's projector matrix gives the support and the nonzero count
    B = tiny8[1].kb.B.copy()
    B.eliminate_zeros()
    st = ctx.kb_stats()
    assert st["tiles"] == 1 and st["tile_points"] == 512 and st["entries"] == 2
    assert st["support_points"] == np.unique(B.tocoo().row).size and st["nnz"] == B.nnz
    for bad in (8, -1):
        with pytest.raises(sgw.SgwError) as e:
            ctx.kernel_timer(bad)
        assert e.value.code == sgw.SGW_EINVAL
    with pytest.raises(sgw.SgwError) as e:
        ctx.kernel_timer_read(3)
    assert e.value.code == sgw.SGW_EINVAL
    ctx.close()
