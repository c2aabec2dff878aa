"""sgw_apply_H_noalloc (the H application for callers that cannot allocate)
against sgw_apply_H through the C ABI: two calls in a row on one context,
the second with fewer vectors, in complex FP32 with projectors (one call
large enough to take two chunks of the static scratch, one with a leading
dimension above N), complex FP64 with projectors and local-only H.  Both
entry points run the same kernels in the same order, so the results agree
bit for bit; the parity bar of H psi (3e-6 normwise in complex FP32, 1e-12
in complex FP64) is asserted as well."""
import numpy as np
import pytest
import torch

from conftest import make_ctx, norm_err
from paper_2601_21005_amd import sgw, systems

pytestmark = pytest.mark.gpu
TOL = {sgw.SGW_C128: 1e-12, sgw.SGW_C64: 3e-6}


def batch(ctx, nvec, ld, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    re = torch.randn((nvec, ld), generator=g, dtype=torch.float64)
    im = torch.randn((nvec, ld), generator=g, dtype=torch.float64)
    return torch.complex(re, im).to(ctx.cdtype).cuda()


def check_pair(ctx, nvec, ld, seed, prec):
    x = batch(ctx, nvec, ld, seed)
    ref = torch.zeros_like(x)
    got = torch.full_like(x, float("nan"))      # the FFT intermediate lives here
    print(f"no-alloc: prec={prec} nvec={nvec} ld={ld} N={ctx.N}", flush=True)
    ctx.apply_H(x, ref)
    ctx.apply_H_noalloc(x, got)
    torch.cuda.synchronize()
    N = ctx.N
    r = ref[:, :N].cpu().numpy()
    o = got[:, :N].cpu().numpy()
    assert np.all(np.isfinite(o))
    assert norm_err(o, r) < TOL[prec]
    assert np.array_equal(o, r)


@pytest.mark.parametrize("prec", [sgw.SGW_C64, sgw.SGW_C128])
def test_noalloc_matches_apply_h_with_projectors(prec):
    s = systems.si35h36() if prec == sgw.SGW_C64 else systems.tiny_system(16, 0.7)
    ctx = make_ctx(s, prec, max_nvec=64)
    big = 700 if prec == sgw.SGW_C64 else 40     # 700: two chunks of the 64 MiB scratch
    check_pair(ctx, big, ctx.N, 11, prec)
    check_pair(ctx, 5, ctx.N + 64, 12, prec)     # second call: fewer vectors, ld > N
    ctx.close()


def test_noalloc_local_only_and_errors():
    s = systems.tiny_system(12, 0.5, with_kb=False)
    ctx = make_ctx(s, sgw.SGW_C64, max_nvec=8)
    check_pair(ctx, 9, ctx.N, 13, sgw.SGW_C64)
    check_pair(ctx, 2, ctx.N, 14, sgw.SGW_C64)
    x = batch(ctx, 2, ctx.N, 15)
    with pytest.raises(sgw.SgwError) as e:
        ctx.apply_H_noalloc(x, x)                # overlapping input and output
    assert e.value.code == sgw.SGW_EINVAL
    ctx.close()
