"""Short driver for hardware-counter profiles of the dominant kernel.

Runs, on the bench's Si35H36-shaped 64^3 workload in complex FP32:
  1. a plain device copy of known size (torch elementwise copy of 256 MiB),
     the reference that scales FETCH_SIZE / WRITE_SIZE to bytes;
  2. sgw_fermi_filter on the bench's launch shape (260 complex vectors =
     8 samples x 65 real orbitals) for a few terms, whose inverse plane pass
     carries the Chebyshev epilogue;
  3. with --hpsi-nvec M > 0, H applications on M vectors (the TDH's launch
     shape for the projector kernels is 1024).
Meant to run under ``rocprofv3 --pmc FETCH_SIZE`` (then WRITE_SIZE) or
``--kernel-trace --stats``.
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nvec", type=int, default=260)
    ap.add_argument("--terms", type=int, default=8)
    ap.add_argument("--hpsi-nvec", type=int, default=0)
    args = ap.parse_args()
    import numpy as np
    import torch

    from paper_2601_21005_amd import sgw, systems
    torch.cuda.set_device(0)
    # 1. reference copy: 256 MiB read + 256 MiB written
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"copy bytes read {a.numel() * 4} written {b.numel() * 4}", flush=True)
    # 2. filter terms at the bench's launch shape
    s = systems.si35h36()
    ctx = sgw.Context(s.grid.n, s.grid.h, s.v_loc, s.projectors, precision=sgw.SGW_C64,
                      ecut=s.ecut, max_nvec=max(args.nvec, args.hpsi_nvec))
    lo, hi = ctx.bounds(0.01)
    coef = sgw.sgw_fermi_coefficients(-4.65, 66.0, lo, hi, args.terms)
    x = torch.randn((args.nvec, s.grid.N), dtype=torch.complex64, device="cuda")
    x /= float(np.sqrt(s.grid.N))
    ctx.fermi_filter(x, coef, lo, hi)
    torch.cuda.synchronize()
    print(f"filter nvec {args.nvec} terms {args.terms} N {s.grid.N}: "
          f"{args.terms - 1} launches of the inverse Chebyshev plane pass, "
          f"40 B x {args.nvec * s.grid.N} pt*vec algorithmic each", flush=True)
    if args.hpsi_nvec > 0:
        del x
        y = torch.randn((args.hpsi_nvec, s.grid.N), dtype=torch.complex64, device="cuda")
        hy = torch.empty_like(y)
        for _ in range(3):
            ctx.apply_H(y, hy)
        torch.cuda.synchronize()
        print(f"H psi nvec {args.hpsi_nvec}: 3 applications", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
