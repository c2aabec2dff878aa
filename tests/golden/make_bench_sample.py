"""Write bench_sample_si35h36_64.npz: one Monte Carlo sample of the benchmark
workload computed by the FP64 oracle alone.

Workload: the Si35H36-shaped cluster on a 64^3 grid (h = 0.5 bohr, E_cut =
28 Ha, 176 KB projectors), N_eta = 64, 400 output steps of 0.05 au (one
Strang substep each), N_xi = 10000 at f_g = 0.003, the gapped filter with
1e-7 at the gap edges and a discarded coefficient tail below 1e-7, seed 1002,
sample 0, with the scale max_j sum_m |c_m(t_j) d_m(t_j)| of its xi
contraction.  Every input the sample needs comes from the oracle: the spectral
interval from 60 Lanczos steps (seed 1, 1 % padding), the band edges and the
HOMO orbital from its Lanczos eigensolver (the orbital is stored rounded to
FP32 and used in that rounded form on both sides).  About 40 minutes on 8
cores.

    python tests/golden/make_bench_sample.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

from conftest import build_oracle_h  # noqa: E402
from oracle import chebyshev as cheb  # noqa: E402
from oracle import eigen  # noqa: E402
from oracle import qp as oqp  # noqa: E402
from oracle.sigma import SGWParams, sample_sigma  # noqa: E402
from paper_2601_21005_amd import systems  # noqa: E402

OUT = os.path.join(HERE, "bench_sample_si35h36_64.npz")


def main():
    t0 = time.time()
    s = systems.si35h36()
    H = build_oracle_h(s, workers=os.cpu_count())
    emin, emax = eigen.lanczos_bounds(H, 60, seed=1, pad=0.01)
    e, V = eigen.lowest_states(H, s.n_occ + 1, tol=1e-10)
    homo, lumo = float(e[s.n_occ - 1]), float(e[s.n_occ])
    phi = V[s.n_occ - 1].astype(np.float32).astype(np.float64)
    eps = 1e-7
    a = cheb.gapped_coefficients(homo, lumo, eps, emin, emax, 8192)
    ncoef = int(cheb.tail_length(a, 1e-7))
    print(f"inputs: [{emin:.6f}, {emax:.6f}] homo {homo:.8f} lumo {lumo:.8f} "
          f"ncoef {ncoef} ({time.time() - t0:.0f} s)", flush=True)
    p = dict(seed=1002, n_zeta=1, n_eta=64, n_tau=400, dt=0.05, m_sub=1, mu=0.0, beta=0.0,
             ncoef=ncoef, emin=emin, emax=emax, n_xi=10000, f_g=0.003, filter="gapped",
             e_homo=homo, e_lumo=lumo, filter_eps=eps)
    sp = SGWParams(mode="xi", **p)
    sig, x, parts = sample_sigma(H, phi, sp, 0, return_parts=True)
    sig, x = sig[None], np.array([x])
    # scale of the contraction Sigma(t_j) = sum_m c_m d_m (rounding errors of
    # the terms add up on this scale, not on |Sigma|)
    scale = max(float(np.max(np.sum(np.abs(parts["c"] * parts["dp"]), axis=0))),
                float(np.max(np.sum(np.abs(parts["c"] * parts["dm"]), axis=0))))
    gam = oqp.default_gamma(p["n_tau"], p["dt"])
    eg, el, z = oqp.qp_solve(sig.mean(0), p["dt"], gam, homo, x.mean())
    np.savez_compressed(OUT, phi=phi.astype(np.float32), sigma=sig, x=x,
                        params=json.dumps(p), eqp=np.array([eg, el, z]),
                        sigma_term_scale=np.array(scale))
    print(f"done in {time.time() - t0:.0f} s: X {x[0]:.8f} eqp {eg:.8f}", flush=True)


if __name__ == "__main__":
    main()
