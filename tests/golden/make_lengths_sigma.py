"""Write lengths_sigma.json: for every built FFT length, the oracle's
Sigma_c,i(t_j), X_i and QP energies of the short case in lengths_cases.py
(FP64; spectral interval = the oracle's rigorous bounds with 1% padding),
and the scale of the xi contraction, max_j sum_m |c_m(t_j) d_m(t_j)|.

    python tests/golden/make_lengths_sigma.py [n ...]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from conftest import build_oracle_h  # noqa: E402
from lengths_cases import EPS_KS, LENGTHS, length_params, length_phi, length_system  # noqa: E402
from oracle import qp as oqp  # noqa: E402
from oracle.sigma import SGWParams, sample_sigma  # noqa: E402

OUT = os.path.join(HERE, "lengths_sigma.json")


def one(n):
    s = length_system(n)
    H = build_oracle_h(s, workers=os.cpu_count())
    emin, emax = H.bounds(0.01)
    kw = length_params(n, emin, emax)
    phi = length_phi(s)
    p = SGWParams(mode="xi", **kw)
    assert p.n_zeta == 1
    sig, x, parts = sample_sigma(H, phi, p, p.first_sample, return_parts=True)
    sig, x = sig[None], np.array([x])
    # scale of the contraction Sigma(t_j) = sum_m c_m d_m: the largest sum of
    # the magnitudes of its terms over the time axis (rounding errors of the
    # terms add up on this scale, not on |Sigma|)
    scale = max(float(np.max(np.sum(np.abs(parts["c"] * parts["dp"]), axis=0))),
                float(np.max(np.sum(np.abs(parts["c"] * parts["dm"]), axis=0))))
    gam = oqp.default_gamma(kw["n_tau"], kw["dt"])
    eg, el, z = oqp.qp_solve(sig.mean(0), kw["dt"], gam, EPS_KS, x.mean())
    return dict(system=s.name, params=kw, sigma_re=sig.real.tolist(), sigma_im=sig.imag.tolist(),
                x=x.tolist(), sigma_term_scale=scale, eqp_graphical=eg, eqp_linear=el, z=z)


def main():
    ns = [int(a) for a in sys.argv[1:]] or list(LENGTHS)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for n in ns:
        t0 = time.time()
        data[str(n)] = one(n)
        print(f"n={n}: {time.time() - t0:.1f} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=0)


if __name__ == "__main__":
    main()
