"""Write lengths_sigma.json: for every built FFT length, the oracle's
Sigma_c,i(t_j), X_i and QP energies of the short case in lengths_cases.py
(FP64; spectral interval = the oracle's rigorous bounds with 1% padding).

    python tests/golden/make_lengths_sigma.py [n ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from conftest import build_oracle_h  # noqa: E402
from lengths_cases import EPS_KS, LENGTHS, length_params, length_phi, length_system  # noqa: E402
from oracle import qp as oqp  # noqa: E402
from oracle.sigma import SGWParams, estimate  # noqa: E402

OUT = os.path.join(HERE, "lengths_sigma.json")


def one(n):
    s = length_system(n)
    H = build_oracle_h(s, workers=os.cpu_count())
    emin, emax = H.bounds(0.01)
    kw = length_params(n, emin, emax)
    phi = length_phi(s)
    sig, x = estimate(H, phi, SGWParams(mode="xi", **kw))
    gam = oqp.default_gamma(kw["n_tau"], kw["dt"])
    eg, el, z = oqp.qp_solve(sig.mean(0), kw["dt"], gam, EPS_KS, x.mean())
    return dict(system=s.name, params=kw, sigma_re=sig.real.tolist(), sigma_im=sig.imag.tolist(),
                x=x.tolist(), eqp_graphical=eg, eqp_linear=el, z=z)


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
