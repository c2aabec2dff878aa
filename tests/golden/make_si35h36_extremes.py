"""Write si35h36_64_extremes.json: the lowest and highest eigenvalues of the
64^3 Si35H36-shaped cluster Hamiltonian (h = 0.5 bohr, E_cut = 28 Ha), from
the FP64 oracle's Lanczos eigensolvers (ARPACK on the oracle's H).  Every
Chebyshev map of Sec. 2.1 needs an interval that encloses these two values.

    python tests/golden/make_si35h36_extremes.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from conftest import build_oracle_h  # noqa: E402
from oracle import eigen  # noqa: E402
from paper_2601_21005_amd import systems  # noqa: E402


def main():
    s = systems.si35h36()
    H = build_oracle_h(s, workers=os.cpu_count())
    e_lo, _ = eigen.lowest_states(H, 1, tol=1e-10)
    e_hi = eigen.highest_eigenvalue(H, tol=1e-6)
    out = dict(system="Si35H36 stand-in, 64^3, h=0.5 bohr, ecut=28 Ha (systems.si35h36())",
               method="oracle.eigen.lowest_states (tol 1e-10) / highest_eigenvalue (tol 1e-6)",
               e_min=float(e_lo[0]), e_max=float(e_hi))
    with open(os.path.join(HERE, "si35h36_64_extremes.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
