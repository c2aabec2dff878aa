"""The per-FFT-length parity cases: one system and one short Sigma_c(t)
parameter set for every built grid length (16 ... 128).  Inputs only (seeded
systems from the shared input generators and plain parameter values); the
expected values are written by make_lengths_sigma.py with the oracle.

Systems: n = 16, 24: the two-well test system with one s and one p_x
projector (boxes too small for a cluster); n >= 40: H-capped Si clusters at
h = 0.6 bohr with E_cut = 28 Ha (the grid spacing of the 128^3 and uneven-
batch configurations), the cluster size growing with the box; n = 128 is the
Si357H204 stand-in of the 128^3 configuration itself.
"""
import numpy as np

from paper_2601_21005_amd import systems

LENGTHS = (16, 24, 40, 48, 56, 80, 96, 112, 128)
CLUSTER_SI = {40: 5, 48: 17, 56: 17, 80: 47, 96: 87, 112: 147}


def length_system(n):
    if n == 16:
        return systems.tiny_system(16, 0.7)
    if n == 24:
        return systems.tiny_system(24, 0.6)
    if n == 128:
        return systems.si357h204()
    species, pos = systems.si_cluster(CLUSTER_SI[n], seed=3000 + n)
    return systems.cluster_model(species, pos, n=n, h=0.6, ecut=28.0,
                                 name=f"Si{CLUSTER_SI[n]}H{species.count('H')}")


def length_phi(system):
    """Normalised Gaussian (width 1.5 bohr) at the box centre: the orbital
    whose self-energy the short runs estimate."""
    g = system.grid
    r = systems.grid_coords(g) - 0.5 * g.L
    phi = np.exp(-np.sum(r * r, axis=1) / (2 * 1.5 ** 2))
    return phi / np.sqrt(g.h ** 3 * np.sum(phi * phi))


def length_params(n, emin, emax):
    """Short estimate: 1 sample, N_eta = 2, 4 output steps of 0.1 au (two
    Strang substeps each), a 60-term Fermi filter, 256 xi functions."""
    return dict(seed=2000 + n, n_zeta=1, n_eta=2, n_tau=4, dt=0.1, m_sub=2,
                mu=emin + 0.2 * (emax - emin), beta=2.0, ncoef=60, emin=emin, emax=emax,
                n_xi=256, f_g=0.02)


EPS_KS = -0.5      # Ha: the KS energy handed to the QP solve (any fixed value)
