import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU oracle test")


def build_oracle_h(system, workers=None):
    """Oracle Hamiltonian for a ``systems.System``."""
    from oracle.grid import Grid
    from oracle.hamiltonian import Hamiltonian, Projectors
    g = Grid(system.grid.n, h=system.grid.h, workers=workers)
    P = None
    if system.projectors is not None:
        p = system.projectors
        P = Projectors(g, p.pos, p.atom_of, p.l, p.m, p.rc, p.ekb, p.rcut_over_rc)
    return Hamiltonian(g, system.v_loc, P, system.ecut)


@pytest.fixture(scope="session")
def tiny8():
    from paper_2601_21005_amd import systems
    s = systems.tiny_system(8, 0.7)
    return s, build_oracle_h(s)


@pytest.fixture(scope="session")
def tiny8_eig(tiny8):
    from oracle import eigen
    s, H = tiny8
    e, V = eigen.dense_eigh(H)
    return e, V


@pytest.fixture(scope="session")
def tiny12():
    from paper_2601_21005_amd import systems
    s = systems.tiny_system(12, 0.5)
    return s, build_oracle_h(s)


@pytest.fixture(scope="session")
def tiny12_eig(tiny12):
    from oracle import eigen
    s, H = tiny12
    return eigen.dense_eigh(H)
