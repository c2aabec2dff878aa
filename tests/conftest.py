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


def make_ctx(system, precision, max_nvec=64):
    """libsgw context for a ``systems.System`` (GPU tests only)."""
    from paper_2601_21005_amd import sgw
    return sgw.Context(system.grid.n, system.grid.h, system.v_loc, system.projectors,
                       precision=precision, ecut=system.ecut, max_nvec=max_nvec)


def rel_err(a, b):
    """max |a - b| / max |b|."""
    import numpy as np
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def row_max_err(a, b):
    """max |a - b| / max |b| per row (max over rows): the element-wise check
    beside the normwise one."""
    import numpy as np
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    return float(np.max(np.max(np.abs(a - b), axis=-1) / np.max(np.abs(b), axis=-1)))


def norm_err(a, b):
    """||a - b|| / ||b|| per row (max over rows)."""
    import numpy as np
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    return float(np.max(np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)))


@pytest.fixture(scope="session")
def cfg1():
    from paper_2601_21005_amd import systems
    s = systems.gaussian_wells()
    return s, build_oracle_h(s)


@pytest.fixture(scope="session")
def si35():
    from paper_2601_21005_amd import systems
    s = systems.si35h36()
    return s, build_oracle_h(s, workers=8)


@pytest.fixture(scope="session")
def tiny12l():
    """12^3 local-only system (radix-3 FFT path; KB tiles need n % 8 == 0)."""
    from paper_2601_21005_amd import systems
    s = systems.tiny_system(12, 0.5, with_kb=False)
    return s, build_oracle_h(s)


@pytest.fixture(scope="session")
def tiny12l_eig(tiny12l):
    from oracle import eigen
    s, H = tiny12l
    return eigen.dense_eigh(H)
