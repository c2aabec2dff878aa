"""Pins for H|psi> (Eq. 1 on the Fourier grid), the KB term and the bounds."""
import numpy as np
import scipy.linalg as sla

from oracle.grid import Grid
from oracle.hamiltonian import Hamiltonian, Projectors, kinetic
from paper_2601_21005_amd import systems


def test_dense_h_symmetric(tiny12):
    s, H = tiny12
    A = H.dense()
    assert np.max(np.abs(A - A.T)) < 1e-12 * np.max(np.abs(A))


def test_plane_waves_are_kinetic_eigenvectors():
    g = Grid(12, 10, 8, h=0.6)
    H = Hamiltonian(g, np.zeros(g.N))
    r = g.coords()
    L = np.array(g.L)
    for m in [(0, 0, 0), (1, 0, 0), (2, -3, 1), (-6, 5, -4)]:   # incl. Nyquist
        k = 2 * np.pi * np.array(m) / L
        psi = np.exp(1j * r @ k)
        out = H.apply(psi)
        # (-6, ...) is the Nyquist index along x: exp(+-i k x) coincide on
        # the grid and T is even, so the eigenvalue is unchanged
        expect = 0.5 * np.dot(k, k)
        assert np.allclose(out, expect * psi, atol=1e-11)


def test_gaussian_laplacian_closed_form():
    g = Grid(32, h=0.5)
    H = Hamiltonian(g, np.zeros(g.N))
    r = g.coords()
    c = np.array(g.L) / 2 + np.array([0.13, -0.21, 0.05])
    s = 1.2
    d2 = np.sum(g.min_image(r - c) ** 2, axis=1)
    f = np.exp(-d2 / (2 * s * s))
    # -1/2 lap exp(-r^2/2s^2) = -1/2 f (r^2/s^4 - 3/s^2)
    expect = -0.5 * f * (d2 / s ** 4 - 3.0 / s ** 2)
    assert np.max(np.abs(H.apply(f) - expect)) < 1e-8


def test_kinetic_cutoff_clips():
    g = Grid(16, h=0.5)
    T = kinetic(g, 5.0)
    T0 = kinetic(g)
    assert np.all(T <= 5.0) and np.allclose(T[T0 <= 5.0], T0[T0 <= 5.0])
    assert np.isclose(T0.max(), 1.5 * (np.pi / 0.5) ** 2)


def test_projector_shape_and_normalisation(tiny12):
    s, H = tiny12
    P = H.kb
    g = H.grid
    B = P.B.toarray()
    assert np.allclose(g.dV * np.sum(B * B, axis=0), 1.0)
    r = g.coords()
    # s projector radial about its atom; p_x odd in x about its atom
    d0 = g.min_image(r - s.projectors.pos[0])
    rad = np.sqrt(np.sum(d0 ** 2, axis=1))
    nz = B[:, 0] != 0
    assert np.all(B[nz, 0] > 0)
    order = np.argsort(rad[nz])
    assert np.all(np.diff(B[nz, 0][order]) <= 1e-15)
    d1 = g.min_image(r - s.projectors.pos[1])
    nz1 = B[:, 1] != 0
    assert np.all(np.sign(B[nz1, 1]) == np.sign(d1[nz1, 0]))
    # cut radius respected
    assert np.max(rad[nz]) <= 3.0 * 0.75 + 1e-12



def test_projector_widths_from_second_moments():
    """The projector shapes fix the second moments of beta^2: for an s
    projector beta^2 is a Gaussian of variance rc^2/2 per axis, so
    <|d|^2> = 3 rc^2 / 2; for p_x it is x^2 times that Gaussian, so
    <x^2> = 3 rc^2 / 2 (fourth over second moment) and <y^2> = <z^2> =
    rc^2 / 2.  On a fine grid with the cut at 5 rc the sums reach these
    values to 1e-7 (the trapezoid rule is spectrally accurate here; what is
    left is the tail beyond the cut)."""
    g = Grid(32, h=0.25)
    rc = 0.8
    pos = np.array([[4.0, 4.0, 4.0]])
    P = Projectors(g, pos, [0, 0], [0, 1], [0, 0], [rc, rc], [1.0, 1.0], rcut_over_rc=5.0)
    d = g.min_image(g.coords() - pos[0])
    B = P.B.toarray()
    w_s, w_p = g.dV * B[:, 0] ** 2, g.dV * B[:, 1] ** 2
    assert np.isclose(w_s.sum(), 1.0) and np.isclose(w_p.sum(), 1.0)
    assert abs(np.sum(w_s * np.sum(d * d, axis=1)) - 1.5 * rc * rc) < 1e-7
    assert abs(np.sum(w_p * d[:, 0] ** 2) - 1.5 * rc * rc) < 1e-7
    for a in (1, 2):
        assert abs(np.sum(w_p * d[:, a] ** 2) - 0.5 * rc * rc) < 1e-7


def test_projector_support_includes_the_cut_sphere():
    """The support is |d| <= rcut, boundary included: with the atom on a grid
    point and rcut = 2 h the s projector covers the lattice points of the
    ball of radius 2 in grid units, 1 + 6 + 12 + 8 + 6 = 33 (distances 0, 1,
    sqrt 2, sqrt 3, 2), of which the last 6 lie on the sphere itself."""
    g = Grid(12, h=0.5)
    P = Projectors(g, np.array([[1.5, 2.0, 2.5]]), [0], [0], [0], [0.5], [1.0],
                   rcut_over_rc=2.0)
    assert P.B.nnz == 33
    d = g.min_image(g.coords() - np.array([1.5, 2.0, 2.5]))
    on_sphere = np.isclose(np.sum(d * d, axis=1), 1.0)
    assert on_sphere.sum() == 6 and np.all(P.B.toarray()[on_sphere, 0] > 0)

def test_nonlocal_matches_dense_sum(tiny8):
    s, H = tiny8
    g = H.grid
    B = H.kb.B.toarray()
    Vnl = g.dV * B @ np.diag(H.kb.ekb) @ B.T
    psi = np.random.default_rng(1).standard_normal((3, g.N))
    assert np.allclose(H.kb.apply(psi), psi @ Vnl.T, atol=1e-12)


def test_bounds_enclose_spectrum(tiny12, tiny12_eig):
    s, H = tiny12
    e, _ = tiny12_eig
    lo, hi = H.bounds(pad=0.0)
    assert lo <= e.min() + 1e-10 and e.max() <= hi + 1e-10
    S = H.kb.gram()
    lam = sla.eigvalsh(S).max()
    assert lam <= np.max(np.sum(np.abs(S), axis=1)) + 1e-12


def test_cluster_projector_count_and_occupation():
    s = systems.si35h36()
    assert s.projectors.nproj == 35 * 4 + 36
    assert s.n_occ == 88


def test_lanczos_bounds_enclose_and_converge(tiny8, tiny8_eig):
    """40 Lanczos steps on the 8^3 system: the interval encloses the dense
    spectrum, its ends lie within 2% of the spectral width of the extreme
    eigenvalues, and it is inside the rigorous bounds."""
    from oracle import eigen
    s, H = tiny8
    e, _ = tiny8_eig
    lo, hi = eigen.lanczos_bounds(H, 40, seed=3, pad=0.01)
    w = e[-1] - e[0]
    assert lo <= e[0] and hi >= e[-1]
    assert e[0] - lo < 0.02 * w and hi - e[-1] < 0.02 * w
    lw, hw = H.bounds(0.0)
    assert lw <= lo and hi <= hw



def test_lanczos_residual_widening_encloses(tiny8, tiny8_eig):
    """Ritz values never leave the spectrum's hull, so it is the residual
    term r = beta_k |y_last| that widens the interval to the extreme
    eigenvalues: with no padding it encloses the 8^3 spectrum after 8, 10, 12
    and 16 steps, while the extreme Ritz values alone stay inside it (after 5
    steps it does not: the widening is a residual estimate, not a bound)."""
    from oracle import eigen
    s, H = tiny8
    e, _ = tiny8_eig
    for k in (8, 10, 12, 16):
        lo, hi = eigen.lanczos_bounds(H, k, seed=3, pad=0.0)
        assert lo <= e[0] and hi >= e[-1], k

def test_lanczos_ritz_values_are_exact_for_a_diagonal_operator():
    """On a 3-level operator every Krylov space of dimension >= 3 holds the
    three eigenvectors' span: the Ritz values are the eigenvalues."""
    import numpy as np
    from oracle import eigen
    from oracle.grid import Grid

    class Diag:
        def __init__(self):
            self.grid = Grid(4, h=1.0)
            self.d = np.repeat([-2.0, 0.5, 3.0], [20, 20, 24])

        def apply(self, x):
            return self.d * x

        def bounds(self, pad=0.0):
            return -10.0, 10.0

    lo, hi = eigen.lanczos_bounds(Diag(), 6, seed=1, pad=0.0)
    assert abs(lo + 2.0) < 1e-10 and abs(hi - 3.0) < 1e-10
