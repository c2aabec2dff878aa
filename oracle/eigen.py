"""Reference eigensolvers for the method's inputs (oracle side).

The method takes the orbital phi_k, and the HOMO/LUMO energies that place the
filter's cutoff, from a preliminary DFT calculation (Sec. 2.1).  With the
synthetic model Hamiltonians used here those come from diagonalising H:
densely on small grids, iteratively (ARPACK Lanczos through scipy) otherwise.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def dense_eigh(H):
    """All eigenpairs of the dense H (small grids).  Columns of the returned
    vectors are normalised so that <phi|phi> = dV sum phi^2 = 1."""
    A = H.dense()
    A = 0.5 * (A + A.T)
    e, V = sla.eigh(A)
    return e, V.T / np.sqrt(H.grid.dV)


def lowest_states(H, k, tol=1e-10, v0_seed=7):
    """The k lowest eigenpairs by Lanczos on the shifted operator.
    Returns energies (k,) and orbitals (k, N) with <phi|phi> = 1."""
    N = H.grid.N
    emin, emax = H.bounds(pad=0.0)
    shift = emax  # H - emax <= 0: the lowest states become the largest in magnitude

    def mv(x):
        x = np.asarray(x, dtype=np.float64).ravel()
        return H.apply(x) - shift * x

    op = spla.LinearOperator((N, N), matvec=mv, dtype=np.float64)
    v0 = np.random.default_rng(v0_seed).standard_normal(N)
    e, V = spla.eigsh(op, k=k, which="LM", tol=tol, v0=v0,
                      ncv=min(N, max(2 * k + 1, k + 32)))
    e = e + shift
    order = np.argsort(e)
    e, V = e[order], V[:, order]
    return e, V.T / np.sqrt(H.grid.dV)
