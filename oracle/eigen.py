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


def lanczos_bounds(H, k, seed=0, pad=0.01):
    """Spectral interval of H from k Lanczos steps (the paper finds the
    interval by shifted power iteration, Sec. 2.1; Lanczos is the Krylov
    method that gives both ends from one sequence).

    Start: the +-1 white-noise vector of stream (BOUNDS, 0, 0), unit norm in
    the plain Euclidean sense.  Steps: w = H v_j - alpha_j v_j - beta_j v_{j-1},
    alpha_j = <v_j, H v_j>, beta_{j+1} = |w|, no reorthogonalisation (it does
    not move the extreme Ritz values).  Ritz values theta and residual norms
    r = beta_k |y_last| of the k x k tridiagonal; every Ritz value lies within
    r of an eigenvalue.  The interval is
        [theta_min - r_min - pad w, theta_max + r_max + pad w],
    w = theta_max - theta_min, each end clipped to the rigorous bounds of
    ``H.bounds(0)`` (Weyl plus Gershgorin), which it can only narrow."""
    from scipy.linalg import eigh_tridiagonal
    from . import rng
    N = H.grid.N
    v = rng.white_noise_signs(seed, rng.stream_id(rng.BOUNDS, 0, 0), N)
    v = v / np.linalg.norm(v)
    v_prev = np.zeros(N)
    alpha, beta = [], []
    b = 0.0
    for _ in range(k):
        w = H.apply(v)
        a = float(v @ w)
        w = w - a * v - b * v_prev
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        if b == 0.0:
            break
        v_prev, v = v, w / b
    theta, Y = eigh_tridiagonal(np.array(alpha), np.array(beta[:-1]))
    r = beta[-1] * np.abs(Y[-1, :])
    lo_w, hi_w = H.bounds(0.0)
    width = theta[-1] - theta[0]
    lo = max(lo_w, theta[0] - r[0] - pad * width)
    hi = min(hi_w, theta[-1] + r[-1] + pad * width)
    return lo, hi


def highest_eigenvalue(H, tol=1e-10, v0_seed=11):
    """The largest eigenvalue of H by Lanczos (ARPACK, largest algebraic)
    on the unshifted operator; the upper end of the interval that every
    Chebyshev map of Sec. 2.1 needs."""
    N = H.grid.N

    def mv(x):
        return H.apply(np.asarray(x, dtype=np.float64).ravel())

    op = spla.LinearOperator((N, N), matvec=mv, dtype=np.float64)
    v0 = np.random.default_rng(v0_seed).standard_normal(N)
    e = spla.eigsh(op, k=1, which="LA", tol=tol, v0=v0, ncv=min(N, 40),
                   return_eigenvectors=False)
    return float(e[0])
