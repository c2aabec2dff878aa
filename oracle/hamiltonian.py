"""Kohn-Sham Hamiltonian on the grid (oracle side).

H = -1/2 nabla^2 + V_loc + V_NL, Eq. (1).  The kinetic term is diagonal in k,
the local potential in r (Sec. 2.2).  Norm-conserving pseudopotentials have a
local part and a separable (Kleinman-Bylander) non-local part whose projectors
of neighbouring atoms overlap (Sec. 3, discussion of the wall times).

Readings (the paper gives no pseudopotential tables):
* V_loc is an input array (the model's local potential, V_H and V_xc folded in).
* Each KB projector p sits on an atom R_p with angular channel l in {0, 1}:
      beta_s(r)       = N_p exp(-|d|^2 / (2 rc^2))
      beta_{p,a}(r)   = N_p d_a exp(-|d|^2 / (2 rc^2)),   a = m in {x, y, z}
  with d the minimum-image displacement r - R_p, cut to zero where
  |d| > rcut_over_rc * rc, and N_p chosen so that dV sum beta_p^2 = 1 on the
  grid.  V_NL = sum_p |beta_p> E_p <beta_p|.
* Kinetic cutoff (Sec. 3 clips the kinetic operator at 28 Ha to bound the
  spectral width): T(k) = min(|k|^2/2, E_cut) when E_cut > 0.
"""
import numpy as np
import scipy.sparse as sp

from .grid import Grid


def kinetic(grid: Grid, ecut=0.0):
    """T(k) on the flat k grid, optionally clipped at the cutoff."""
    T = 0.5 * grid.k2()
    if ecut and ecut > 0:
        T = np.minimum(T, ecut)
    return T


class Projectors:
    """Kleinman-Bylander projectors as a sparse (N_g x N_p) matrix B."""

    def __init__(self, grid: Grid, pos, atom_of, l, m, rc, ekb, rcut_over_rc=6.0):
        self.grid = grid
        pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
        self.atom_of = np.asarray(atom_of, dtype=np.int64)
        self.l = np.asarray(l, dtype=np.int64)
        self.m = np.asarray(m, dtype=np.int64)
        self.rc = np.asarray(rc, dtype=np.float64)
        self.ekb = np.asarray(ekb, dtype=np.float64)
        self.np_ = len(self.l)
        nx, ny, nz = grid.n
        L = np.asarray(grid.L)
        rows, cols, vals = [], [], []
        for p in range(self.np_):
            rcut = rcut_over_rc * self.rc[p]
            # candidate points: the box of grid lines whose per-axis
            # minimum-image offset is within rcut (it holds the whole sphere);
            # flat indices ascending, as over the full grid
            ax = []
            for a, m in enumerate((nx, ny, nz)):
                da = np.mod(grid.h * np.arange(m) - pos[self.atom_of[p], a] + 0.5 * L[a],
                            L[a]) - 0.5 * L[a]
                ax.append(np.nonzero(np.abs(da) <= rcut)[0])
            ix, iy, iz = ax
            cand = (ix[None, None, :] + nx * (iy[None, :, None] + ny * iz[:, None, None])).ravel()
            cand.sort()
            rr = grid.h * np.stack([cand % nx, (cand // nx) % ny, cand // (nx * ny)], axis=1)
            d = grid.min_image(rr - pos[self.atom_of[p]])
            d2 = np.sum(d * d, axis=1)
            inside = d2 <= rcut * rcut
            g = np.exp(-d2[inside] / (2.0 * self.rc[p] ** 2))
            if self.l[p] == 1:
                g = g * d[inside, self.m[p]]
            elif self.l[p] != 0:
                raise ValueError("only s and p projectors are modelled")
            nrm = np.sqrt(grid.dV * np.sum(g * g))
            idx = cand[inside]
            rows.append(idx)
            cols.append(np.full(idx.size, p))
            vals.append(g / nrm)
        self.B = sp.csc_matrix((np.concatenate(vals),
                                (np.concatenate(rows), np.concatenate(cols))),
                               shape=(grid.N, self.np_))

    def gram(self):
        """S_pq = <beta_p|beta_q> (dense, FP64)."""
        S = (self.B.T @ self.B).toarray() * self.grid.dV
        return S

    def project(self, psi):
        """C[v, p] = <beta_p|psi_v> for psi of shape (nvec, N)."""
        return self.grid.dV * (self.B.T @ psi.T).T

    def expand(self, C):
        """sum_p beta_p C[v, p] for C of shape (nvec, N_p)."""
        return (self.B @ C.T).T

    def apply(self, psi):
        """V_NL psi = sum_p beta_p E_p <beta_p|psi>."""
        return self.expand(self.project(psi) * self.ekb[None, :])


class Hamiltonian:
    """H = T + V_loc + V_NL acting on batches (nvec, N) of grid vectors."""

    def __init__(self, grid: Grid, v_loc, projectors: Projectors = None, ecut=0.0):
        self.grid = grid
        self.v = np.asarray(v_loc, dtype=np.float64).ravel()
        assert self.v.size == grid.N
        self.kb = projectors
        self.ecut = float(ecut) if ecut else 0.0
        self.T = kinetic(grid, self.ecut)

    def apply_local(self, psi):
        psi = np.atleast_2d(psi)
        out = self.grid.ifft(self.T * self.grid.fft(psi)) + self.v * psi
        if np.isrealobj(psi):
            out = out.real
        return out

    def apply(self, psi):
        """H|psi> for psi of shape (N,) or (nvec, N)  (Eq. 1, Sec. 2.2)."""
        single = np.ndim(psi) == 1
        psi2 = np.atleast_2d(psi)
        out = self.apply_local(psi2)
        if self.kb is not None:
            out = out + self.kb.apply(psi2)
        return out[0] if single else out

    def dense(self):
        """Dense matrix of H, column by column (small grids only)."""
        N = self.grid.N
        I = np.eye(N)
        return self.apply(I).T  # apply acts on rows; column j = H e_j

    # ---- spectral bounds ------------------------------------------------
    def tmax(self):
        return float(np.max(self.T))

    def kb_bounds(self):
        """Rigorous bounds of spec(V_NL): V_NL = dV B E B^T, whose non-zero
        spectrum lies in [min(E,0), max(E,0)] * lambda_max(S), S = dV B^T B,
        with lambda_max(S) bounded by the Gershgorin row sum."""
        if self.kb is None:
            return 0.0, 0.0
        S = self.kb.gram()
        smax = float(np.max(np.sum(np.abs(S), axis=1)))
        lo = min(0.0, float(np.min(self.kb.ekb))) * smax
        hi = max(0.0, float(np.max(self.kb.ekb))) * smax
        return lo, hi

    def bounds(self, pad=0.01):
        """Weyl bounds [E_min, E_max] of H, padded by ``pad`` times the width
        on each side.  The paper obtains the bounds by shifted power iteration
        (Sec. 2.1); any enclosing interval gives the same filter definition
        once the interval is fixed, so the oracle uses rigorous bounds."""
        lo, hi = self.kb_bounds()
        emin = float(np.min(self.v)) + lo
        emax = self.tmax() + float(np.max(self.v)) + hi
        w = emax - emin
        return emin - pad * w, emax + pad * w
