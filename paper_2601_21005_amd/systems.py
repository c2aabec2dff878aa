"""Seeded synthetic inputs: grids, model potentials and projector lists.

The paper's inputs are DFT-derived: atomic coordinates of relaxed
H-passivated Si clusters cut from a diamond superlattice (a = 10.26 bohr),
pseudopotentials per atom type, the ground-state density and the orbital of
interest (Sec. 2.1, Sec. 3).  None of these is available, so this module
builds stand-ins of the same shape, deterministically from a seed:

* ``gaussian_wells``: 8 attractive Gaussians (depth 2 Ha, width 1 bohr) at
  seeded positions in the central half of a periodic box.
* ``si_cluster``: atom-centred shells of the diamond lattice, H caps along
  the missing tetrahedral bonds, uniform +-0.05 bohr seeded jitter.
* ``cluster_model``: a model local potential (one Gaussian well per atom) and
  Kleinman-Bylander projector descriptions (1 s + 3 p per Si, 1 s per H) with
  Gaussian radial parts.  The parameters are a synthetic model chosen so that
  the lowest N_p / 2 states (N_p = number of projectors = number of valence
  electrons) lie below a clear gap; they are not fitted to silicon.

This module is the only code shared by the oracle side and the library side
of the tests.  It holds inputs only, none of the method's arithmetic: it
never applies H, filters, propagates or contracts anything.
"""
from dataclasses import dataclass, field

import numpy as np

A_SI = 10.26                       # bohr, diamond cubic Si (Sec. 3)
D_SISI = A_SI * np.sqrt(3.0) / 4.0  # nearest-neighbour distance
D_SIH = 2.80                       # bohr, Si-H cap distance (model choice)

# Model parameters per species: local Gaussian well (depth A, width s) and
# KB projectors (radius rc, energies).  Synthetic, frozen.
SPECIES = {
    "Si": dict(A=1.0, s=1.3, rc=1.25, e_s=-6.0, e_p=-4.0, zval=4),
    "H": dict(A=1.0, s=0.8, rc=0.9, e_s=-6.0, e_p=None, zval=1),
}
RCUT_OVER_RC = 6.0


@dataclass
class GridSpec:
    n: int
    h: float

    @property
    def N(self):
        return self.n ** 3

    @property
    def L(self):
        return self.n * self.h


@dataclass
class ProjectorSpec:
    """Projector list in the library's CSR layout."""
    pos: np.ndarray            # (natom, 3) bohr
    proj_begin: np.ndarray     # (natom + 1,) int32
    l: np.ndarray              # (nproj,) int32
    m: np.ndarray              # (nproj,) int32, 0..2l
    rc: np.ndarray             # (nproj,) bohr
    ekb: np.ndarray            # (nproj,) Ha
    rcut_over_rc: float = RCUT_OVER_RC

    @property
    def nproj(self):
        return int(self.l.size)

    @property
    def atom_of(self):
        counts = np.diff(self.proj_begin)
        return np.repeat(np.arange(counts.size), counts)


@dataclass
class System:
    name: str
    grid: GridSpec
    v_loc: np.ndarray          # (N,) Ha, x fastest
    projectors: ProjectorSpec = None
    n_occ: int = 0
    ecut: float = 0.0
    species: list = field(default_factory=list)
    pos: np.ndarray = None


def grid_coords(g: GridSpec):
    i = np.arange(g.n)
    iz, iy, ix = np.meshgrid(i, i, i, indexing="ij")
    return g.h * np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)


def _min_image(d, L):
    return np.mod(d + 0.5 * L, L) - 0.5 * L


def gaussian_wells(seed=1010, n=32, h=0.5, nwell=8, depth=2.0, width=1.0,
                   n_occ=8):
    """8 Gaussian wells, depth 2 Ha, width 1 bohr, centres uniform in the
    central half [L/4, 3L/4]^3 of the box (local-only H)."""
    g = GridSpec(n, h)
    L = g.L
    rs = np.random.default_rng(seed)
    centres = rs.uniform(0.25 * L, 0.75 * L, size=(nwell, 3))
    r = grid_coords(g)
    v = np.zeros(g.N)
    for c in centres:
        d = _min_image(r - c, L)
        v -= depth * np.exp(-np.sum(d * d, axis=1) / (2.0 * width ** 2))
    return System("gaussian_wells", g, v, None, n_occ=n_occ, pos=centres)


def diamond_sites(nmax=6):
    """Diamond-lattice positions (bohr) around an atom at the origin."""
    base = np.array([[0, 0, 0], [0, 2, 2], [2, 0, 2], [2, 2, 0],
                     [1, 1, 1], [1, 3, 3], [3, 1, 3], [3, 3, 1]], dtype=np.int64)
    r = np.arange(-nmax, nmax + 1)
    cells = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3) * 4
    sites = (cells[:, None, :] + base[None, :, :]).reshape(-1, 3)  # units a/4
    return sites


def si_cluster(n_si=35, seed=1002, jitter=0.05):
    """Atom-centred H-capped diamond fragment with ``n_si`` Si atoms.
    ``n_si`` must close a neighbour shell around the central atom
    (1, 5, 17, 29, 35, 47, 71, 87, 99, 123, 147, ...).  Returns
    (species list, positions (natom, 3) bohr, centred at the origin)."""
    sites = diamond_sites()
    d2 = np.sum(sites * sites, axis=1)
    order = np.lexsort((sites[:, 2], sites[:, 1], sites[:, 0], d2))
    sites, d2 = sites[order], d2[order]
    if n_si < len(sites) and d2[n_si - 1] == d2[n_si]:
        raise ValueError("n_si does not close a shell")
    si = sites[:n_si]
    present = {tuple(s) for s in si}
    # sublattice A (all coordinates even, units a/4) bonds along
    # (1,1,1),(1,-1,-1),(-1,1,-1),(-1,-1,1); sublattice B the opposite.
    dirs = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]])
    hs = []
    for s in si:
        sgn = 1 if s[0] % 2 == 0 else -1
        for dvec in dirs * sgn:
            nb = tuple(s + dvec)
            if nb not in present:
                u = dvec / np.sqrt(3.0)
                hs.append(s * (A_SI / 4.0) + u * D_SIH)
    pos = np.vstack([si * (A_SI / 4.0), np.array(hs).reshape(-1, 3)])
    species = ["Si"] * n_si + ["H"] * len(hs)
    rs = np.random.default_rng(seed)
    pos = pos + rs.uniform(-jitter, jitter, size=pos.shape)
    return species, pos


def cluster_model(species, pos, n=64, h=0.5, ecut=28.0, params=None,
                  name="cluster"):
    """Local potential and KB projector list for a cluster centred in the
    box.  Returns a System with n_occ = (number of projectors) / 2."""
    params = SPECIES if params is None else params
    g = GridSpec(n, h)
    L = g.L
    pos = np.asarray(pos, dtype=np.float64) + 0.5 * L
    v = np.zeros((n, n, n))                  # [z][y][x]
    l, m, rc, ekb, begin = [], [], [], [], [0]
    for sp_, R in zip(species, pos):
        prm = params[sp_]
        # each well on the periodic grid points within 8 widths of its atom
        # (the tail left out is below 1e-13 of the depth)
        reach = int(np.ceil(8.0 * prm["s"] / h))
        ax = []
        for a in range(3):
            c = int(np.floor(R[a] / h))
            idx = np.arange(c - reach, c + reach + 2)
            if idx.size >= n:
                idx = np.arange(n)
            d = _min_image(idx * h - R[a], L) if idx.size == n else idx * h - R[a]
            ax.append((np.mod(idx, n), d))
        (ix, dx), (iy, dy), (iz, dz) = ax
        d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        v[np.ix_(iz, iy, ix)] -= prm["A"] * np.exp(-d2 / (2.0 * prm["s"] ** 2))
        l.append(0); m.append(0); rc.append(prm["rc"]); ekb.append(prm["e_s"])
        if prm["e_p"] is not None:
            for a in range(3):
                l.append(1); m.append(a); rc.append(prm["rc"]); ekb.append(prm["e_p"])
        begin.append(len(l))
    v = v.ravel()
    proj = ProjectorSpec(pos=pos, proj_begin=np.array(begin, dtype=np.int32),
                         l=np.array(l, dtype=np.int32), m=np.array(m, dtype=np.int32),
                         rc=np.array(rc, dtype=np.float64),
                         ekb=np.array(ekb, dtype=np.float64))
    nel = sum(params[s]["zval"] for s in species)
    return System(name, g, v, proj, n_occ=nel // 2, ecut=ecut,
                  species=list(species), pos=pos)


def si35h36(seed=1002, n=64, h=0.5, ecut=28.0):
    species, pos = si_cluster(35, seed=seed)
    return cluster_model(species, pos, n=n, h=h, ecut=ecut, name="Si35H36")


def si357h204(seed=1003, n=128, h=0.6, ecut=28.0):
    """Stand-in for the Si353H196 cluster on a 128^3 grid (h = 0.6 bohr):
    357 Si atoms is the atom-centred shell closure nearest 353; 204 H caps,
    1632 projectors, 816 occupied states."""
    species, pos = si_cluster(357, seed=seed)
    return cluster_model(species, pos, n=n, h=h, ecut=ecut, name="Si357H204")


SHELLS = (5, 17, 29, 35, 47, 71, 87, 99, 123, 147)     # atom-centred shell closures
BATCH_SIZES = (40, 48, 56, 64, 80, 96, 112)            # FFT lengths for the uneven batch


def si705h300(seed=1006, n=160, h=0.6, ecut=28.0):
    """The Si705H300-shaped cluster (705 Si, 300 H caps: 3120 projectors,
    1560 occupied states) on a 160^3 grid (h = 0.6 bohr)."""
    species, pos = si_cluster(705, seed=seed)
    return cluster_model(species, pos, n=n, h=h, ecut=ecut, name="Si705H300")


def uneven_batch(count=32, seed=1004, h=0.6, margin=8.0, ecut=28.0):
    """Uneven batch of H-capped Si clusters: for each of ``count`` clusters a
    seeded shell size from SHELLS (5 to 147 Si), its own jitter seed, the
    smallest grid in BATCH_SIZES whose box holds the cluster with ``margin``
    bohr on every side (at most 112^3), and a seeded number of stochastic
    orbitals from (16, 32, 64, 128).  Returns a list of (System, n_eta)."""
    rs = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n_si = int(SHELLS[rs.integers(len(SHELLS))])
        species, pos = si_cluster(n_si, seed=seed + 1 + i)
        radius = float(np.max(np.linalg.norm(pos, axis=1)))
        n = next((m for m in BATCH_SIZES if m * h >= 2 * (radius + margin)), BATCH_SIZES[-1])
        neta = int((16, 32, 64, 128)[rs.integers(4)])
        out.append((cluster_model(species, pos, n=n, h=h, ecut=ecut,
                                  name=f"Si{n_si}H{species.count('H')}"), neta))
    return out


def uneven_batch_spread(count=32, seed=1005, h=0.6, margin=4.0, ecut=28.0,
                        shells=(17, 29, 35, 47, 71, 87, 99, 123, 147)):
    """Uneven batch spanning the grid range: for each of ``count`` clusters a
    grid drawn uniformly from BATCH_SIZES (40^3 ... 112^3), a seeded shell
    size from ``shells`` (17 to 147 Si) among those whose cluster the box
    holds with ``margin`` bohr on every side, its own jitter seed, and a
    seeded number of stochastic orbitals from (16, 32, 64, 128).  Returns a
    list of (System, n_eta)."""
    rs = np.random.default_rng(seed)
    radius = {}
    for n_si in shells:
        _, pos = si_cluster(n_si, seed=0)
        radius[n_si] = float(np.max(np.linalg.norm(pos, axis=1))) + 0.1   # + jitter
    out = []
    for i in range(count):
        n = int(BATCH_SIZES[rs.integers(len(BATCH_SIZES))])
        fits = [k for k in shells if n * h >= 2 * (radius[k] + margin)] or [shells[0]]
        n_si = int(fits[rs.integers(len(fits))])
        species, pos = si_cluster(n_si, seed=seed + 1 + i)
        neta = int((16, 32, 64, 128)[rs.integers(4)])
        out.append((cluster_model(species, pos, n=n, h=h, ecut=ecut,
                                  name=f"Si{n_si}H{species.count('H')}"), neta))
    return out


def tiny_system(n=8, h=0.7, with_kb=True, n_occ=2):
    """Small periodic test system (8^3 or 12^3 points): two Gaussian wells
    and, optionally, one s and one p_x KB projector."""
    g = GridSpec(n, h)
    L = g.L
    centres = np.array([[L / 3, L / 2 + 0.11, L / 2 - 0.07],
                        [2 * L / 3, L / 2 - 0.05, L / 2 + 0.13]])
    r = grid_coords(g)
    v = np.zeros(g.N)
    for c in centres:
        d = _min_image(r - c, L)
        v -= 3.0 * np.exp(-np.sum(d * d, axis=1) / (2.0 * 0.8 ** 2))
    proj = None
    if with_kb:
        proj = ProjectorSpec(pos=centres, proj_begin=np.array([0, 1, 2], dtype=np.int32),
                             l=np.array([0, 1], dtype=np.int32),
                             m=np.array([0, 0], dtype=np.int32),
                             rc=np.array([0.75, 0.8]), ekb=np.array([-1.5, 0.8]),
                             rcut_over_rc=3.0)
    return System("tiny", g, v, proj, n_occ=n_occ, pos=centres)


# ------------------------------------------------------------------ MLP inputs
MLP_SIZES = (64, 256, 256)          # features -> hidden -> hidden (-> 1)


def mlp_param_count(din=64, h1=256, h2=256):
    return h1 * din + h1 + h2 * h1 + h2 + h2 + 1


def mlp_init(seed=7, din=64, h1=256, h2=256):
    """Seeded initial parameters of the control-variate network, packed as
    W1 [h1][din], b1 [h1], W2 [h2][h1], b2 [h2], w3 [h2], b3 (FP64): uniform
    +-sqrt(6 / (fan_in + fan_out)) weights (Glorot), zero biases."""
    rs = np.random.default_rng(seed)

    def glorot(fo, fi):
        a = np.sqrt(6.0 / (fi + fo))
        return rs.uniform(-a, a, size=(fo, fi))

    parts = [glorot(h1, din).ravel(), np.zeros(h1), glorot(h2, h1).ravel(), np.zeros(h2),
             glorot(1, h2).ravel(), np.zeros(1)]
    return np.concatenate(parts)
