"""Sparse stochastic basis {xi_{i,m}} for u^R (oracle side).

Sec. 2.1: instead of storing u^R(r, t) on the full grid, it is projected on
N_xi random functions living on short, fragmented segments of the grid and
accumulated in that basis.  Sec. 2.2: the cost of the accumulation is
O(N_zeta N_xi N_tau N_g f_g), f_g being the fraction of the grid each xi
covers; Sec. 2.3: the segments have length L = 32.

Readings (the construction is in the paper's references, not its text):
* xi_m covers n_seg = max(1, floor(f_g N_g / 32 + 1/2)) segments of 32
  consecutive flat grid indices, aligned to multiples of 32.  N_g must be a
  multiple of 32 (nblocks = N_g / 32 aligned blocks).
* Segment s of xi_m starts at block b = word(seed, XI_SUPPORT stream of the
  sample, m * n_seg + s) mod nblocks; a block already used by xi_m is replaced
  by the next free block (b + 1 mod nblocks, ...), which keeps every block's
  marginal probability equal.
* Point p (0..31) of segment s has the sign given by bit p of
  word(seed, XI_SIGN stream of the sample, m * n_seg + s): 0 -> +, 1 -> -.
* Values are +-1/sqrt(N_xi f_g' dV), f_g' = 32 n_seg / N_g, so that
  E[sum_m |xi_m><xi_m|] is the identity, i.e. u = sum_m xi_m <xi_m|u>
  in expectation.
* A fresh set per Monte Carlo sample.
"""
import numpy as np

from . import rng

SEG = 32


def n_segments(N, f_g):
    return max(1, int(np.floor(f_g * N / SEG + 0.5)))


def amplitude(N, n_xi, f_g, dV):
    nseg = n_segments(N, f_g)
    fgp = SEG * nseg / N
    return 1.0 / np.sqrt(n_xi * fgp * dV)


def supports(seed, sample, N, n_xi, f_g):
    """(n_xi, n_seg) array of aligned block indices."""
    if N % SEG:
        raise ValueError("grid size must be a multiple of 32")
    nblocks = N // SEG
    nseg = n_segments(N, f_g)
    if nseg > nblocks:
        raise ValueError("f_g too large")
    st = rng.stream_id(rng.XI_SUPPORT, sample)
    w = rng.words(seed, st, np.arange(n_xi * nseg, dtype=np.uint64))
    draws = (w % np.uint64(nblocks)).astype(np.int64).reshape(n_xi, nseg)
    out = np.empty_like(draws)
    for m in range(n_xi):
        used = set()
        for s in range(nseg):
            b = int(draws[m, s])
            while b in used:
                b = (b + 1) % nblocks
            used.add(b)
            out[m, s] = b
    return out


def signs(seed, sample, n_xi, nseg):
    """(n_xi, n_seg, 32) array of +-1."""
    st = rng.stream_id(rng.XI_SIGN, sample)
    w = rng.words(seed, st, np.arange(n_xi * nseg, dtype=np.uint64))
    p = np.arange(SEG, dtype=np.uint64)
    bits = (w[:, None] >> p[None, :]) & np.uint64(1)
    return (1.0 - 2.0 * bits.astype(np.float64)).reshape(n_xi, nseg, SEG)


class XiBasis:
    """The xi functions of one sample as (index, value) lists."""

    def __init__(self, seed, sample, N, n_xi, f_g, dV):
        self.N, self.n_xi, self.dV = N, n_xi, dV
        self.nseg = n_segments(N, f_g)
        blocks = supports(seed, sample, N, n_xi, f_g)
        self.idx = (blocks[:, :, None] * SEG
                    + np.arange(SEG)[None, None, :]).reshape(n_xi, -1)
        amp = amplitude(N, n_xi, f_g, dV)
        self.val = amp * signs(seed, sample, n_xi, self.nseg).reshape(n_xi, -1)

    def overlaps(self, f):
        """<xi_m|f> = dV sum_r xi_m(r) f(r) for a grid function f (N,)."""
        return self.dV * np.sum(self.val * f[self.idx], axis=1)

    def dense(self):
        """Dense (n_xi, N) matrix (small grids only)."""
        X = np.zeros((self.n_xi, self.N))
        rows = np.repeat(np.arange(self.n_xi), self.idx.shape[1])
        np.add.at(X, (rows, self.idx.ravel()), self.val.ravel())
        return X
