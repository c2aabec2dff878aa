"""Periodic real-space Fourier grid (oracle side).

The paper applies H on a uniform grid where FFT pairs switch between the
position representation (potential diagonal) and the momentum representation
(kinetic energy diagonal), Sec. 2.2 and Eq. (1).

Conventions (reading; the paper states none):
* points r = h * (ix, iy, iz), box L = n * h, periodic;
* flat index i = ix + nx * (iy + ny * iz)  (x fastest);
* k = 2 pi m / L with m in numpy ``fftfreq`` order, the Nyquist index being
  -n/2, so T(k) is even in k and H stays real-symmetric;
* forward FFT unnormalised, inverse FFT carries 1/N;
* dV = h^3 and <f|g> = dV * sum(conj(f) * g).
"""
import numpy as np
import scipy.fft as sfft


class Grid:
    def __init__(self, nx, ny=None, nz=None, h=0.5, workers=None):
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        self.n = (int(nx), int(ny), int(nz))
        self.h = float(h)
        self.N = int(nx) * int(ny) * int(nz)
        self.dV = self.h ** 3
        self.L = tuple(m * self.h for m in self.n)
        self.shape3 = (int(nz), int(ny), int(nx))
        self.workers = workers

    # ---- coordinates ---------------------------------------------------
    def coords(self):
        """(N, 3) array of point positions, x fastest."""
        nx, ny, nz = self.n
        iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                                 indexing="ij")
        return self.h * np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)

    def min_image(self, d):
        """Wrap displacement vectors (..., 3) into [-L/2, L/2)."""
        L = np.asarray(self.L)
        return np.mod(d + 0.5 * L, L) - 0.5 * L

    def kvecs(self):
        """Per-axis wave numbers kx (nx,), ky (ny,), kz (nz,)."""
        return tuple(2.0 * np.pi * np.fft.fftfreq(m, d=self.h) for m in self.n)

    def k2(self):
        """|k|^2 on the flat grid."""
        kx, ky, kz = self.kvecs()
        K2 = (kz[:, None, None] ** 2 + ky[None, :, None] ** 2
              + kx[None, None, :] ** 2)
        return K2.ravel()

    # ---- transforms ----------------------------------------------------
    def fft(self, f):
        """Unnormalised forward 3D FFT of (..., N) arrays."""
        f = np.asarray(f)
        s = f.shape[:-1] + self.shape3
        F = sfft.fftn(f.reshape(s), axes=(-3, -2, -1), workers=self.workers)
        return F.reshape(f.shape)

    def ifft(self, F):
        """Inverse 3D FFT (with 1/N) of (..., N) arrays."""
        F = np.asarray(F)
        s = F.shape[:-1] + self.shape3
        f = sfft.ifftn(F.reshape(s), axes=(-3, -2, -1), workers=self.workers)
        return f.reshape(F.shape)

    # ---- inner products -----------------------------------------------
    def dot(self, f, g):
        """<f|g> = dV sum conj(f) g over the last axis."""
        return self.dV * np.sum(np.conj(f) * g, axis=-1)

    def norm2(self, f):
        return np.real(self.dot(f, f))
