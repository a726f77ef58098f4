"""Periodic lattice, momentum grid and spectral derivatives (paper Sec. 3.1).

Units hbar = m = k_B = 1 (Sec. 2.1).  A function on an N_x x N_y x N_z mesh
is stored as a numpy array of that shape; the flat index order is
ixyz = (ix*N_y + iy)*N_z + iz (z fastest), which is numpy's C order.

Part of the oracle: test infrastructure only (tests, the smoke check and
the benchmark's CPU baseline use it; the product path never does).
"""
import numpy as np
import scipy.fft as sfft

_WORKERS = -1  # scipy.fft: use every host core


def kgrid(n, d):
    """Momenta of an n-point periodic axis with spacing d (Sec. 3.1, the
    definition of k_l): 2*pi*l/L for l < n/2, else 2*pi*(l-n)/L.  n is even,
    so l = n/2 (the Nyquist mode) carries the negative momentum -pi/d."""
    if n % 2:
        raise ValueError("lattice sizes are even")
    L = n * d
    l = np.arange(n)
    return 2.0 * np.pi / L * np.where(l < n // 2, l, l - n)


def centered_coords(n, d):
    """Physical coordinate of site l, x = (l - n/2)*d, the centred convention
    the paper's user code uses for external potentials."""
    return (np.arange(n) - n // 2) * float(d)


class Lattice:
    """A full 3D periodic box (Sec. 3.1)."""

    def __init__(self, nx, ny, nz, dx=1.0, dy=1.0, dz=1.0):
        self.n = (int(nx), int(ny), int(nz))
        self.d = (float(dx), float(dy), float(dz))
        self.shape = self.n
        self.M = nx * ny * nz
        self.dV = dx * dy * dz
        self.V = self.M * self.dV
        self.k = [kgrid(ni, di) for ni, di in zip(self.n, self.d)]
        kx, ky, kz = np.meshgrid(*self.k, indexing="ij")
        self.k2 = kx ** 2 + ky ** 2 + kz ** 2

    def coords(self):
        """Centred coordinate arrays X, Y, Z of shape (nx, ny, nz)."""
        return np.meshgrid(*[centered_coords(ni, di) for ni, di in zip(self.n, self.d)],
                           indexing="ij")


def spectral_derivative(f, k, axis, order, zero_nyquist=None):
    """r-th derivative along one axis by Eq. derivative-spectral: FFT,
    multiply by (i k)^r, inverse FFT.  The paper zeroes the Nyquist mode for
    odd r; zero_nyquist overrides that choice (None = the paper's rule)."""
    if zero_nyquist is None:
        zero_nyquist = (order % 2 == 1)
    n = f.shape[axis]
    fac = (1j * k) ** order
    if zero_nyquist:
        fac = fac.copy()
        fac[n // 2] = 0.0
    shp = [1] * f.ndim
    shp[axis] = n
    ft = sfft.fft(f, axis=axis, workers=_WORKERS)
    return sfft.ifft(ft * fac.reshape(shp), axis=axis, workers=_WORKERS)


def laplacian(f, lat, batch_axes=0):
    """Spectral Laplacian of fields of shape (..., nx, ny, nz): the full
    -k^2 multiplier including the Nyquist mode, which is what D^(2) of
    Eq. D2 represents exactly."""
    axes = tuple(range(f.ndim - 3, f.ndim))
    ft = sfft.fftn(f, axes=axes, workers=_WORKERS)
    return sfft.ifftn(-lat.k2 * ft, axes=axes, workers=_WORKERS)


def gradient(f, lat, zero_nyquist):
    """Spectral gradient (three arrays) of fields of shape (..., nx, ny, nz).
    zero_nyquist selects the paper's odd-derivative rule (True) or the full
    i*k multiplier (False)."""
    out = []
    for a in range(3):
        axis = f.ndim - 3 + a
        out.append(spectral_derivative(f, lat.k[a], axis, 1, zero_nyquist=zero_nyquist))
    return out


def d1_matrix(n, d):
    """Dense first-derivative matrix of Eq. D1 for one axis (n even)."""
    L = n * d
    l = np.arange(n)
    diff = l[:, None] - l[None, :]
    D = np.zeros((n, n))
    off = diff != 0
    D[off] = (np.pi / L) * (-1.0) ** diff[off] / np.tan(np.pi * diff[off] / n)
    return D


def d2_matrix(n, d):
    """Dense second-derivative matrix of Eq. D2 for one axis (n even)."""
    L = n * d
    l = np.arange(n)
    diff = l[:, None] - l[None, :]
    D = np.zeros((n, n))
    off = diff != 0
    D[off] = (2.0 * np.pi ** 2 / L ** 2) * (-1.0) ** (diff[off] - 1) / np.sin(np.pi * diff[off] / n) ** 2
    D[~off] = -(np.pi ** 2 / (3.0 * d ** 2)) * (1.0 + 2.0 / n ** 2)
    return D


def dense_laplacian(lat):
    """M x M matrix of the Laplacian built from the Eq. D2 matrices of the
    three axes (Kronecker sum), independent of any FFT."""
    nx, ny, nz = lat.n
    Dx, Dy, Dz = (d2_matrix(n, d) for n, d in zip(lat.n, lat.d))
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(np.kron(Dx, Iy), Iz) + np.kron(np.kron(Ix, Dy), Iz)
            + np.kron(np.kron(Ix, Iy), Dz))
