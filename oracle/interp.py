"""Fourier interpolation between periodic lattices of the same box (test
infrastructure: only tests/, the smoke check and the benchmark's CPU leg use
the oracle).

Sec. 5.2, refining lattice resolution: a field stored on an N_x x N_y
lattice is evaluated at any point as
    f(x, y) = 1/(L_x L_y) sum_{l,m} f~_{lm} exp[i (k_l x + k_m y)],
with f~ the lattice Fourier coefficients (an FFT) and the k grid of Sec. 3.1
(the Nyquist mode at -pi/d); at a lattice point this is the inverse FFT and
returns the stored value.  Reading: positions are measured from the box
corner that both lattices share (site j of either lattice sits at j d), and
a real field takes the real part of the sum.  The sum is evaluated directly,
point by point, as the paper describes.
"""
import numpy as np

from . import lattice as L


def coefficients(f, dx, dy):
    """f~_{lm} = dx dy sum_{ij} f_ij exp[-i (k_l x_i + k_m y_j)], x_i = i dx."""
    return dx * dy * np.fft.fft2(np.asarray(f, float))


def evaluate(ft, dx, dy, x, y):
    """The interpolant at the points (x, y) (arrays of one shape, measured
    from the box corner), real part."""
    nx, ny = ft.shape
    kx, ky = L.kgrid(nx, dx), L.kgrid(ny, dy)
    Lx, Ly = nx * dx, ny * dy
    ex = np.exp(1j * np.multiply.outer(np.ravel(x), kx))  # [P, nx]
    ey = np.exp(1j * np.multiply.outer(np.ravel(y), ky))  # [P, ny]
    val = np.einsum("pl,lm,pm->p", ex, ft, ey) / (Lx * Ly)
    return np.real(val).reshape(np.shape(x))


def to_lattice(f, dx, dy, nx2, ny2, dx2, dy2):
    """f from an nx x ny lattice (spacings dx, dy) onto an nx2 x ny2 lattice
    (spacings dx2, dy2) of the same box."""
    ft = coefficients(f, dx, dy)
    X, Y = np.meshgrid(np.arange(nx2) * dx2, np.arange(ny2) * dy2, indexing="ij")
    return evaluate(ft, dx, dy, X, Y)
