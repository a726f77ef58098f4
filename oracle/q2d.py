"""Quasi-2D time-dependent mode (paper Sec. 3.1, quasi-2D item): states are
phi(x, y) exp(i k_z z) / sqrt(L_z) on an N_x x N_y lattice, so each k_z gives
an independent BdG problem on the x-y lattice with mu -> mu - k_z^2 / 2
(A = 1), and the densities carry 1 / L_z and the extra k_z^2 |v|^2 term in
tau; j_z cancels between +k_z and -k_z.  Problems with the same |k_z| are
equal: one of them is evolved and its states carry the multiplicity in
their weights (1 for k_z = 0 and the Nyquist momentum, 2 otherwise).

States of all problems are one flat batch of shape (n, 2, N_x, N_y); every
state carries its own k_z^2.

Part of the oracle: test infrastructure only (tests, the smoke check and
the benchmark's CPU baseline use it; the product path never does).
"""
import numpy as np

from . import lattice as L
from . import densities as D
from . import static as ST


class GeometryQ2D:
    def __init__(self, nx, ny, nz, dx=1.0, dy=1.0, dz=1.0):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy, self.dz = float(dx), float(dy), float(dz)
        self.shape = (self.nx, self.ny)
        self.k = (L.kgrid(self.nx, self.dx), L.kgrid(self.ny, self.dy))
        self.Lz = self.nz * self.dz
        self.dV = self.dx * self.dy          # state normalisation
        self.dV_energy = self.dV * self.Lz   # energy / particle-number integrals
        self.kz2 = None                      # per state, set by set_states
        self.static = ST.GeometryQ2D(nx, ny, nz, dx, dy, dz)

    def classes(self):
        """(|k_z|, multiplicity) of the distinct problems."""
        return list(zip(self.static.kz, self.static.mult))

    def set_states(self, kz2):
        self.kz2 = np.asarray(kz2, float)

    def _lap(self, f):
        ax = (f.ndim - 2, f.ndim - 1)
        k2 = self.k[0][:, None] ** 2 + self.k[1][None, :] ** 2
        return np.fft.ifft2(-k2 * np.fft.fft2(f, axes=ax), axes=ax)

    def apply_h(self, phi, hfield, delta, alpha=None, avec=None):
        """H of every problem (A = 1: -1/2 of the 2D lattice Laplacian
        plus k_z^2 / 2 on the diagonal blocks)."""
        if alpha is not None or avec is not None:
            raise NotImplementedError("the quasi-2D mode is written for the A = 1 functional")
        u, v = phi[:, 0], phi[:, 1]
        off = 0.5 * self.kz2[:, None, None]
        hu = -0.5 * self._lap(u) + (hfield + off) * u + delta * v
        hv = np.conj(delta) * u - (-0.5 * self._lap(v) + (hfield + off) * v)
        return np.stack([hu, hv], axis=1)

    def rho_nu(self, phi, wu, wv):
        rho, nu = D.local_densities(phi, wu, wv)
        return rho / self.Lz, nu / self.Lz

    def _grad_sq(self, f, axis):
        """|d f|^2 along one lattice axis in the symmetric-Nyquist
        convention of the 3D densities, and D1 f (Nyquist zeroed)."""
        d1 = L.spectral_derivative(f, self.k[axis], f.ndim - 2 + axis, 1, zero_nyquist=True)
        n = f.shape[f.ndim - 2 + axis]
        shp = [1] * f.ndim
        shp[f.ndim - 2 + axis] = n
        sgn = ((-1.0) ** np.arange(n)).reshape(shp)
        c = np.sum(sgn * f, axis=f.ndim - 2 + axis, keepdims=True) / n
        d = (self.dx, self.dy)[axis]
        return np.abs(d1) ** 2 + (np.pi / d) ** 2 * np.abs(c) ** 2, d1

    def full_densities(self, phi, wu, wv):
        wu = np.asarray(wu, float)[:, None, None]
        wv = np.asarray(wv, float)[:, None, None]
        u, v = phi[:, 0], phi[:, 1]
        kz2 = self.kz2[:, None, None]
        rho, nu = self.rho_nu(phi, wu[:, 0, 0], wv[:, 0, 0])
        tau = np.sum(kz2 * (wv * np.abs(v) ** 2 + wu * np.abs(u) ** 2), axis=0)
        j = []
        for a in range(2):
            gu, du = self._grad_sq(u, a)
            gv, dv = self._grad_sq(v, a)
            tau = tau + np.sum(wv * gv + wu * gu, axis=0)
            j.append(np.sum(wv * np.imag(v * np.conj(dv)) - wu * np.imag(u * np.conj(du)), axis=0) / self.Lz)
        j.append(np.zeros(self.shape))
        return rho, tau / self.Lz, nu, j


def eigenstates(geom, hfield, delta, ec=None):
    """Diagonalise every |k_z| class (the dense matrices of the static
    oracle); keep 0 < E < ec.  Returns (E, kz2, multiplicity, phi) with phi
    of shape (n, 2, N_x, N_y) normalised to int (|u|^2 + |v|^2) dx dy = 1."""
    Es, kz2s, ms, phis = [], [], [], []
    M = geom.nx * geom.ny
    for kz, w in geom.classes():
        E, W = np.linalg.eigh(ST.build_h(geom.static, hfield, delta, kz))
        keep = E > 0
        if ec is not None:
            keep &= E < ec
        sel = np.nonzero(keep)[0]
        if sel.size == 0:
            continue
        Es.append(E[sel])
        kz2s.append(np.full(sel.size, kz * kz))
        ms.append(np.full(sel.size, w))
        phis.append(W[:, sel].T.reshape(sel.size, 2, geom.nx, geom.ny) / np.sqrt(geom.dV))
    return np.concatenate(Es), np.concatenate(kz2s), np.concatenate(ms), np.concatenate(phis, axis=0)


def plane_wave_states(geom, kidx, hshift, delta0):
    """Uniform-system start (Sec. 4.5.1) of the quasi-2D mode: for kidx[n] =
    (l_x, l_y, m) the x-y lattice momentum (k_x, k_y) of grid indices l_x,
    l_y and the |k_z| class m, xi = (k_x^2 + k_y^2 + k_z^2)/2 + hshift,
    E = sqrt(xi^2 + |Delta|^2), u = sqrt((1 + xi/E)/2), v = sqrt((1 - xi/E)/2)
    Delta^*/|Delta|, times exp(i (k_x x + k_y y)) / sqrt(L_x L_y) with x, y
    measured from the lattice corner.  Returns (E, k_z^2, multiplicity, phi)."""
    kidx = np.asarray(kidx)
    kx = geom.k[0][kidx[:, 0]]
    ky = geom.k[1][kidx[:, 1]]
    kz = geom.static.kz[kidx[:, 2]]
    xi = 0.5 * (kx ** 2 + ky ** 2 + kz ** 2) + hshift
    ad = abs(delta0)
    E = np.sqrt(xi ** 2 + ad ** 2)
    uk = np.sqrt(0.5 * (1.0 + xi / E))
    vk = np.sqrt(0.5 * (1.0 - xi / E)) * (np.conj(delta0) / ad)
    x = np.arange(geom.nx) * geom.dx
    y = np.arange(geom.ny) * geom.dy
    ph = np.exp(1j * (kx[:, None, None] * x[None, :, None] + ky[:, None, None] * y[None, None, :]))
    ph = ph / np.sqrt(geom.nx * geom.dx * geom.ny * geom.dy)
    phi = np.stack([uk[:, None, None] * ph, vk[:, None, None] * ph], axis=1)
    return E, kz ** 2, geom.static.mult[kidx[:, 2]], phi

