"""Quasi-1D mode (paper Sec. 3.1, quasi-1D item): states are
phi(z) exp(i (k_x x + k_y y)) / sqrt(L_x L_y), so each transverse momentum
k_perp gives an independent BdG problem on the z lattice with
mu -> mu - k_perp^2 / 2 (A = 1), and the densities carry the factor
1/(L_x L_y) and the extra k_perp^2 |v|^2 term in tau.

States of all problems are one flat batch of shape (n, 2, N_z); every state
carries its own k_perp^2.  The free directions are called x and y here, the
lattice axis z (the paper keeps x and puts the plane waves on y, z; the
labels do not matter).

Part of the oracle: test infrastructure only (tests, the smoke check and
the benchmark's CPU baseline use it; the product path never does).
"""
import numpy as np

from . import lattice as L
from . import densities as D


class GeometryQ1D:
    def __init__(self, nz, dz, nkx, nky, dperp):
        self.nz, self.dz = int(nz), float(dz)
        self.shape = (self.nz,)
        self.kz = L.kgrid(self.nz, self.dz)
        self.Lx = nkx * dperp
        self.Ly = nky * dperp
        self.kx = L.kgrid(nkx, dperp)
        self.ky = L.kgrid(nky, dperp)
        self.area = self.Lx * self.Ly
        self.dV = self.dz
        self.dV_energy = self.dz * self.area
        self.kperp2 = None  # per state, set by set_states

    def problems(self):
        """(k_perp^2, (ix, iy)) of every transverse momentum, x index slow."""
        out = []
        for ix, kx in enumerate(self.kx):
            for iy, ky in enumerate(self.ky):
                out.append((kx * kx + ky * ky, (ix, iy)))
        return out

    def set_states(self, kperp2):
        self.kperp2 = np.asarray(kperp2, float)

    def _lap(self, f):
        return L.spectral_derivative(f, self.kz, f.ndim - 1, 2)

    def apply_h(self, phi, hfield, delta, alpha=None, avec=None):
        """H of every problem.  With alpha / avec (the A != 1 functional,
        Eq. h_sigma) the z kinetic part takes the symmetrised form of Eq.
        kinop-alpha, the transverse plane waves add 1/2 alpha k_perp^2 (the
        paper's mu -> mu - 1/2 alpha k_perp^2 of the quasi-1D item), and the
        current term is -(i/2) {A_z, d_z} with D1 (Nyquist zeroed); the
        transverse components of A vanish (j_perp cancels between +k_perp and
        -k_perp)."""
        u, v = phi[:, 0], phi[:, 1]
        if alpha is None and avec is None:
            off = 0.5 * self.kperp2[:, None]
            hu = -0.5 * self._lap(u) + (hfield + off) * u + delta * v
            hv = np.conj(delta) * u - (-0.5 * self._lap(v) + (hfield + off) * v)
            return np.stack([hu, hv], axis=1)
        al = np.broadcast_to(np.asarray(1.0 if alpha is None else alpha, float), self.shape)
        off = 0.5 * al[None, :] * self.kperp2[:, None]
        lap_a = self._lap(al.astype(complex))

        def kin(f):
            return -0.25 * (self._lap(al * f) + al * self._lap(f) - f * lap_a) + off * f

        def cur(f):
            if avec is None:
                return 0.0
            az = avec[2]
            d1 = L.spectral_derivative(f, self.kz, f.ndim - 1, 1)
            d1a = L.spectral_derivative(az * f, self.kz, f.ndim - 1, 1)
            return -0.5j * (az * d1 + d1a)
        hu = kin(u) + hfield * u + cur(u) + delta * v
        hv = np.conj(delta) * u - (kin(v) + hfield * v) + cur(v)
        return np.stack([hu, hv], axis=1)

    def rho_nu_j(self, phi, wu, wv):
        rho, _, nu, j = self.full_densities(phi, wu, wv)
        return rho, nu, j

    def _gsq(self, f, dzf):
        """|d_z f|^2 in the symmetric-Nyquist convention of the 3D densities."""
        sgn = (-1.0) ** np.arange(self.nz)
        c = np.sum(sgn * f, axis=-1, keepdims=True) / self.nz
        return np.abs(dzf) ** 2 + (np.pi / self.dz) ** 2 * np.abs(c) ** 2

    def rho_nu(self, phi, wu, wv):
        rho, nu = D.local_densities(phi, wu, wv)
        return rho / self.area, nu / self.area

    def full_densities(self, phi, wu, wv):
        wu = np.asarray(wu, float)[:, None]
        wv = np.asarray(wv, float)[:, None]
        u, v = phi[:, 0], phi[:, 1]
        kp = self.kperp2[:, None]
        rho, nu = self.rho_nu(phi, wu[:, 0], wv[:, 0])
        dzu = L.spectral_derivative(u, self.kz, 1, 1, zero_nyquist=True)
        dzv = L.spectral_derivative(v, self.kz, 1, 1, zero_nyquist=True)
        tau = np.sum(wv * (kp * np.abs(v) ** 2 + self._gsq(v, dzv))
                     + wu * (kp * np.abs(u) ** 2 + self._gsq(u, dzu)), axis=0) / self.area
        jz = np.sum(wv * np.imag(v * np.conj(dzv)) - wu * np.imag(u * np.conj(dzu)), axis=0) / self.area
        zero = np.zeros(self.nz)
        return rho, tau, nu, [zero, zero.copy(), jz]


    def friction_sources(self, phi, wu, wv):
        """What the dissipative fields of the quantum-friction evolution
        need (Sec. 5.2, correcting the initial state by a time-dependent
        approach), in this geometry (fields depend on z only):
          div j = d_z j_z (D1 with the Nyquist mode zeroed, as j itself),
          B'    = -1/2 sum_n (f_v - f_u) [u grad^2 v^* + v^* grad^2 u] / (L_x L_y)
                  with grad^2 = D2z - k_perp^2 and the weights of nu,
          N     = int rho_+ d^3r.
        Returns (div_j, B', N)."""
        rho, _, _, j = self.full_densities(phi, wu, wv)
        div_j = np.real(L.spectral_derivative(j[2], self.kz, 0, 1))
        u, v = phi[:, 0], phi[:, 1]
        kp = self.kperp2[:, None]
        lu = self._lap(u) - kp * u
        lv = self._lap(v) - kp * v
        w = (np.asarray(wv, float) - np.asarray(wu, float))[:, None]
        Bp = -0.5 * np.sum(w * (u * np.conj(lv) + np.conj(v) * lu), axis=0) / self.area
        N = self.dV_energy * np.sum(2.0 * rho)
        return div_j, Bp, N


def dense_h_1d(hfield, delta, nz, dz, kperp2):
    """2N_z x 2N_z BdG matrix of one problem (Eq. D2 along z)."""
    K = -0.5 * L.d2_matrix(nz, dz)
    h = K + np.diag(hfield + 0.5 * kperp2)
    d = np.diag(delta)
    return np.block([[h, d], [np.conj(d), -h]])


def eigenstates(geom, hfield, delta, ec=None, positive_only=True):
    """Diagonalise every problem; keep E > 0 (spin-symmetric half) and
    |E| < ec.  Returns (E, kperp2, problem_index, phi) with phi of shape
    (n, 2, N_z) normalised to int (|u|^2 + |v|^2) dz = 1."""
    Es, kps, pid, phis = [], [], [], []
    for ip, (kp2, _) in enumerate(geom.problems()):
        H = dense_h_1d(hfield, delta, geom.nz, geom.dz, kp2)
        E, W = np.linalg.eigh(H)
        keep = np.ones(E.shape, bool)
        if positive_only:
            keep &= E > 0
        if ec is not None:
            keep &= np.abs(E) < ec
        sel = np.nonzero(keep)[0]
        if sel.size == 0:
            continue
        Es.append(E[sel])
        kps.append(np.full(sel.size, kp2))
        pid.append(np.full(sel.size, ip))
        phis.append(W[:, sel].T.reshape(sel.size, 2, geom.nz) / np.sqrt(geom.dz))
    return (np.concatenate(Es), np.concatenate(kps), np.concatenate(pid),
            np.concatenate(phis, axis=0))
