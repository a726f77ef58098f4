"""Spin-imbalanced ASLDA (paper Sec. 2.4, ASLDA item; Sec. 2.3, Eqs.
HpsiEpsi, h_sigma, na3D-jb3D and the SLDA-type energy density) in the
quasi-1D and full 3D geometries.

Without spin symmetry both branches of the reduced problem are evolved
(states of either sign of E, no halving): a state is (u_a, v_b), the u row
carries h_a - mu_a and the v row -h_b^* + mu_b, and the densities are
spin-resolved,
    rho_a = sum_n f(E_n) |u_n|^2,      rho_b = sum_n f(-E_n) |v_n|^2,
    tau_a = sum_n f(E_n) |grad u_n|^2, tau_b = sum_n f(-E_n) |grad v_n|^2,
    nu    = 1/2 sum_n (f(-E_n) - f(E_n)) u_n v_n^*,
    j_a   = -sum_n f(E_n) Im(u_n grad u_n^*),  j_b = sum_n f(-E_n) Im(v_n grad v_n^*),
with the quasi-1D factor 1/(L_x L_y) and k_perp^2 in tau.  The functional
parameters depend on the local polarisation p = (rho_a - rho_b) / rho_+,
rho_+ = rho_a + rho_b: A_a(p) = A(p), A_b(p) = A(-p), B(p), C = -11.11.
The potentials are the functional derivatives of
    E = sum_s A_s/2 (tau_s - j_s^2/rho_s) + 3/5 B rho_+ eF(rho_+)
        + g_eff |nu|^2 + sum_s j_s^2 / (2 rho_s)
with the regulator frozen (1/g_eff = rho_+^(1/3)/C - Lambda_c).

Part of the oracle: test infrastructure only (tests, the smoke check and
the benchmark's CPU baseline use it; the product path never does).
"""
import numpy as np

from . import bdg
from . import densities as D
from . import functional as F
from . import lattice as L

C_ASLDA = F.C_SLDA
RHO_FLOOR = F.RHO_FLOOR


def A_of_p(p):
    return F.aslda_A(p)


def dA_dp(p):
    """Derivative of A(p) (the polynomial of the ASLDA item)."""
    return 0.156 * (1 - 2 * p ** 2 + p ** 4) - 0.532 * (2 * p - 4 * p ** 3 + 2 * p ** 5)


def B_of_p(p):
    return F.aslda_B(p)


def dB_dp(p):
    """Derivative of B(p) = 2^(2/3) [0.357 + 0.642 p^2 - A(p) ((1+p)/2)^(5/3)
    - A(-p) ((1-p)/2)^(5/3)]."""
    hp, hm = (1 + p) / 2, (1 - p) / 2
    return 2.0 ** (2.0 / 3.0) * (1.284 * p
                                 - dA_dp(p) * hp ** (5.0 / 3.0) - A_of_p(p) * (5.0 / 6.0) * hp ** (2.0 / 3.0)
                                 + dA_dp(-p) * hm ** (5.0 / 3.0) + A_of_p(-p) * (5.0 / 6.0) * hm ** (2.0 / 3.0))


def _prep(rho_a, rho_b):
    ra = np.maximum(rho_a, RHO_FLOOR / 2)
    rb = np.maximum(rho_b, RHO_FLOOR / 2)
    rp = ra + rb
    p = (ra - rb) / rp
    return ra, rb, rp, p


def energy_density(rho_a, rho_b, tau_a, tau_b, ja, jb, nu, lam):
    """The SLDA-type energy density (Eqs. sldae-functional-generic, -CM and
    the intrinsic part) with the ASLDA parameters; ja, jb: |j_s|^2-carrying
    arrays (one component per array in a list)."""
    ra, rb, rp, p = _prep(rho_a, rho_b)
    jsa = sum(np.abs(c) ** 2 for c in ja)
    jsb = sum(np.abs(c) ** 2 for c in jb)
    Aa, Ab, B = A_of_p(p), A_of_p(-p), B_of_p(p)
    g = 1.0 / (rp ** (1.0 / 3.0) / C_ASLDA - lam)
    return (0.5 * Aa * (tau_a - jsa / ra) + 0.5 * Ab * (tau_b - jsb / rb)
            + 0.6 * B * rp * F.eF(rp) + g * np.abs(nu) ** 2
            + jsa / (2 * ra) + jsb / (2 * rb))


def potentials(rho_a, rho_b, tau_a, tau_b, ja, jb, nu, lam):
    """Functional derivatives of energy_density (Sec. 2.3 list of
    potentials):
        alpha_s = 2 dE/dtau_s = A_s(p),
        A_s     = dE/dj_s     = (1 - A_s) j_s / rho_s,
        Delta   = -dE/dnu^*   = -g_eff nu,
        V_s     = dE/drho_s   = dp/drho_s [1/2 (A_a' K_a + A_b' K_b) + 3/5 B'(p) rho_+ eF]
                                + (A_s - 1) j_s^2 / (2 rho_s^2) + B eF - |Delta|^2 / (3 C rho_+^(2/3)),
    with K_s = tau_s - j_s^2 / rho_s, A_a' = A'(p), A_b' = -A'(-p),
    dp/drho_a = 2 rho_b / rho_+^2, dp/drho_b = -2 rho_a / rho_+^2.
    Returns (V_a, V_b, Delta, alpha_a, alpha_b, Avec_a, Avec_b) with the
    vector potentials as lists like ja, jb."""
    ra, rb, rp, p = _prep(rho_a, rho_b)
    jsa = sum(np.abs(c) ** 2 for c in ja)
    jsb = sum(np.abs(c) ** 2 for c in jb)
    Aa, Ab, B = A_of_p(p), A_of_p(-p), B_of_p(p)
    g = 1.0 / (rp ** (1.0 / 3.0) / C_ASLDA - lam)
    delta = -g * nu
    Ka, Kb = tau_a - jsa / ra, tau_b - jsb / rb
    common = 0.5 * (dA_dp(p) * Ka - dA_dp(-p) * Kb) + 0.6 * dB_dp(p) * rp * F.eF(rp)
    base = B * F.eF(rp) - np.abs(delta) ** 2 / (3.0 * C_ASLDA * rp ** (2.0 / 3.0))
    Va = 2 * rb / rp ** 2 * common + (Aa - 1) * jsa / (2 * ra ** 2) + base
    Vb = -2 * ra / rp ** 2 * common + (Ab - 1) * jsb / (2 * rb ** 2) + base
    Avec_a = [(1 - Aa) * c / ra for c in ja]
    Avec_b = [(1 - Ab) * c / rb for c in jb]
    return Va, Vb, delta, Aa, Ab, Avec_a, Avec_b


class SpinGeometryQ1D:
    """Quasi-1D geometry with spin-resolved densities and the two rows of
    the reduced problem carrying the fields of their own spin (built on the
    quasi-1D general operator, which is pinned against the 3D one)."""

    def __init__(self, base):
        self.base = base  # an oracle.q1d.GeometryQ1D
        self.shape = base.shape
        self.dV = base.dV
        self.dV_energy = base.dV_energy

    def set_states(self, kperp2):
        self.base.set_states(kperp2)

    def apply_h(self, phi, hf_a, hf_b, delta, al_a, al_b, av_a, av_b):
        """u row: h_a u (hf_a = V_a + V_ext - mu_a) + Delta v;
        v row: Delta^* u - h_b^* v (hf_b = V_b + V_ext - mu_b); each h with
        its own alpha_s and A_s (av_s: [A_s,z])."""
        ha = self.base.apply_h(phi, hf_a, delta, al_a, [0, 0, av_a[0]])
        hb = self.base.apply_h(phi, hf_b, delta, al_b, [0, 0, av_b[0]])
        return np.stack([ha[:, 0], hb[:, 1]], axis=1)

    def densities(self, phi, wu, wv, tau_form="gradient"):
        """(rho_a, rho_b, tau_a, tau_b, nu, j_a, j_b) of Eqs. na3D-jb3D
        (quasi-1D: 1/(L_x L_y), k_perp^2 in tau, j along z).

        tau_form = "gradient": tau_s = |D1 f|^2 with the Nyquist amplitude
        at full weight (the paper's |grad f|^2, as in the 3D densities).
        tau_form = "laplacian": tau_s = -Re(f^* D2 f) + 1/2 D2 |f|^2, the
        density whose integral against any alpha(z) is the expectation of
        the symmetrised kinetic operator of Eq. kinop-alpha; with it the
        energy is the exact generator of the evolution (used to pin the
        assembly); the two agree in the continuum and differ on the lattice
        where alpha varies."""
        g = self.base
        if tau_form == "laplacian":
            wu_ = np.asarray(wu, float)[:, None]
            wv_ = np.asarray(wv, float)[:, None]
            u, v = phi[:, 0], phi[:, 1]
            kp = g.kperp2[:, None]

            def t(f):
                return (-np.real(np.conj(f) * g._lap(f)) + 0.5 * np.real(g._lap(np.abs(f) ** 2 + 0j))
                        + kp * np.abs(f) ** 2)
            out = list(self.densities(phi, wu, wv))
            out[2] = np.sum(wu_ * t(u), axis=0) / g.area
            out[3] = np.sum(wv_ * t(v), axis=0) / g.area
            return tuple(out)
        wu = np.asarray(wu, float)[:, None]
        wv = np.asarray(wv, float)[:, None]
        u, v = phi[:, 0], phi[:, 1]
        kp = g.kperp2[:, None]
        du = L.spectral_derivative(u, g.kz, 1, 1, zero_nyquist=True)
        dv = L.spectral_derivative(v, g.kz, 1, 1, zero_nyquist=True)
        a = g.area
        rho_a = np.sum(wu * np.abs(u) ** 2, axis=0) / a
        rho_b = np.sum(wv * np.abs(v) ** 2, axis=0) / a
        tau_a = np.sum(wu * (kp * np.abs(u) ** 2 + g._gsq(u, du)), axis=0) / a
        tau_b = np.sum(wv * (kp * np.abs(v) ** 2 + g._gsq(v, dv)), axis=0) / a
        nu = 0.5 * np.sum((wv - wu) * u * np.conj(v), axis=0) / a
        ja = -np.sum(wu * np.imag(u * np.conj(du)), axis=0) / a
        jb = np.sum(wv * np.imag(v * np.conj(dv)), axis=0) / a
        return rho_a, rho_b, tau_a, tau_b, nu, ja, jb


class SpinGeometry3D:
    """Full 3D lattice with the spin-resolved densities of Eqs. na3D-jb3D
    (oracle.densities.general) and the rows of the reduced problem carrying
    their own spin's fields (the 3D general operator, oracle.bdg)."""

    def __init__(self, lat):
        self.lat = lat
        self.shape = lat.shape
        self.dV = lat.dV
        self.dV_energy = lat.dV

    def apply_h(self, phi, hf_a, hf_b, delta, al_a, al_b, av_a, av_b):
        ha = bdg.apply_h_general(phi, hf_a, delta, al_a, av_a, self.lat)
        hb = bdg.apply_h_general(phi, hf_b, delta, al_b, av_b, self.lat)
        return np.stack([ha[:, 0], hb[:, 1]], axis=1)

    def densities(self, phi, wu, wv, tau_form="gradient"):
        if tau_form != "gradient":
            raise NotImplementedError("the 3D geometry takes the paper's gradient form of tau")
        d = D.general(phi, wu, wv, self.lat)
        return d["rho_a"], d["rho_b"], d["tau_a"], d["tau_b"], d["nu"], d["j_a"], d["j_b"]


def _as_list(j):
    return j if isinstance(j, list) else [j]


class ASLDASystem:
    """What the right-hand side needs (the TDSystem interface of td.py):
    mu_a, mu_b fixed, vext static, lam the frozen regulator, wu, wv the
    frozen weights f(E_n), f(-E_n) of states of both signs of E."""

    def __init__(self, geom, mu_a, mu_b, vext, lam, wu, wv, tau_form="gradient"):
        self.geom = geom
        self.tau_form = tau_form
        self.mu_a, self.mu_b = float(mu_a), float(mu_b)
        self.vext = np.asarray(vext, float)
        self.lam = np.asarray(lam, float)
        self.wu = np.asarray(wu, float)
        self.wv = np.asarray(wv, float)
        self.n_f_evals = 0

    def fields(self, phi):
        ra, rb, ta, tb, nu, ja, jb = self.geom.densities(phi, self.wu, self.wv, self.tau_form)
        Va, Vb, delta, Aa, Ab, Ava, Avb = potentials(ra, rb, ta, tb, _as_list(ja), _as_list(jb), nu, self.lam)
        return (Va + self.vext - self.mu_a, Vb + self.vext - self.mu_b, delta, Aa, Ab, Ava, Avb)

    def expect(self, phi, hphi):
        ax = tuple(range(1, phi.ndim))
        return self.geom.dV * np.real(np.sum(np.conj(phi) * hphi, axis=ax))

    def f(self, phi):
        self.n_f_evals += 1
        hphi = self.geom.apply_h(phi, *self.fields(phi))
        e = self.expect(phi, hphi)
        return -1j * (hphi - e.reshape((-1,) + (1,) * (phi.ndim - 1)) * phi)

    def normalize(self, phi):
        n = np.sqrt(self.geom.dV * np.sum(np.abs(phi) ** 2, axis=tuple(range(1, phi.ndim))))
        return phi / n.reshape((-1,) + (1,) * (phi.ndim - 1))

    def observables(self, phi):
        """E = int [energy density + V_ext rho_+] dV_e and N_a, N_b."""
        ra, rb, ta, tb, nu, ja, jb = self.geom.densities(phi, self.wu, self.wv, self.tau_form)
        e = energy_density(ra, rb, ta, tb, _as_list(ja), _as_list(jb), nu, self.lam) + self.vext * (ra + rb)
        dVe = self.geom.dV_energy
        return dict(E=dVe * np.sum(e), Na=dVe * np.sum(ra), Nb=dVe * np.sum(rb))


def dense_h_imbalanced(hf_a, hf_b, delta, nz, dz, kp2):
    """Dense reduced matrix [[h_a, D], [D^*, -h_b]] of one transverse
    momentum with A = 1: h_s = -1/2 D2 + hf_s + k_perp^2 / 2 (Eq. D2)."""
    K = -0.5 * L.d2_matrix(nz, dz) + 0.5 * kp2 * np.eye(nz)
    d = np.diag(np.asarray(delta, complex))
    return np.block([[K + np.diag(hf_a), d], [np.conj(d), -(K + np.diag(hf_b))]])


def eigenstates_imbalanced(geom, hf_a, hf_b, delta, ec):
    """Both branches: every eigenpair with |E| < ec of every transverse
    momentum.  Returns (E, kperp2, phi) normalised on the z lattice."""
    Es, kps, phis = [], [], []
    for kp2, _ in geom.problems():
        E, W = np.linalg.eigh(dense_h_imbalanced(hf_a, hf_b, delta, geom.nz, geom.dz, kp2))
        sel = np.nonzero(np.abs(E) < ec)[0]
        Es.append(E[sel])
        kps.append(np.full(sel.size, kp2))
        phis.append(W[:, sel].T.reshape(sel.size, 2, geom.nz) / np.sqrt(geom.dz))
    return np.concatenate(Es), np.concatenate(kps), np.concatenate(phis, axis=0)


def dense_h_imbalanced_3d(lat, hf_a, hf_b, delta):
    """Dense reduced matrix [[h_a, D], [D^*, -h_b]] on the 3D lattice with
    A = 1: h_s = -1/2 (D2_x + D2_y + D2_z) + hf_s (Eq. D2 per axis, flat
    index (ix N_y + iy) N_z + iz)."""
    nx, ny, nz = lat.n
    d2 = [L.d2_matrix(n, d) for n, d in zip(lat.n, lat.d)]
    K = -0.5 * (np.kron(np.kron(d2[0], np.eye(ny)), np.eye(nz)) + np.kron(np.kron(np.eye(nx), d2[1]), np.eye(nz))
                + np.kron(np.kron(np.eye(nx), np.eye(ny)), d2[2]))
    d = np.diag(np.ravel(delta).astype(complex))
    return np.block([[K + np.diag(np.ravel(hf_a)), d], [np.conj(d), -(K + np.diag(np.ravel(hf_b)))]])


def eigenstates_imbalanced_3d(lat, hf_a, hf_b, delta, ec):
    """Both branches: every eigenpair with |E| < ec of the 3D reduced
    matrix, normalised to int (|u|^2 + |v|^2) dV = 1.  Returns (E, phi)."""
    E, W = np.linalg.eigh(dense_h_imbalanced_3d(lat, hf_a, hf_b, delta))
    sel = np.nonzero(np.abs(E) < ec)[0]
    return E[sel], W[:, sel].T.reshape((sel.size, 2) + lat.shape) / np.sqrt(lat.dV)
