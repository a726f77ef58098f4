"""Pins of the oracle's BdG operator, initial states and densities
(Sec. 2.3; Eqs. HpsiEpsi, HBdG, na3D-jb3D, nab3D-jab3D)."""
import numpy as np
import pytest

from oracle import lattice as L, bdg, densities as D, functional as F, uniform as UN
import synth


def _all_k(lat):
    return np.array(np.meshgrid(*[range(n) for n in lat.n], indexing="ij")).reshape(3, -1).T


@pytest.mark.parametrize("shape,d", [((4, 4, 4), 1.0), ((4, 6, 8), 0.9)])
def test_uniform_dispersion(shape, d):
    """P2: eigenvalues of the dense H with constant fields are
    +-sqrt((k^2/2 + U - mu)^2 + |Delta|^2) over the lattice momenta."""
    lat = L.Lattice(*shape, d, d, d)
    U, mu, delta = 0.3, 1.1, 0.5 * np.exp(0.7j)
    E, _ = bdg.eigenstates(np.full(lat.shape, U - mu), np.full(lat.shape, delta), lat)
    xi = 0.5 * lat.k2.ravel() + U - mu
    Ek = np.sqrt(xi ** 2 + abs(delta) ** 2)
    ref = np.sort(np.concatenate([Ek, -Ek]))
    assert np.abs(E - ref).max() < 1e-12 * ref.max()


def test_plane_wave_states_are_eigenvectors():
    """P3a: H phi_k = E_k phi_k for the analytic uniform states, with
    orthonormality."""
    lat = L.Lattice(4, 4, 6, 1.0, 1.0, 0.8)
    U, mu, delta = -0.2, 1.0, 0.45 * np.exp(-0.3j)
    E, phi = bdg.plane_wave_states(lat, _all_k(lat), U - mu, delta)
    hphi = bdg.apply_h(phi, np.full(lat.shape, U - mu), np.full(lat.shape, delta), lat)
    assert np.abs(hphi - E[:, None, None, None, None] * phi).max() < 1e-13
    G = lat.dV * phi.reshape(len(E), -1).conj() @ phi.reshape(len(E), -1).T
    assert np.abs(G - np.eye(len(E))).max() < 1e-13
    assert np.all(E > 0)


def test_dense_matvec_equals_spectral_apply():
    """P3b: the dense matrix built from Eq. D2 and diagonal fields applied
    to random states equals the FFT-based operator."""
    lat = L.Lattice(4, 6, 4, 1.0, 0.7, 1.2)
    hf = synth.uniform_field(21, lat.shape)
    de = synth.complex_normal(22, lat.shape, 0.3)
    phi = synth.complex_normal(23, (3, 2) + lat.shape)
    H = bdg.dense_h(hf, de, lat)
    a = (H @ phi.reshape(3, -1).T).T.reshape(phi.shape)
    b = bdg.apply_h(phi, hf, de, lat)
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
    assert np.allclose(H, H.conj().T)


@pytest.mark.parametrize("T", [0.0, 0.4])
@pytest.mark.parametrize("gauge", [False, True])
def test_general_equals_spin_symmetric(T, gauge):
    """P7: densities of all 2M states with both branches explicit
    (Eqs. na3D-jb3D) equal the spin-symmetric form over E>0 states only
    (Eqs. nab3D-jab3D).  With the gauge, the vortex imprint is applied to
    the whole eigenbasis (both signs of E): the imprinted E>0 states must
    still reproduce the densities of the imprinted complete set, tau and j
    included, which holds only if the imprint commutes with the partner map
    (u, v) -> (v^*, -u^*) of the spin-symmetric case (a phase on u alone
    fails here: tau_a != tau_b)."""
    lat = L.Lattice(4, 4, 4)
    hf = synth.uniform_field(31, lat.shape) - 0.8
    de = synth.complex_normal(32, lat.shape, 0.4)
    E, phi = bdg.eigenstates(hf, de, lat)
    pos = E > 0
    Ep, php = E[pos], phi[pos]
    # the E<0 half of the spectrum is the partner set, up to phases
    assert np.allclose(np.sort(-E[~pos]), np.sort(Ep), atol=1e-12)
    phi_all, E_all = phi, E
    if gauge:
        theta = bdg.vortex_phase(lat, [(0.3, -0.2, 1)])
        phi_all = bdg.imprint_phase(phi, theta)
        php = bdg.imprint_phase(php, theta)
    g = D.general(phi_all, F.fermi_weight(E_all, T), F.fermi_weight(-E_all, T), lat)
    rho, tau, nu, j = D.spin_symmetric(php, F.fermi_weight(Ep, T), F.fermi_weight(-Ep, T), lat)
    tol = 1e-13
    assert np.abs(g["rho_a"] - rho).max() < tol and np.abs(g["rho_b"] - rho).max() < tol
    assert np.abs(g["tau_a"] - tau).max() < 10 * tol and np.abs(g["tau_b"] - tau).max() < 10 * tol
    assert np.abs(g["nu"] - nu).max() < tol
    for c in range(3):
        assert np.abs(g["j_a"][c] - j[c]).max() < tol and np.abs(g["j_b"][c] - j[c]).max() < tol


def test_imprint_commutes_with_partner_map():
    """The vortex imprint maps the partner (v^*, -u^*) of a state to the
    partner of the imprinted state, keeps states orthonormal and multiplies
    nu by e^{i theta} while leaving rho unchanged."""
    lat = L.Lattice(6, 6, 2)
    phi = D.normalize(synth.complex_normal(35, (4, 2) + lat.shape), lat.dV)
    theta = bdg.vortex_phase(lat, [(0.4, 0.1, 1), (-1.3, 0.7, -1)])
    partner = lambda p: np.stack([np.conj(p[:, 1]), -np.conj(p[:, 0])], axis=1)
    a = bdg.imprint_phase(partner(phi), theta)
    b = partner(bdg.imprint_phase(phi, theta))
    assert np.abs(a - b).max() < 1e-15
    G0 = np.einsum("aclmn,bclmn->ab", np.conj(phi), phi)
    G1 = np.einsum("aclmn,bclmn->ab", np.conj(bdg.imprint_phase(phi, theta)), bdg.imprint_phase(phi, theta))
    assert np.abs(G1 - G0).max() < 1e-13
    w = np.linspace(0.1, 0.9, 4)
    r0, _, n0, _ = D.spin_symmetric(phi, w, 1 - w, lat)
    r1, _, n1, _ = D.spin_symmetric(bdg.imprint_phase(phi, theta), w, 1 - w, lat)
    assert np.abs(r1 - r0).max() < 1e-15 * np.abs(r0).max() * 10
    assert np.abs(n1 - np.exp(1j * theta) * n0).max() < 1e-14 * np.abs(n0).max()


def test_kinetic_density_integrates_to_laplacian_expectation():
    """int tau dV = sum_n w_n <v_n| -nabla^2 |v_n> exactly (the D^(2)
    operator of H), which the energy of Sec. 3.2 needs to be conserved."""
    lat = L.Lattice(4, 6, 8, 1.0, 0.8, 1.1)
    phi = synth.complex_normal(33, (5, 2) + lat.shape)
    w = synth.uniform_field(34, 5, 0, 1)
    rho, tau, nu, j = D.spin_symmetric(phi, np.zeros(5), w, lat)
    lap = L.laplacian(phi[:, 1], lat)
    ref = -lat.dV * np.sum(w[:, None, None, None] * np.real(np.conj(phi[:, 1]) * lap))
    assert lat.dV * tau.sum() == pytest.approx(ref, rel=1e-13)


def test_free_gas_lattice_sums():
    """P4: with Delta = 0 the densities of the uniform states reproduce the
    brute-force count of occupied lattice momenta; int tau dV is the sum of
    k^2 over them."""
    for n in (8, 12):
        lat = L.Lattice(n, n, n)
        mu = 1.0
        E, phi = bdg.plane_wave_states(lat, _all_k(lat), -mu, 0.0)
        rho, tau, nu, j = D.spin_symmetric(phi, np.zeros(len(E)), np.ones(len(E)), lat)
        nocc, esum = UN.free_gas_lattice_count(n, 1.0, mu)
        assert lat.dV * rho.sum() == pytest.approx(nocc, rel=1e-13)
        assert lat.dV * tau.sum() == pytest.approx(2 * esum, rel=1e-12)
        assert np.abs(nu).max() < 1e-15 and max(np.abs(c).max() for c in j) < 1e-14


def test_free_gas_energy_tends_to_EFG():
    """P4: E / (3/5 N eF) -> 1 as the box grows at fixed density scale."""
    dev = []
    for n in (16, 32, 64):
        nocc, esum = UN.free_gas_lattice_count(n, 1.0, 1.0)
        N = 2 * nocc
        V = n ** 3
        dev.append(abs(2 * esum / (0.6 * N * F.eF(N / V)) - 1))
    assert dev[-1] < 0.03 and dev[-1] < dev[0]


def test_vortex_phase_winding():
    lat = L.Lattice(16, 16, 2)
    th = bdg.vortex_phase(lat, [(0.25, 0.35, 1)])
    # winding around the core along a closed lattice loop is 2 pi
    loop = [(i, 4) for i in range(4, 12)] + [(11, j) for j in range(4, 12)] + \
           [(i, 11) for i in range(11, 3, -1)] + [(4, j) for j in range(11, 3, -1)]
    ph = np.array([th[i, j, 0] for i, j in loop] + [th[loop[0][0], loop[0][1], 0]])
    w = np.sum(np.angle(np.exp(1j * np.diff(ph))))
    assert w == pytest.approx(2 * np.pi, abs=1e-12)
