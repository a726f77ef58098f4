"""Pins of the A != 1 (general SLDA-type) functional path of the oracle:
the operator of Eq. h_sigma with the symmetrised kinetic term of Eq.
kinop-alpha and the current-potential anticommutator (matrix forms of Eqs.
D1, D2, Ad_dx, d_dxA), its potentials (Sec. 2.3 functional derivatives),
the uniform dispersion, energy conservation of a complete set that carries
currents, and the exact quasi-1D reduction."""
import numpy as np
import pytest

from oracle import lattice as L, bdg, densities as D, functional as F, td, q1d
import synth


def _fields(lat, seed):
    hf = synth.uniform_field(seed, lat.shape) * 0.6 - 0.4
    de = 0.3 * synth.complex_normal(seed + 1, lat.shape, 0.5)
    alpha = 1.0 + 0.3 * synth.uniform_field(seed + 2, lat.shape)
    avec = [0.4 * synth.uniform_field(seed + 3 + d, lat.shape) for d in range(3)]
    return hf, de, alpha, avec


def test_spectral_general_operator_equals_dense_matrices():
    """apply_h_general (FFTs) equals the dense matrix built from the D1 / D2
    matrices of Eqs. D1, D2 in the forms of Eqs. kinop-alpha, Ad_dx and
    d_dxA, for spatially varying alpha and A; the matrix is Hermitian."""
    lat = L.Lattice(4, 6, 4, 1.0, 0.9, 1.2)
    hf, de, alpha, avec = _fields(lat, 60)
    H = bdg.dense_h_general(hf, de, alpha, avec, lat)
    assert np.abs(H - H.conj().T).max() < 1e-13
    phi = synth.complex_normal(70, (3, 2) + lat.shape)
    got = bdg.apply_h_general(phi, hf, de, alpha, avec, lat)
    ref = np.array([(H @ p.reshape(-1)).reshape(p.shape) for p in phi])
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_general_operator_reduces_to_the_a1_operator():
    lat = L.Lattice(4, 4, 6)
    hf, de, _, _ = _fields(lat, 61)
    phi = synth.complex_normal(71, (2, 2) + lat.shape)
    a = bdg.apply_h_general(phi, hf, de, 1.0, None, lat)
    b = bdg.apply_h(phi, hf, de, lat)
    assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()


def test_general_uniform_dispersion():
    """Uniform fields, A = 0: E_k = +-sqrt((alpha k^2/2 + hfield)^2 + |Delta|^2)."""
    lat = L.Lattice(4, 4, 4)
    alpha, hf0, d0 = 1.094, -0.7, 0.4 + 0.1j
    H = bdg.dense_h_general(np.full(lat.shape, hf0), np.full(lat.shape, d0), alpha, None, lat)
    E = np.linalg.eigvalsh(H)
    xi = 0.5 * alpha * lat.k2.ravel() + hf0
    ek = np.sqrt(xi ** 2 + abs(d0) ** 2)
    assert np.abs(E - np.sort(np.concatenate([ek, -ek]))).max() < 1e-12


def test_general_potentials_are_functional_derivatives():
    """alpha = 2 dE/dtau_sigma, A = dE/dj_sigma and U = dE/drho_sigma of the
    A != 1 energy density (intrinsic + centre-of-mass parts) by central
    differences, for the SLDA constants at p = 0 (A = 1.094)."""
    fun = F.Functional(F.SLDA, force_a1=False)
    assert fun.A == pytest.approx(1.094)
    n = 12
    rho = 0.02 + 0.05 * synth.uniform_field(21, n, 0, 1)
    tau = 0.3 * synth.uniform_field(22, n, 0, 1)
    nu = 0.01 * synth.complex_normal(23, n)
    lam = 0.1 + 0.05 * synth.uniform_field(24, n, 0, 1)
    j = [0.01 * synth.uniform_field(25 + d, n) for d in range(3)]
    U, delta, alpha, avec = F.potentials_general(rho, nu, j, lam, fun)

    def e(r, t, jj):
        return F.energy_density(r, t, sum(c ** 2 for c in jj), nu, lam, fun)
    # the symmetric form depends on both spins: d/dx of it is 2 d/dx_sigma
    h = 1e-6 * rho
    assert np.allclose((e(rho + h, tau, j) - e(rho - h, tau, j)) / (2 * h) / 2, U, rtol=1e-7, atol=1e-10)
    ht = 1e-6
    assert np.allclose((e(rho, tau + ht, j) - e(rho, tau - ht, j)) / (2 * ht), alpha, rtol=1e-8)
    hj = 1e-6
    for d in range(3):
        jp = [c + (hj if k == d else 0.0) for k, c in enumerate(j)]
        jm = [c - (hj if k == d else 0.0) for k, c in enumerate(j)]
        assert np.allclose((e(rho, tau, jp) - e(rho, tau, jm)) / (2 * hj) / 2, avec[d], rtol=1e-6, atol=1e-12)
    # and the A = 1 case has no current potential
    U1, d1, a1, av1 = F.potentials_general(rho, nu, j, lam, F.Functional(F.SLDA))
    assert a1 == 1.0 and all(np.abs(c).max() == 0 for c in av1)


def _complete_set_with_currents(n=6):
    """The complete E > 0 set of the uniform 6^3 SLDA state at A = 1.094
    (dense diagonalisation of the general operator), with a vortex imprint
    so that the evolution carries currents."""
    lat = L.Lattice(n, n, n)
    fun = F.Functional(F.SLDA, force_a1=False)
    mu = 1.0
    H = bdg.dense_h_general(np.full(lat.shape, -mu), np.full(lat.shape, 0.5 + 0j), fun.A, None, lat)
    E, W = np.linalg.eigh(H)
    phi = W.T.reshape((2 * lat.M, 2) + lat.shape) / np.sqrt(lat.dV)
    pos = E > 0
    E, phi = E[pos], phi[pos]
    phi = bdg.imprint_phase(phi, bdg.vortex_phase(lat, [(0.3, -0.2, 1.0)]))
    lam = F.lambda_c(np.zeros(lat.shape), mu, 0.5 * np.pi ** 2, A=fun.A)
    return lat, fun, mu, lam, E, phi


class _FlippedCurrent(td.TDSystem):
    """Planted mistake: the current potential enters H with the wrong sign."""

    def fields(self, phi):
        hf, de, al, av = super().fields(phi)
        return hf, de, al, [-c for c in av]


def _drift(cls, dt):
    lat, fun, mu, lam, E, phi = _complete_set_with_currents()
    s = cls(td.Geometry3D(lat), fun, mu, np.zeros(lat.shape), lam, F.fermi_weight(E), F.fermi_weight(-E))
    p, hist, _ = td.start(s, phi, dt, "AB4AM5", 1)
    o0 = td.observables(s, p)
    for _ in range(int(round(0.1 / dt))):
        p, hist = td.abm_step(s, p, hist, dt, "AB4AM5")
    o1 = td.observables(s, p)
    jmax = max(np.abs(c).max() for c in D.spin_symmetric(p, s.wu, s.wv, lat)[3])
    return abs(o1["total"] - o0["total"]) / o0["EFG"], abs(o1["N"] - o0["N"]) / o0["N"], jmax, o1


def test_general_functional_conserves_energy_with_currents():
    """With A != 1 the energy E_kin + E_curr + E_pot + E_pair (Sec. 3.2) of
    a complete set carrying currents is conserved to the integrator's
    accuracy (drift falling at its order); with the current potential's
    sign flipped it is not."""
    d1, n1, j1, o1 = _drift(td.TDSystem, 0.01)
    d2, n2, j2, o2 = _drift(td.TDSystem, 0.005)
    assert j2 > 1e-3 and abs(o2["curr"]) > 1e-4 * o2["EFG"]  # the currents are there
    assert n1 < 1e-7 and n2 < 1e-8
    assert d2 < 1e-7 and d1 / d2 > 16
    bad, _, _, _ = _drift(_FlippedCurrent, 0.005)
    assert bad > 100 * d2


def test_quasi_1d_general_operator_is_the_3d_one_on_product_states():
    """Exact mode reduction with A != 1 (Sec. 3.1, quasi-1D item): for fields
    depending on z only (alpha(z), A = (0, 0, A_z(z))), the 3D general
    operator on exp(i k_perp . r_perp) phi(z) equals the quasi-1D one on
    phi(z) (kinetic with 1/2 alpha k_perp^2, current along z only)."""
    nz, nk = 8, 4
    geom = q1d.GeometryQ1D(nz, 1.0, nk, nk, 1.3)
    lat = L.Lattice(nk, nk, nz, 1.3, 1.3, 1.0)
    hf = synth.uniform_field(81, nz) - 0.5
    de = 0.3 * synth.complex_normal(82, nz)
    al = 1.0 + 0.2 * synth.uniform_field(83, nz)
    az = 0.3 * synth.uniform_field(84, nz)
    probs = geom.problems()
    picks = [0, 5, 10, 15]
    geom.set_states([probs[p][0] for p in picks])
    phi1 = synth.complex_normal(85, (len(picks), 2, nz))
    h1 = geom.apply_h(phi1, hf, de, al, [np.zeros(nz), np.zeros(nz), az])
    b3 = lambda f: np.broadcast_to(f, lat.shape).copy()
    x = np.arange(nk) * 1.3
    for n, p in enumerate(picks):
        ix, iy = probs[p][1]
        pw = np.exp(1j * (geom.kx[ix] * x[:, None] + geom.ky[iy] * x[None, :]))
        phi3 = (pw[None, :, :, None] * phi1[n][:, None, None, :])[None]
        h3 = bdg.apply_h_general(phi3, b3(hf), b3(de), b3(al), [np.zeros(lat.shape)] * 2 + [b3(az)], lat)[0]
        ref = pw[None, :, :, None] * h1[n][:, None, None, :]
        assert np.abs(h3 - ref).max() < 1e-12 * np.abs(ref).max()
