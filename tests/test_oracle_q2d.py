"""The quasi-2D time-dependent mode (Sec. 3.1) is an exact reduction of the
full 3D problem when the fields do not depend on z: the static densities of
the |k_z| classes (one state per class, weighted by its multiplicity) equal
those of the dense 3D diagonalisation, and the evolution of the quasi-2D
states equals the 3D evolution of the product states exp(i k_z z) phi(x, y)
of both signs of k_z."""
import numpy as np
import pytest

from oracle import lattice as L, bdg, densities as D, functional as F, td, q2d
import synth


def _setup(nx=6, ny=4, nz=4):
    geom = q2d.GeometryQ2D(nx, ny, nz, 1.0, 1.2, 1.0)
    lat = L.Lattice(nx, ny, nz, 1.0, 1.2, 1.0)
    X, Y = geom.static.coords()
    mu = 1.0
    vext = 0.5 * 0.2 ** 2 * (X ** 2 + Y ** 2) + 0.3 * np.exp(-((X - 0.7) ** 2 + Y ** 2) / 2.0)
    delta = 0.5 + 0.05 * synth.uniform_field(61, geom.shape)
    return geom, lat, mu, vext, delta


def test_static_densities_match_3d():
    geom, lat, mu, vext, delta = _setup()
    E2, kz2, mult, phi2 = q2d.eigenstates(geom, vext - mu, delta)
    geom.set_states(kz2)
    r2, t2, n2, j2 = geom.full_densities(phi2, mult * F.fermi_weight(E2), mult * F.fermi_weight(-E2))
    b = lambda f: np.repeat(np.asarray(f)[:, :, None], lat.n[2], axis=2)
    E3, phi3 = bdg.eigenstates(b(vext - mu), b(delta) + 0j, lat)
    pos = E3 > 0
    r3, t3, n3, j3 = D.spin_symmetric(phi3[pos], F.fermi_weight(E3[pos]), F.fermi_weight(-E3[pos]), lat)
    # the same spectrum: every class eigenvalue with its multiplicity
    assert np.allclose(np.sort(E3[pos]), np.sort(np.repeat(E2, mult.astype(int))), atol=1e-11)
    for a, c in ((r3, r2), (t3, t2), (n3, n2)):
        assert np.abs(a - b(c)).max() < 1e-12 * max(1.0, np.abs(c).max())
    assert np.abs(j3[2]).max() < 1e-13


def test_td_matches_3d_product_states():
    geom, lat, mu, vext, delta = _setup()
    E2, kz2, mult, phi2 = q2d.eigenstates(geom, vext - mu, delta)
    geom.set_states(kz2)
    fun = F.Functional(F.SLDA)
    lam = F.lambda_c(vext, mu, 0.5 * np.pi ** 2)
    wu, wv = mult * F.fermi_weight(E2), mult * F.fermi_weight(-E2)
    trap = vext - 0.3 * np.exp(-((geom.static.coords()[0] - 0.7) ** 2 + geom.static.coords()[1] ** 2) / 2.0)
    s2 = td.TDSystem(geom, fun, mu, trap, lam, wu, wv)  # the obstacle is removed at t = 0
    # 3D product states of both signs of k_z (the Nyquist momentum once)
    z = np.arange(lat.n[2]) * lat.d[2]
    kzs = L.kgrid(lat.n[2], lat.d[2])
    phi3, E3 = [], []
    for n in range(len(E2)):
        for kz in kzs:
            if np.isclose(kz * kz, kz2[n]):
                phi3.append(phi2[n][:, :, :, None] * np.exp(1j * kz * z)[None, None, None, :] / np.sqrt(geom.Lz))
                E3.append(E2[n])
    phi3, E3 = np.array(phi3), np.array(E3)
    assert len(E3) == int(mult.sum())
    b = lambda f: np.repeat(np.asarray(f)[:, :, None], lat.n[2], axis=2)
    s3 = td.TDSystem(td.Geometry3D(lat), fun, mu, b(trap), b(lam), F.fermi_weight(E3), F.fermi_weight(-E3))
    p2 = td.evolve(s2, phi2, 0.01, 5)
    p3 = td.evolve(s3, phi3, 0.01, 5)
    r2, t2, n2, j2 = geom.full_densities(p2, wu, wv)
    r3, t3, n3, j3 = D.spin_symmetric(p3, s3.wu, s3.wv, lat)
    for a, c in ((r3, r2), (t3, t2), (n3, n2), (j3[0], j2[0]), (j3[1], j2[1])):
        assert np.abs(a - b(c)).max() < 1e-11 * max(1.0, np.abs(c).max())
    r0, _ = geom.rho_nu(phi2, wu, wv)
    assert np.abs(r2 - r0).max() > 1e-6  # the quench did move the density
    o2, o3 = td.observables(s2, p2), td.observables(s3, p3)
    for key in ("kin", "pot", "pair", "curr", "potext", "N", "total"):
        assert o2[key] == pytest.approx(o3[key], rel=1e-10, abs=1e-12)


def test_plane_waves_are_eigenstates_of_the_uniform_problem():
    """The quasi-2D uniform start is an eigenvector of H with constant
    fields (hfield = U - mu, Delta real) with eigenvalue E, for every class,
    and normalised on the x-y lattice; the multiplicities count the two
    signs of k_z except for k_z = 0 and the Nyquist class."""
    geom = q2d.GeometryQ2D(6, 4, 6, 1.0, 1.3, 0.9)
    kidx = np.array([(a, b, m) for a in range(6) for b in range(4) for m in range(4)])
    E, kz2, mult, phi = q2d.plane_wave_states(geom, kidx, -0.7, 0.4)
    geom.set_states(kz2)
    hphi = geom.apply_h(phi, np.full(geom.shape, -0.7), np.full(geom.shape, 0.4 + 0j))
    assert np.abs(hphi - E[:, None, None, None] * phi).max() < 1e-13
    assert np.abs(geom.dV * np.sum(np.abs(phi) ** 2, axis=(1, 2, 3)) - 1).max() < 1e-13
    assert set(mult[kidx[:, 2] == 0]) == {1.0} and set(mult[kidx[:, 2] == 3]) == {1.0}
    assert set(mult[(kidx[:, 2] == 1) | (kidx[:, 2] == 2)]) == {2.0}
    assert np.allclose(kz2, (2 * np.pi * kidx[:, 2] / (6 * 0.9)) ** 2)
