"""P11: the quasi-1D mode (Sec. 3.1) is an exact reduction of the full 3D
problem when the fields depend on z only.  Checked on an 8 x 8 x 16 box:
static densities from the dense 3D diagonalisation and from the 64 1D
problems, and densities after TD steps from product states."""
import numpy as np
import pytest

from oracle import lattice as L, bdg, densities as D, functional as F, td, q1d
import synth


def _setup():
    nz, nk = 16, 8
    geom = q1d.GeometryQ1D(nz, 1.0, nk, nk, 1.0)
    lat = L.Lattice(nk, nk, nz)
    z = L.centered_coords(nz, 1.0)
    mu = 1.0
    vext = 0.5 * 0.15 ** 2 * z ** 2 - 0.2 * np.exp(-(z - 1.3) ** 2 / 8.0)
    delta = 0.5 * np.exp(0.1j * synth.uniform_field(41, nz))
    return geom, lat, mu, vext, delta


def test_static_densities_match_3d():
    geom, lat, mu, vext, delta = _setup()
    E1, kp2, pid, phi1 = q1d.eigenstates(geom, vext - mu, delta)
    geom.set_states(kp2)
    w = (F.fermi_weight(E1), F.fermi_weight(-E1))
    r1, t1, n1, j1 = geom.full_densities(phi1, *w)
    hf3 = np.broadcast_to(vext - mu, lat.shape).copy()
    de3 = np.broadcast_to(delta, lat.shape).copy()
    E3, phi3 = bdg.eigenstates(hf3, de3, lat)
    pos = E3 > 0
    r3, t3, n3, j3 = D.spin_symmetric(phi3[pos], F.fermi_weight(E3[pos]), F.fermi_weight(-E3[pos]), lat)
    assert np.allclose(np.sort(E3[pos]), np.sort(E1), atol=1e-11)
    for a, b in ((r3, r1), (t3, t1), (n3, n1), (j3[2], j1[2])):
        assert np.abs(a - b[None, None, :]).max() < 1e-12 * max(1.0, np.abs(b).max())
    assert np.abs(j3[0]).max() < 1e-13 and np.abs(j3[1]).max() < 1e-13


def test_td_matches_3d_product_states():
    geom, lat, mu, vext, delta = _setup()
    E1, kp2, pid, phi1 = q1d.eigenstates(geom, vext - mu, delta)
    geom.set_states(kp2)
    wu, wv = F.fermi_weight(E1), F.fermi_weight(-E1)
    fun = F.Functional(F.SLDA)
    lam = F.lambda_c(vext, mu, 0.5 * np.pi ** 2)
    s1 = td.TDSystem(geom, fun, mu, vext, lam, wu, wv)
    # 3D product states exp(i k_perp . r_perp) / sqrt(L_x L_y) * phi(z)
    probs = geom.problems()
    x = np.arange(lat.n[0]) * 1.0
    y = np.arange(lat.n[1]) * 1.0
    phi3 = np.empty((len(E1), 2) + lat.shape, complex)
    for n in range(len(E1)):
        ix, iy = probs[pid[n]][1]
        pw = np.exp(1j * (geom.kx[ix] * x[:, None] + geom.ky[iy] * y[None, :])) / np.sqrt(geom.area)
        phi3[n] = pw[None, :, :, None] * phi1[n][:, None, None, :]
    vext3 = np.broadcast_to(vext, lat.shape).copy()
    lam3 = np.broadcast_to(lam, lat.shape).copy()
    s3 = td.TDSystem(td.Geometry3D(lat), fun, mu, vext3, lam3, wu, wv)
    # a quench: the bump is removed at t = 0
    z = L.centered_coords(geom.nz, 1.0)
    s1.vext = 0.5 * 0.15 ** 2 * z ** 2
    s3.vext = np.broadcast_to(s1.vext, lat.shape).copy()
    p1 = td.evolve(s1, phi1, 0.01, 6)
    p3 = td.evolve(s3, phi3, 0.01, 6)
    r1, n1 = geom.rho_nu(p1, wu, wv)
    r3, n3 = D.local_densities(p3, wu, wv)
    assert np.abs(r3 - r1[None, None, :]).max() < 1e-12 * np.abs(r1).max()
    assert np.abs(n3 - n1[None, None, :]).max() < 1e-12 * np.abs(n1).max()
    r0, _ = geom.rho_nu(phi1, wu, wv)
    assert np.abs(r1 - r0).max() > 1e-6  # the quench did move the density
    o1 = td.observables(s1, p1)
    o3 = td.observables(s3, p3)
    for key in ("kin", "pot", "pair", "potext", "N"):
        assert o1[key] == pytest.approx(o3[key], rel=1e-11, abs=1e-12)
