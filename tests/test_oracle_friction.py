"""Pins of the quantum-friction evolution (Sec. 5.2, correcting the initial
state by a time-dependent approach) in the quasi-1D geometry, from what the
paper states about each term: without parameters the evolution is the
plain one; the beta term lowers the energy at every step (it damps the
pairing field) and keeps N; the alpha term lowers the energy, against a
conserved energy without it; the gamma term moves N towards N_req from
either side."""
import numpy as np
import pytest

from oracle import lattice as L, functional as F, td, q1d
import synth

STEPS = 30


@pytest.fixture(scope="module")
def setup():
    # the complete set of states (no energy cut-off), so that the plain
    # evolution conserves the energy
    nz, nk, dperp, ec = 32, 4, 1.3, None
    geom = q1d.GeometryQ1D(nz, 1.0, nk, nk, dperp)
    z = L.centered_coords(nz, 1.0)
    mu = 1.0
    vb, wb, zb = synth.gaussian_bump(3)
    zb = zb * nz / 256.0
    trap = 0.5 * (0.0175 * 256 / nz) ** 2 * z ** 2
    vext = trap + vb * np.exp(-(z - zb) ** 2 / (2 * wb ** 2))
    E, kp2, pid, phi = q1d.eigenstates(geom, vext - mu, np.full(nz, 0.5 + 0j), ec=ec)
    geom.set_states(kp2)
    lam = F.lambda_c(vext, mu, 0.5 * np.pi ** 2)
    return geom, mu, trap, lam, E, phi


def run(setup, friction):
    geom, mu, trap, lam, E, phi = setup
    s = td.TDSystem(geom, F.Functional(F.SLDA), mu, trap, lam, F.fermi_weight(E), F.fermi_weight(-E),
                    friction=friction)
    out = []
    td.evolve(s, phi, 0.01, STEPS, callback=lambda k, p: out.append(td.observables(s, p)))
    return np.array([o["total"] for o in out]), np.array([o["N"] for o in out]), s


def test_zero_parameters_are_the_plain_evolution(setup):
    e0, n0, s0 = run(setup, None)
    e1, n1, s1 = run(setup, td.Friction(0.0, 0.0, 0.0, rho0=1.0, N_req=100.0))
    assert np.array_equal(e0, e1) and np.array_equal(n0, n1)
    assert abs(e0[-1] - e0[0]) < 1e-6 * abs(e0[0])


def test_beta_term_lowers_the_energy_every_step(setup):
    e, n, _ = run(setup, td.Friction(beta=5.0))
    assert np.all(np.diff(e) < 0)
    assert e[0] - e[-1] > 1e-3 * abs(e[0])
    assert np.abs(n - n[0]).max() < 1e-6 * n[0]


def test_alpha_term_lowers_the_energy(setup):
    e0, _, _ = run(setup, None)
    e, _, _ = run(setup, td.Friction(alpha=5.0, rho0=0.05))
    drift = abs(e0[-1] - e0[0])
    assert e[0] - e[-1] > 20 * drift


@pytest.mark.parametrize("side", [1.01, 0.99])
def test_gamma_term_moves_n_towards_n_req(setup, side):
    _, n0, _ = run(setup, None)
    N_req = side * n0[0]
    _, n, _ = run(setup, td.Friction(gamma=0.1, N_req=N_req))
    gap = np.abs(n - N_req)
    assert np.all(np.diff(gap) < 0)


# ---------------------------------------------------------------------------
# full 3D

def test_3d_sources_are_the_quasi_1d_ones_on_product_states(setup):
    """Exact mode reduction (Sec. 3.1): on product states exp(i k_perp.r_perp)
    phi(z) / sqrt(L_x L_y) of every transverse momentum, the 3D sources (div j
    from all three axes, B' with the full Laplacian) equal the quasi-1D ones
    (d_z j_z, B' with D2z - k_perp^2)."""
    geom, mu, trap, lam, E, phi = setup
    nk = len(geom.kx)
    lat = L.Lattice(nk, nk, geom.nz, geom.Lx / nk, geom.Ly / nk, geom.dz)
    probs = geom.problems()
    x = np.arange(nk) * lat.d[0]
    phi3 = np.empty((len(E), 2) + lat.shape, complex)
    # the problem of every state, as q1d.eigenstates orders them (the fixture's
    # static fields include the bump)
    z = L.centered_coords(geom.nz, 1.0)
    vb, wb, zb = synth.gaussian_bump(3)
    vext = trap + vb * np.exp(-(z - zb * geom.nz / 256.0) ** 2 / (2 * wb ** 2))
    _, _, pid, _ = q1d.eigenstates(geom, vext - mu, np.full(geom.nz, 0.5 + 0j))
    assert len(pid) == len(E)
    wu, wv = F.fermi_weight(E), F.fermi_weight(-E)
    # a current along z and a complex B': evolve a little first (the quasi-1D
    # trap without the bump sets the states in motion)
    s1 = td.TDSystem(geom, F.Functional(F.SLDA), mu, trap, lam, wu, wv)
    p1 = td.evolve(s1, phi, 0.01, 3)
    for n in range(len(E)):
        ix, iy = probs[pid[n]][1]
        pw = np.exp(1j * (geom.kx[ix] * x[:, None] + geom.ky[iy] * x[None, :])) / np.sqrt(geom.area)
        phi3[n] = pw[None, :, :, None] * p1[n][:, None, None, :]
    d1, b1, n1 = geom.friction_sources(p1, wu, wv)
    d3, b3, n3 = td.Geometry3D(lat).friction_sources(phi3, wu, wv)
    assert np.abs(d1).max() > 1e-6
    assert np.abs(d3 - d1[None, None, :]).max() < 1e-10 * np.abs(d1).max()
    assert np.abs(b3 - b1[None, None, :]).max() < 1e-10 * np.abs(b1).max()
    assert n3 == pytest.approx(n1, rel=1e-12)


@pytest.fixture(scope="module")
def setup3d():
    """Complete E > 0 set of a uniform 6^3 state in a weak trap with a vortex
    (currents and a pairing field out of equilibrium)."""
    from oracle import bdg
    lat = L.Lattice(6, 6, 6)
    mu = 1.0
    E, phi = bdg.eigenstates(np.full(lat.shape, -mu), np.full(lat.shape, 0.5 + 0j), lat)
    pos = E > 0
    E, phi = E[pos], phi[pos]
    phi = bdg.imprint_phase(phi, bdg.vortex_phase(lat, [(0.3, -0.2, 1.0)]))
    X, Y, Z = lat.coords()
    trap = 0.5 * 0.15 ** 2 * (X ** 2 + Y ** 2 + Z ** 2)
    lam = F.lambda_c(np.zeros(lat.shape), mu, 0.5 * np.pi ** 2)
    return lat, mu, trap, lam, E, phi


def run3d(setup3d, friction, steps=20):
    lat, mu, trap, lam, E, phi = setup3d
    s = td.TDSystem(td.Geometry3D(lat), F.Functional(F.SLDA), mu, trap, lam, F.fermi_weight(E),
                    F.fermi_weight(-E), friction=friction)
    out = []
    td.evolve(s, phi, 0.01, steps, callback=lambda k, p: out.append(td.observables(s, p)))
    return np.array([o["total"] for o in out]), np.array([o["N"] for o in out])


def test_3d_friction_terms(setup3d):
    """In 3D, as in quasi-1D: zero parameters are the plain (energy
    conserving) evolution; the beta term lowers the energy at every step and
    keeps N; the alpha term lowers the energy; the gamma term moves N towards
    N_req."""
    e0, n0 = run3d(setup3d, None)
    drift = abs(e0[-1] - e0[0])
    assert drift < 1e-6 * abs(e0[0])
    e1, n1 = run3d(setup3d, td.Friction(0.0, 0.0, 0.0, rho0=1.0, N_req=10.0))
    assert np.array_equal(e0, e1)
    eb, nb = run3d(setup3d, td.Friction(beta=5.0))
    assert np.all(np.diff(eb) < 0) and eb[0] - eb[-1] > 1e-4 * abs(eb[0])
    assert np.abs(nb - nb[0]).max() < 1e-6 * nb[0]
    ea, _ = run3d(setup3d, td.Friction(alpha=5.0, rho0=0.05))
    assert ea[0] - ea[-1] > 20 * drift
    N_req = 1.01 * n0[0]
    _, ng = run3d(setup3d, td.Friction(gamma=0.1, N_req=N_req))
    assert np.all(np.diff(np.abs(ng - N_req)) < 0)
