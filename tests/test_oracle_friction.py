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
