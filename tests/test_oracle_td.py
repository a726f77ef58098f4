"""Pins of the oracle's time integration (Sec. 3.3): multistep
coefficients, convergence order, stationarity, conservation laws,
reversibility and the Taylor start-up."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import lattice as L, bdg, densities as D, functional as F, td, uniform as UN
import synth


@pytest.mark.parametrize("q", [3, 4, 5])
def test_adams_bashforth_is_exact_on_polynomials(q):
    """P13: AB_q integrates polynomials of degree < q exactly over one step
    from the q previous samples, and not degree q (the defining property of
    the Adams-Bashforth weights)."""
    b = td.AB[q]
    assert b.sum() == pytest.approx(1.0, abs=1e-15)
    h, k = 0.1, 7
    for m in range(q + 1):
        exact = ((k * h) ** (m + 1) - ((k - 1) * h) ** (m + 1)) / (m + 1)
        approx = h * sum(b[j] * ((k - 1 - j) * h) ** m for j in range(q))
        if m < q:
            assert approx == pytest.approx(exact, rel=1e-13)
        else:
            assert abs(approx - exact) > 1e-8 * abs(exact)


@pytest.mark.parametrize("q", [4, 5])
def test_adams_moulton_is_exact_on_polynomials(q):
    a = td.AM[q]
    h, k = 0.1, 7
    for m in range(q + 1):
        exact = ((k * h) ** (m + 1) - ((k - 1) * h) ** (m + 1)) / (m + 1)
        approx = h * sum(a[j] * ((k - j) * h) ** m for j in range(q))
        if m < q:
            assert approx == pytest.approx(exact, rel=1e-13)
        else:
            assert abs(approx - exact) > 1e-8 * abs(exact)


def _linear_system(seed=1):
    lat = L.Lattice(4, 4, 4, 1.5, 1.5, 1.5)
    hf = synth.uniform_field(seed, lat.shape) * 0.5 - 0.3
    de = 0.4 * synth.complex_normal(seed + 1, lat.shape, 0.5)
    phi0 = D.normalize(synth.complex_normal(seed + 2, (2, 2) + lat.shape), lat.dV)
    sysl = td.TDSystem(td.Geometry3D(lat), None, 0.0, np.zeros(lat.shape), np.zeros(lat.shape),
                       [0, 0], [1, 1], frozen=(hf, de))
    H = bdg.dense_h(hf, de, lat)

    def exact(phi, t):
        out = []
        for p in phi:
            x = p.ravel() * np.sqrt(lat.dV)
            h = np.vdot(x, H @ x).real
            out.append((np.exp(1j * h * t) * (expm(-1j * H * t) @ x)).reshape(p.shape) / np.sqrt(lat.dV))
        return np.array(out)
    return lat, sysl, phi0, exact


@pytest.mark.parametrize("scheme,order", [("AB3AM4", 4), ("AB4AM5", 5), ("AB5AM5", 5)])
def test_convergence_order_in_linear_mode(scheme, order):
    """P9: with the fields frozen the shifted equation has the exact
    solution exp(i <H> t) exp(-i H t) phi(0); the global error of the
    integrator falls with the order of its corrector."""
    lat, sysl, phi0, exact = _linear_system()
    T = 1.2
    ref = exact(phi0, T)
    errs = []
    for dt in (0.04, 0.02, 0.01):
        n = int(round(T / dt))
        phi, hist, ns = td.start(sysl, phi0, dt, scheme, 1)
        for _ in range(n - ns):
            phi, hist = td.abm_step(sysl, phi, hist, dt, scheme)
        errs.append(np.abs(phi - ref).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.4), rates


def test_taylor_step_in_linear_mode():
    """One Taylor start-up step of order r equals the exact propagator up to
    the truncation of the exponential series (error ~ (|H| dt)^(r+1))."""
    lat, sysl, phi0, exact = _linear_system(5)
    for dt, tol in ((0.05, 1e-7), (0.025, 5e-9)):
        p1 = td.taylor_step(sysl, phi0, dt, 5)
        assert np.abs(p1 - exact(phi0, dt)).max() < tol


def test_stationary_uniform_state():
    """P8: the self-consistent uniform lattice state is stationary: f = 0 and
    the states do not move over 20 steps (Sec. 3.3: in the stationary case
    the shifted equation gives phi(t) = phi(0))."""
    lat = L.Lattice(6, 6, 6)
    fun = F.Functional(F.SLDA)
    mu, ec = 1.0, 0.5 * np.pi ** 2
    lam = float(F.lambda_c(0.0, mu, ec))
    U, d = UN.lattice_uniform(lat, fun, mu, lam)
    kidx = np.array(np.meshgrid(*[range(n) for n in lat.n], indexing="ij")).reshape(3, -1).T
    E, phi = bdg.plane_wave_states(lat, kidx, U - mu, d)
    sys_ = td.TDSystem(td.Geometry3D(lat), fun, mu, np.zeros(lat.shape), np.full(lat.shape, lam),
                       np.zeros(len(E)), np.ones(len(E)))
    assert np.abs(sys_.f(phi)).max() < 1e-13
    out = td.evolve(sys_, phi, 0.005, 20)
    assert np.abs(out - phi).max() < 1e-12


def config1_initial(seed=0):
    """8^3 unitary-gas SLDA (A=1), dense BdG with U=0, Delta = 0.5 exp(0.01 i
    eta), mu = 1; E>0 half of the spectrum, T = 0; Lambda_c frozen with the
    lattice cutoff (pi/dx)^2/2 and V_+ = V_ext = 0."""
    lat = L.Lattice(8, 8, 8)
    fun = F.Functional(F.SLDA)
    mu = 1.0
    eta = synth.uniform_field(seed, lat.shape)
    E, phi = bdg.eigenstates(np.full(lat.shape, -mu), 0.5 * np.exp(1j * 0.01 * eta), lat)
    pos = E > 0
    lam = F.lambda_c(np.zeros(lat.shape), mu, 0.5 * np.pi ** 2)
    sys_ = td.TDSystem(td.Geometry3D(lat), fun, mu, np.zeros(lat.shape), lam,
                       F.fermi_weight(E[pos]), F.fermi_weight(-E[pos]))
    return lat, sys_, phi[pos]


def test_config1_conservation():
    """P10: with the complete set of states, the number of particles, the
    energy (A=1 kinetic term from the Laplacian, frozen regulator) and the
    orthonormality of the states are conserved by the ABM steps."""
    lat, sys_, phi0 = config1_initial()
    phi, hist, ns = td.start(sys_, phi0, 0.005, "AB4AM5", 1)
    o0 = td.observables(sys_, phi)
    for s in range(20):
        phi, hist = td.abm_step(sys_, phi, hist, 0.005, "AB4AM5")
        if s == 4:
            o5 = td.observables(sys_, phi)
    o1 = td.observables(sys_, phi)
    # the first steps still carry the start-up's error in the history;
    # after them N is conserved to the integrator's accuracy
    assert abs(o1["N"] - o5["N"]) / o0["N"] < 1e-10
    assert abs(o1["N"] - o0["N"]) / o0["N"] < 1e-9
    G = td.gram(phi, lat.dV)
    assert abs(o1["total"] - o0["total"]) / o0["EFG"] < 1e-9
    assert np.abs(G - np.eye(len(G))).max() < 1e-10
    # the start-up itself moves N only at the level of its own truncation
    oi = td.observables(sys_, D.normalize(phi0, lat.dV))
    assert abs(o0["N"] - oi["N"]) / oi["N"] < 1e-6


def test_vortex_imprint_conserves_energy():
    """P10 with a vortex: the complete set of the uniform 6^3 state with the
    vortex imprint (gauge rotation by theta/2 of both components) evolves
    with N and the energy conserved to the integrator's accuracy: the drift
    over t = 0.1 is small and falls with dt at the integrator's order.  (A
    phase put on u alone breaks the partner closure of the E>0 set and the
    energy then drifts by a few percent independently of dt.)"""
    lat = L.Lattice(6, 6, 6)
    mu = 1.0
    E, phi = bdg.eigenstates(np.full(lat.shape, -mu), np.full(lat.shape, 0.5 + 0j), lat)
    pos = E > 0
    E, phi = E[pos], phi[pos]
    phi = bdg.imprint_phase(phi, bdg.vortex_phase(lat, [(0.3, -0.2, 1.0)]))
    lam = F.lambda_c(np.zeros(lat.shape), mu, 0.5 * np.pi ** 2)
    sys_ = td.TDSystem(td.Geometry3D(lat), F.Functional(F.SLDA), mu, np.zeros(lat.shape), lam,
                       F.fermi_weight(E), F.fermi_weight(-E))
    drift = []
    for dt in (0.01, 0.005):
        p, hist, _ = td.start(sys_, phi, dt, "AB4AM5", 1)
        o0 = td.observables(sys_, p)
        for _ in range(int(round(0.1 / dt))):
            p, hist = td.abm_step(sys_, p, hist, dt, "AB4AM5")
        o1 = td.observables(sys_, p)
        assert abs(o1["N"] - o0["N"]) / o0["N"] < 1e-7
        drift.append(abs(o1["total"] - o0["total"]) / o0["EFG"])
    assert drift[1] < 1e-7
    assert drift[0] / drift[1] > 16  # order >= 4


def test_time_reversibility():
    """P14: evolving forward n steps and then n steps with dt -> -dt returns
    to the initial densities within the integrator error."""
    lat, sys_, phi0 = config1_initial()
    phi_f = td.evolve(sys_, phi0, 0.005, 8)
    # both runs take 3 start-up steps + 8 ABM steps
    phi_b = td.evolve(sys_, phi_f, -0.005, 8)
    r0, n0 = D.local_densities(D.normalize(phi0, lat.dV), sys_.wu, sys_.wv)
    r1, n1 = D.local_densities(phi_b, sys_.wu, sys_.wv)
    rf, nf = D.local_densities(phi_f, sys_.wu, sys_.wv)
    # the densities moved by ~5e-4 (rho) and ~1e-2 (nu) relative; the round
    # trip must undo that to the level of the integration error
    drho = np.abs(rf - r0).max()
    dnu = np.abs(nf - n0).max()
    assert drho / np.abs(r0).max() > 1e-4 and dnu / np.abs(n0).max() > 1e-2
    assert np.abs(r1 - r0).max() < 1e-3 * drho
    assert np.abs(n1 - n0).max() < 1e-4 * dnu
