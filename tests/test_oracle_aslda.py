"""Spin-imbalanced ASLDA (Sec. 2.4, ASLDA item; Sec. 2.3) in the quasi-1D
geometry, pinned by: the potentials are the functional derivatives of the
energy density (finite differences), p -> 0 gives the spin-symmetric
general functional's potentials, a balanced complete set of both branches
evolves exactly as the spin-symmetric A = 1.094 path evolves its E > 0
half, and an imbalanced complete set conserves E, N_a and N_b at the
integrator's order (and stops doing so when the polarisation terms of V_s
are dropped)."""
import numpy as np
import pytest

from oracle import aslda as AS, functional as F, td, q1d
from oracle import lattice as L


def _fields(seed, n=12):
    r = np.random.default_rng(seed)
    ra = 0.05 + 0.05 * r.random(n)
    rb = 0.02 + 0.05 * r.random(n)
    ta = 0.3 + 0.2 * r.random(n)
    tb = 0.2 + 0.2 * r.random(n)
    ja = 0.01 * r.standard_normal(n)
    jb = 0.01 * r.standard_normal(n)
    nu = 0.03 * (r.standard_normal(n) + 1j * r.standard_normal(n))
    lam = 0.05 + 0.02 * r.random(n)
    return ra, rb, ta, tb, ja, jb, nu, lam


def test_derivatives_of_A_and_B():
    p = np.linspace(-0.9, 0.9, 13)
    h = 1e-6
    assert np.allclose(AS.dA_dp(p), (AS.A_of_p(p + h) - AS.A_of_p(p - h)) / (2 * h), atol=1e-8)
    assert np.allclose(AS.dB_dp(p), (AS.B_of_p(p + h) - AS.B_of_p(p - h)) / (2 * h), atol=1e-8)
    assert AS.A_of_p(0.0) == pytest.approx(1.094) and AS.dB_dp(0.0) == pytest.approx(0.0, abs=1e-15)


def test_potentials_are_functional_derivatives():
    ra, rb, ta, tb, ja, jb, nu, lam = _fields(3)
    Va, Vb, D, Aa, Ab, Ava, Avb = AS.potentials(ra, rb, ta, tb, [ja], [jb], nu, lam)
    e = lambda *a: AS.energy_density(*a)
    h = 1e-7

    def fd(k):
        args = [ra, rb, ta, tb, ja, jb, nu]
        up = [x.copy() for x in args]
        dn = [x.copy() for x in args]
        up[k] = up[k] + h
        dn[k] = dn[k] - h
        f = lambda a: e(a[0], a[1], a[2], a[3], [a[4]], [a[5]], a[6], lam)
        return (f(up) - f(dn)) / (2 * h)
    assert np.allclose(Va, fd(0), rtol=1e-6, atol=1e-8)
    assert np.allclose(Vb, fd(1), rtol=1e-6, atol=1e-8)
    assert np.allclose(Aa, 2 * fd(2), rtol=1e-7)
    assert np.allclose(Ab, 2 * fd(3), rtol=1e-7)
    assert np.allclose(Ava[0], fd(4), rtol=1e-6, atol=1e-9)
    assert np.allclose(Avb[0], fd(5), rtol=1e-6, atol=1e-9)
    # Delta = -dE/dnu^*: dE/dRe nu = 2 Re(dE/dnu^*) for a real E
    dre = fd(6)
    args = [ra, rb, ta, tb, ja, jb]
    dim = (AS.energy_density(*args[:4], [ja], [jb], nu + 1j * h, lam)
           - AS.energy_density(*args[:4], [ja], [jb], nu - 1j * h, lam)) / (2 * h)
    assert np.allclose(-0.5 * (dre + 1j * dim), D, rtol=1e-6, atol=1e-10)


def test_balanced_limit_is_the_spin_symmetric_general_functional():
    ra, rb, ta, tb, ja, jb, nu, lam = _fields(5)
    Va, Vb, D, Aa, Ab, Ava, Avb = AS.potentials(ra, ra, ta, ta, [ja], [ja], nu, lam)
    fun = F.Functional(F.SLDA, force_a1=False)
    U, D2, al, av = F.potentials_general(ra, nu, [0 * ja, 0 * ja, ja], lam, fun)
    assert np.allclose(Va, U, rtol=1e-13) and np.allclose(Vb, U, rtol=1e-13)
    assert np.allclose(D, D2, rtol=1e-14) and np.allclose(Aa, al) and np.allclose(Ab, al)
    assert np.allclose(Ava[0], av[2], rtol=1e-13) and np.allclose(Avb[0], av[2], rtol=1e-13)


def _geom():
    return q1d.GeometryQ1D(16, 1.0, 2, 2, 1.7)


def _trap(geom):
    z = L.centered_coords(geom.nz, geom.dz)
    return 0.5 * 0.12 ** 2 * z ** 2


def test_balanced_complete_set_evolves_as_the_spin_symmetric_half():
    geom = _geom()
    vext = _trap(geom)
    mu = 0.9
    delta = 0.4 + 0.05 * np.cos(np.arange(16) * 0.7)
    ec = 1e9
    E, kp2, phi = AS.eigenstates_imbalanced(geom, vext - mu, vext - mu, delta, ec)
    lam = F.lambda_c(vext, mu, 0.5 * np.pi ** 2, A=1.094)
    sg = AS.SpinGeometryQ1D(geom)
    sg.set_states(kp2)
    sysa = AS.ASLDASystem(sg, mu, mu, vext, lam, F.fermi_weight(E), F.fermi_weight(-E))
    pa = td.evolve(sysa, phi, 0.01, 6)
    pos = E > 0
    g2 = _geom()
    g2.set_states(kp2[pos])
    syss = td.TDSystem(g2, F.Functional(F.SLDA, force_a1=False), mu, vext, lam,
                       F.fermi_weight(E[pos]), F.fermi_weight(-E[pos]))
    ps = td.evolve(syss, phi[pos], 0.01, 6)
    ra, rb, ta, tb, nu, ja, jb = sg.densities(pa, sysa.wu, sysa.wv)
    r, t, n, j = g2.full_densities(ps, syss.wu, syss.wv)
    for a, b in ((ra, r), (rb, r), (ta, t), (tb, t), (nu, n), (ja, j[2]), (jb, j[2])):
        assert np.abs(a - b).max() < 1e-12 * max(1.0, np.abs(b).max())
    assert np.abs(ra - sg.densities(phi, sysa.wu, sysa.wv)[0]).max() > 1e-5  # it moved


def _imbalanced(dt, nsteps, tau_form="laplacian"):
    geom = _geom()
    vext = _trap(geom)
    mu_a, mu_b = 1.3, 0.5  # Zeeman split 0.4 above the gap: polarised
    delta = 0.15 + 0.05 * np.sin(np.arange(16) * 0.9)
    E, kp2, phi = AS.eigenstates_imbalanced(geom, vext - mu_a, vext - mu_b, delta, 1e9)
    lam = F.lambda_c(vext, 0.5 * (mu_a + mu_b), 0.5 * np.pi ** 2, A=1.094)
    sg = AS.SpinGeometryQ1D(geom)
    sg.set_states(kp2)
    sysa = AS.ASLDASystem(sg, mu_a, mu_b, vext - 0.02 * L.centered_coords(16, 1.0), lam,
                          F.fermi_weight(E), F.fermi_weight(-E), tau_form=tau_form)
    o0 = sysa.observables(sysa.normalize(phi))
    p = td.evolve(sysa, phi, dt, nsteps)
    return o0, sysa.observables(p), sg.densities(p, sysa.wu, sysa.wv)


def test_imbalanced_complete_set_conserves_energy_and_particle_numbers(monkeypatch):
    o0, o1, d = _imbalanced(0.01, 40)
    ra, rb = d[0], d[1]
    p = (ra - rb) / (ra + rb)
    assert p.max() > 0.2  # polarised
    o0h, o1h, _ = _imbalanced(0.005, 80)
    for k in ("E", "Na", "Nb"):  # conserved to the integrator's accuracy and order
        e1, e2 = abs(o1[k] - o0[k]), abs(o1h[k] - o0h[k])
        assert e1 < 1e-7 * abs(o0[k]) and e2 < e1 / 8, (k, e1, e2)
    err2 = abs(o1h["E"] - o0h["E"])
    # with the paper's gradient form of tau the particle numbers are kept
    # the same way and the energy up to the lattice difference of the two
    # forms (independent of dt)
    g0, g1, _ = _imbalanced(0.01, 40, "gradient")
    for k in ("Na", "Nb"):
        assert abs(g1[k] - g0[k]) < 1e-7 * g0[k]
    assert abs(g1["E"] - g0["E"]) < 1e-4 * abs(g0["E"])
    # without the polarisation terms of V_s (a planted mistake in the oracle)
    monkeypatch.setattr(AS, "dA_dp", lambda q: 0.0 * q)
    monkeypatch.setattr(AS, "dB_dp", lambda q: 0.0 * q)
    ob0, ob1, _ = _imbalanced(0.005, 80)
    assert abs(ob1["E"] - ob0["E"]) > 100 * err2


def test_3d_evolution_of_product_states_is_the_quasi_1d_one():
    """3D ASLDA on product states exp(i k_perp . r_perp) phi(z) / sqrt(L_x L_y)
    of a complete polarised quasi-1D set (fields depending on z only)
    reproduces the quasi-1D ASLDA evolution: spin-resolved densities, tau,
    nu, j and the energy (exact mode reduction, Sec. 3.1)."""
    nz, nxy, dxy = 8, 4, 2.0
    geom = q1d.GeometryQ1D(nz, 1.0, nxy, nxy, dxy)
    lat = L.Lattice(nxy, nxy, nz, dxy, dxy, 1.0)
    z = L.centered_coords(nz, 1.0)
    vext = 0.5 * 0.2 ** 2 * z ** 2 - 0.03 * z
    mu_a, mu_b = 1.3, 0.5
    delta = 0.15 + 0.05 * np.sin(np.arange(nz) * 0.9)
    E, kp2, phi1 = AS.eigenstates_imbalanced(geom, vext - mu_a, vext - mu_b, delta, 1e9)
    probs = geom.problems()
    per = 2 * nz  # eigenpairs per problem (complete set)
    x = np.arange(nxy) * dxy
    phi3 = np.empty((len(E), 2) + lat.shape, complex)
    for n in range(len(E)):
        ix, iy = probs[n // per][1]
        pw = np.exp(1j * (geom.kx[ix] * x[:, None] + geom.ky[iy] * x[None, :])) / np.sqrt(geom.area)
        phi3[n] = pw[None, :, :, None] * phi1[n][:, None, None, :]
    lam = F.lambda_c(vext, 0.5 * (mu_a + mu_b), 0.5 * np.pi ** 2, A=1.094)
    wu, wv = F.fermi_weight(E), F.fermi_weight(-E)
    s1g = AS.SpinGeometryQ1D(geom)
    s1g.set_states(kp2)
    s1 = AS.ASLDASystem(s1g, mu_a, mu_b, vext, lam, wu, wv)
    b = lambda f: np.broadcast_to(f, lat.shape).copy()
    s3 = AS.ASLDASystem(AS.SpinGeometry3D(lat), mu_a, mu_b, b(vext), b(lam), wu, wv)
    p1 = td.evolve(s1, phi1, 0.01, 5)
    p3 = td.evolve(s3, phi3, 0.01, 5)
    d1 = s1g.densities(p1, wu, wv)
    d3 = s3.geom.densities(p3, wu, wv)
    for k in range(5):
        assert np.abs(d3[k] - b(d1[k])).max() < 1e-11 * max(1.0, np.abs(d1[k]).max()), k
    assert np.abs(d3[5][2] - b(d1[5])).max() < 1e-11 and np.abs(d3[6][2] - b(d1[6])).max() < 1e-11
    assert max(np.abs(d3[5][0]).max(), np.abs(d3[6][1]).max()) < 1e-12
    assert ((d1[0] - d1[1]) / (d1[0] + d1[1])).max() > 0.2  # polarised
    assert s1.observables(p1)["E"] == pytest.approx(s3.observables(p3)["E"], rel=1e-11)
