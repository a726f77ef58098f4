"""External pairing potential Delta_ext through tdslda_set_external (Sec. 2.2,
Eq. E_tot; Sec. 2.3, Eq. HpsiEpsi): the device evolution with Delta +
Delta_ext in H and the external pairing energy against the oracle, in 3D
(self-consistent and linear mode) and in the quasi-1D kernel set; the
conservation check follows E - mu N.  FP64 bar 1e-10, FP32-mixed 1e-5."""
import numpy as np
import pytest

from oracle import lattice as L, bdg, densities as D, functional as F, td, q1d
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    torch.cuda.set_device(0)


def T():
    from paper_2602_08982_amd import tdslda
    return tdslda


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _config(seed=50):
    lat = L.Lattice(8, 8, 8)
    mu, ec = 1.0, 0.5 * np.pi ** 2
    eta = synth.uniform_field(seed, lat.shape)
    E, phi = bdg.eigenstates(np.full(lat.shape, -mu), 0.5 * np.exp(1j * 0.02 * eta), lat)
    pos = E > 0
    lam = F.lambda_c(np.zeros(lat.shape), mu, ec)
    dext = 0.05 * synth.complex_normal(seed + 1, lat.shape)
    sysm = td.TDSystem(td.Geometry3D(lat), F.Functional(F.SLDA), mu, np.zeros(lat.shape), lam,
                       F.fermi_weight(E[pos]), F.fermi_weight(-E[pos]), dext=dext)
    return lat, mu, ec, E[pos], phi[pos], dext, sysm


@pytest.fixture(scope="module")
def config_ref():
    lat, mu, ec, E, phi, dext, sysm = _config()
    out = {}

    def cb(step, p):
        if step in (2, 6):
            out[step] = (p.copy(), td.observables(sysm, p))
    td.evolve(sysm, phi, 0.005, 6, callback=cb)
    return lat, mu, ec, E, phi, dext, sysm, out


@pytest.mark.parametrize("prec", [0, 1])
def test_dext_selfconsistent(config_ref, prec):
    lat, mu, ec, E, phi, dext, sysm, ref = config_ref
    t = T()
    ctx = t.Context(t.lattice_3d((8, 8, 8)), t.functional_slda(mu, ec), t.run_config(precision=prec), len(E))
    try:
        ctx.set_external(np.zeros(lat.shape), freeze_regulator=True, dext=dext)
        ctx.load_states(phi, E)
        tol = 1e-10 if prec == 0 else 1e-5
        done = 0
        for step in (2, 6):
            ctx.abm_step(step - done)
            done = step
            p_ref, o = ref[step]
            d = ctx.densities()
            r, t_, n, j = D.spin_symmetric(p_ref, sysm.wu, sysm.wv, lat)
            assert rel(d["rho"], r) < tol
            assert rel(d["nu"], n) < tol
            e = ctx.energy()
            for k in ("kin", "pot", "pair", "N", "total"):
                assert abs(e[k] - o[k]) <= tol * abs(o[k]), (k, e[k], o[k])
            # E_pair.ext = -2 Re int Delta_ext nu^* sums terms of random
            # phase that largely cancel: its bar is relative to the size of
            # the integrand, 2 int |Delta_ext| |nu|, which bounds the error
            # a relative error of nu of tol can cause
            scale = 2.0 * lat.dV * np.sum(np.abs(dext) * np.abs(n))
            assert abs(e["pairext"] - o["pairext"]) <= tol * scale, (e["pairext"], o["pairext"], scale)
            if prec == 0:
                assert np.abs(ctx.get_states() - p_ref).max() < 1e-9
        # Delta_ext changes N
        r0, n0 = D.local_densities(D.normalize(phi, lat.dV), sysm.wu, sysm.wv)
        assert abs(np.sum(d["rho"]) - np.sum(r0)) / np.sum(r0) > 1e-6
    finally:
        ctx.close()


def test_dext_check_follows_omega():
    """tdslda_check with tight tolerances passes on the Delta_ext evolution
    (Omega = E - mu N conserved, N not checked)."""
    lat, mu, ec, E, phi, dext, sysm = _config()
    t = T()
    ctx = t.Context(t.lattice_3d((8, 8, 8)), t.functional_slda(mu, ec),
                    t.run_config(precision=0, tol_N=1e-12, tol_E=1e-8), len(E))
    try:
        ctx.set_external(np.zeros(lat.shape), freeze_regulator=True, dext=dext)
        ctx.load_states(phi, E)
        ctx.abm_step(3)
        st, _ = ctx.check()
        assert st == t.OK
        ctx.abm_step(10)
        st, info = ctx.check()
        assert st == t.OK, info
        assert info["dN"] == 0.0 and info["dE"] < 1e-8
    finally:
        ctx.close()


def test_dext_linear_mode():
    """Frozen U, Delta plus Delta_ext: H uses Delta + Delta_ext."""
    lat = L.Lattice(6, 6, 6, 1.1, 1.1, 1.1)
    mu = 0.3
    U = synth.uniform_field(61, lat.shape, -0.3, 0.3)
    delta = synth.complex_normal(62, lat.shape, 0.3)
    dext = synth.complex_normal(63, lat.shape, 0.1)
    nst = 7
    phi = D.normalize(synth.complex_normal(64, (nst, 2) + lat.shape), lat.dV)
    sysl = td.TDSystem(td.Geometry3D(lat), None, mu, np.zeros(lat.shape), np.zeros(lat.shape),
                       np.zeros(nst), np.ones(nst), frozen=(U - mu, delta), dext=dext)
    ref = td.evolve(sysl, phi, 0.01, 8)
    t = T()
    lt = t.Lattice(t.MODE_3D, *lat.n, *lat.d, 0.0, 0.0)
    ctx = t.Context(lt, t.functional_slda(mu, 10.0), t.run_config(dt=0.01), nst)
    try:
        ctx.set_external(np.zeros(lat.shape), freeze_regulator=False, dext=dext)
        ctx.load_states(phi, np.ones(nst))
        ctx.set_fields(U, delta)
        ctx.abm_step(8)
        assert np.abs(ctx.get_states() - ref).max() < 1e-11
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_dext_q1d(prec):
    """Quasi-1D kernel set (N_z = 64, 6 x 6 transverse momenta) with a
    Delta_ext(z) profile: densities, energy terms and states vs the oracle."""
    nz, nk, dperp, ec = 64, 6, 1.3, 6.0
    geom = q1d.GeometryQ1D(nz, 1.0, nk, nk, dperp)
    z = L.centered_coords(nz, 1.0)
    mu = 1.0
    vext = 0.5 * (0.0175 * 4) ** 2 * z ** 2
    E, kp2, pid, phi = q1d.eigenstates(geom, vext - mu, np.full(nz, 0.5 + 0j), ec=ec)
    geom.set_states(kp2)
    lam = F.lambda_c(vext, mu, ec)
    dext = 0.04 * np.exp(-(z / 10.0) ** 2) * np.exp(0.3j)
    sysm = td.TDSystem(geom, F.Functional(F.SLDA), mu, vext, lam, F.fermi_weight(E), F.fermi_weight(-E),
                       dext=dext)
    ref = td.evolve(sysm, phi, 0.005, 8)
    t = T()
    ctx = t.Context(t.lattice_q1d(nz, 1.0, geom.Lx, geom.Ly), t.functional_slda(mu, ec),
                    t.run_config(precision=prec), len(E))
    try:
        ctx.set_external(vext, freeze_regulator=False, dext=dext)
        ctx.set_regulator(lam)
        ctx.load_states(phi, E, kp2)
        ctx.abm_step(8)
        d = ctx.densities()
        r, t_, n, j = geom.full_densities(ref, sysm.wu, sysm.wv)
        tol = 1e-10 if prec == 0 else 1e-5
        assert rel(d["rho"], r) < tol
        assert rel(d["nu"], n) < tol
        e = ctx.energy()
        o = td.observables(sysm, ref)
        for k in ("kin", "pot", "pair", "pairext", "N", "total"):
            assert abs(e[k] - o[k]) <= tol * abs(o[k]), (k, e[k], o[k])
        if prec == 0:
            assert np.abs(ctx.get_states() - ref).max() < 1e-9
    finally:
        ctx.close()
