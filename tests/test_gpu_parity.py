"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

FP64 bar: 1e-10 relative on densities and energies after TD steps, 1e-12 on
single operator applications; FP32-mixed bar: 1e-5 relative.
"""
import numpy as np
import pytest

from oracle import lattice as L, bdg, densities as D, functional as F, td, uniform as UN
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    torch.cuda.set_device(0)
    from paper_2602_08982_amd import tdslda
    tdslda.load_library()


def T():
    from paper_2602_08982_amd import tdslda
    return tdslda


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def make_ctx(lat, mu, ec, n, precision=0, integrator=45, dt=0.005, selfstart=1, **kw):
    t = T()
    lt = t.Lattice(t.MODE_3D, *lat.n, *lat.d, 0.0, 0.0)
    run = t.run_config(precision=precision, integrator=integrator, dt=dt, selfstart=selfstart, **kw)
    return t.Context(lt, t.functional_slda(mu, ec), run, n)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape,nst", [((8, 8, 8), 37), ((12, 12, 12), 5), ((6, 6, 6), 3),
                                       ((8, 8, 16), 4), ((32, 32, 32), 3), ((48, 48, 48), 2)])
@pytest.mark.parametrize("prec", [0, 1])
def test_apply_hbdg(shape, nst, prec):
    """H psi through tdslda_apply_hbdg equals the oracle's spectral
    operator (Eq. HpsiEpsi with Eq. h_sigma_A1) on random states and fields."""
    lat = L.Lattice(*shape, 1.0, 0.9 if shape[1] != shape[0] else 1.0, 1.1 if shape[2] != shape[0] else 1.0)
    mu = 0.7
    U = synth.uniform_field(1, lat.shape, -0.5, 0.5)
    delta = synth.complex_normal(2, lat.shape, 0.3)
    phi = synth.complex_normal(3, (nst, 2) + lat.shape)
    ref = bdg.apply_h(phi, U - mu, delta, lat)
    ctx = make_ctx(lat, mu, 0.5 * np.pi ** 2, nst, precision=prec)
    ctx.set_fields(U, delta)
    cdt = torch.complex128 if prec == 0 else torch.complex64
    x = torch.from_numpy(phi.reshape(nst, 2, -1)).to(cdt).cuda()
    y = torch.zeros_like(x)
    ctx.apply_hbdg(x, y, nst)
    torch.cuda.synchronize()
    out = y.cpu().numpy().astype(np.complex128).reshape(phi.shape)
    tol = 1e-12 if prec == 0 else 3e-6
    err = np.abs(out - ref).max() / np.abs(ref).max()
    assert err < tol, err
    ctx.close()


@pytest.mark.parametrize("shape,nst", [((8, 8, 8), 70), ((12, 12, 12), 33), ((16, 16, 16), 6)])
def test_densities(shape, nst):
    """rho, tau, nu, j of normalised random states with both signs of E
    (frozen T=0 weights) against the oracle (Eqs. nab3D-jab3D)."""
    lat = L.Lattice(*shape)
    phi = synth.complex_normal(7, (nst, 2) + lat.shape)
    E = synth.uniform_field(8, nst, -2.0, 2.0)
    ctx = make_ctx(lat, 1.0, 0.5 * np.pi ** 2, nst)
    ctx.load_states(phi, E)
    d = ctx.densities()
    ph = D.normalize(phi, lat.dV)
    rho, tau, nu, j = D.spin_symmetric(ph, F.fermi_weight(E), F.fermi_weight(-E), lat)
    assert rel(d["rho"], rho) < 1e-13
    assert rel(d["tau"], tau) < 1e-13
    assert rel(d["nu"], nu) < 1e-13
    for c in range(3):
        assert np.abs(d["j"][c] - j[c]).max() < 1e-13 * np.abs(tau).max()
    st = ctx.get_states()
    assert np.abs(st - ph).max() < 1e-14
    ctx.close()


# ---------------------------------------------------------------------------
def config1(seed=0):
    lat = L.Lattice(8, 8, 8)
    mu, ec = 1.0, 0.5 * np.pi ** 2
    eta = synth.uniform_field(seed, lat.shape)
    E, phi = bdg.eigenstates(np.full(lat.shape, -mu), 0.5 * np.exp(1j * 0.01 * eta), lat)
    pos = E > 0
    lam = F.lambda_c(np.zeros(lat.shape), mu, ec)
    sysm = td.TDSystem(td.Geometry3D(lat), F.Functional(F.SLDA), mu, np.zeros(lat.shape), lam,
                       F.fermi_weight(E[pos]), F.fermi_weight(-E[pos]))
    return lat, mu, ec, E[pos], phi[pos], sysm


@pytest.fixture(scope="module")
def config1_ref():
    lat, mu, ec, E, phi, sysm = config1()
    out = {}

    def cb(step, p):
        if step in (1, 5, 20):
            out[step] = (p.copy(), td.observables(sysm, p))
    td.evolve(sysm, phi, 0.005, 20, callback=cb)
    return lat, mu, ec, E, phi, sysm, out


@pytest.mark.parametrize("prec", [0, 1])
def test_config1_td(config1_ref, prec):
    """Config-1 workload (8^3, all 1024 states, 512 evolved, Taylor start-up
    + 20 AB4AM5 steps at dt = 0.005): densities and energy terms after 1, 5
    and 20 steps against the oracle; FP64 to 1e-10, FP32-mixed to 1e-5."""
    lat, mu, ec, E, phi, sysm, ref = config1_ref
    ctx = make_ctx(lat, mu, ec, len(E), precision=prec)
    ctx.set_external(np.zeros(lat.shape), freeze_regulator=True)
    ctx.load_states(phi, E)
    done = 0
    tol = 1e-10 if prec == 0 else 1e-5
    for step in (1, 5, 20):
        ctx.abm_step(step - done)
        done = step
        p_ref, o_ref = ref[step]
        d = ctx.densities()
        r, t_, n, j = D.spin_symmetric(p_ref, sysm.wu, sysm.wv, lat)
        assert rel(d["rho"], r) < tol
        assert rel(d["nu"], n) < tol
        assert rel(d["tau"], t_) < tol
        e = ctx.energy()
        for k in ("kin", "pot", "pair", "N", "total"):
            # each term against its own size (E_FG only for a term that is exactly zero)
            sc = abs(o_ref[k]) if o_ref[k] != 0 else o_ref["EFG"]
            assert abs(e[k] - o_ref[k]) / sc < tol, (k, e[k], o_ref[k])
        if prec == 0:
            st = ctx.get_states()
            assert np.abs(st - p_ref).max() < 1e-9
    ctx.close()


@pytest.mark.parametrize("scheme,code", [("AB3AM4", 34), ("AB4AM5", 45), ("AB5AM5", 55)])
@pytest.mark.parametrize("selfstart", [0, 1])
def test_linear_mode_schemes(scheme, code, selfstart):
    """Frozen fields (linear mode): every integrator and both start-ups
    against the oracle's integrator on the same frozen operator."""
    lat = L.Lattice(6, 6, 6, 1.2, 1.2, 1.2)
    mu = 0.3
    U = synth.uniform_field(11, lat.shape, -0.3, 0.3)
    delta = synth.complex_normal(12, lat.shape, 0.3)
    nst = 9
    phi = D.normalize(synth.complex_normal(13, (nst, 2) + lat.shape), lat.dV)
    sysl = td.TDSystem(td.Geometry3D(lat), None, mu, np.zeros(lat.shape), np.zeros(lat.shape),
                       np.zeros(nst), np.ones(nst), frozen=(U - mu, delta))
    ref = td.evolve(sysl, phi, 0.01, 12, scheme=scheme, selfstart=selfstart)
    ctx = make_ctx(lat, mu, 10.0, nst, integrator=code, dt=0.01, selfstart=selfstart)
    ctx.load_states(phi, np.ones(nst))
    ctx.set_fields(U, delta)
    ctx.abm_step(5)
    ctx.abm_step(7)   # a second call resumes from the canonical history
    st = ctx.get_states()
    assert np.abs(st - ref).max() < 1e-11
    ctx.close()


def test_plane_waves_and_vortex():
    """Uniform-system start and vortex imprint generated on the device equal
    the oracle's plane-wave states times exp(i theta) on u."""
    lat = L.Lattice(12, 12, 12)
    mu, u0, d0 = 1.0, 0.1, 0.5
    kidx = np.array(np.meshgrid(*[range(n) for n in lat.n], indexing="ij")).reshape(3, -1).T
    sel = kidx[::7]
    E, phi = bdg.plane_wave_states(lat, sel, u0 - mu, d0)
    vort = [(0.37, -0.61, 1.0), (-2.1, 1.3, -1.0)]
    phi = bdg.imprint_phase(phi, bdg.vortex_phase(lat, vort))
    ctx = make_ctx(lat, mu, 0.5 * np.pi ** 2, len(sel))
    ctx.init_plane_waves(sel, u0, d0)
    ctx.imprint_vortices(vort)
    st = ctx.get_states()
    assert np.abs(st - phi).max() < 1e-13
    ctx.close()


def test_uniform_state_is_stationary():
    """P8 on the device: the self-consistent uniform state (all k, T=0) does
    not move over 20 steps."""
    lat = L.Lattice(8, 8, 8)
    fun = F.Functional(F.SLDA)
    mu, ec = 1.0, 0.5 * np.pi ** 2
    lam = float(F.lambda_c(0.0, mu, ec))
    U, d = UN.lattice_uniform(lat, fun, mu, lam)
    kidx = np.array(np.meshgrid(*[range(n) for n in lat.n], indexing="ij")).reshape(3, -1).T
    E, phi = bdg.plane_wave_states(lat, kidx, U - mu, d)
    ctx = make_ctx(lat, mu, ec, len(E))
    ctx.set_external(np.zeros(lat.shape), freeze_regulator=True)
    ctx.init_plane_waves(kidx, U, d)
    ctx.abm_step(20)
    st = ctx.get_states()
    assert np.abs(st - phi).max() < 1e-12
    ctx.close()


def test_checkpoint_resume_is_bit_exact(tmp_path):
    lat, mu, ec, E, phi, sysm = config1()
    a = make_ctx(lat, mu, ec, len(E))
    a.set_external(np.zeros(lat.shape), freeze_regulator=True)
    a.load_states(phi, E)
    a.abm_step(3)
    a.save(str(tmp_path / "ck.bin"))
    a.abm_step(4)
    sa = a.get_states()
    b = make_ctx(lat, mu, ec, len(E))
    b.set_external(np.zeros(lat.shape), freeze_regulator=True)
    b.load(str(tmp_path / "ck.bin"))
    b.abm_step(4)
    sb = b.get_states()
    assert np.array_equal(sa, sb)
    assert a.info()[1:] == b.info()[1:]
    a.close()
    b.close()


def test_failure_detection():
    """Sec. 4.5.1 diagnostics forced from the host: a zero-width tolerance,
    an unstable time step and a NaN in a state all return EUNSTABLE; calls
    out of order return EORDER."""
    t = T()
    lat, mu, ec, E, phi, sysm = config1()
    c = make_ctx(lat, mu, ec, len(E), tol_N=1e-300, tol_E=0.0)
    with pytest.raises(t.TdsldaError) as ei:
        c.abm_step(1)
    assert ei.value.status == t.EORDER
    c.set_external(np.zeros(lat.shape), freeze_regulator=True)
    c.load_states(phi, E)
    st, _ = c.check()          # first check records N0, E0
    assert st == t.OK
    c.abm_step(2)
    st, info = c.check()
    assert st == t.EUNSTABLE and info["dN"] > 0
    c.close()
    c = make_ctx(lat, mu, ec, len(E), dt=0.5, tol_N=1e-6, tol_E=1e-6)
    c.set_external(np.zeros(lat.shape), freeze_regulator=True)
    c.load_states(phi, E)
    c.check()
    c.abm_step(30)
    st, info = c.check()
    assert st == t.EUNSTABLE
    c.close()
    bad = phi.copy()
    bad[3, 0, 1, 2, 3] = np.nan
    c = make_ctx(lat, mu, ec, len(E), tol_N=1e-6, tol_E=1e-6)
    c.load_states(bad, E)
    st, _ = c.check()
    assert st == t.EUNSTABLE
    c.close()
