"""Parity of the quasi-1D (batched reduced-dimension) kernel set with the
oracle's quasi-1D mode (Sec. 3.1): many independent 1D BdG problems, one per
transverse momentum, with uneven state counts after the energy cut-off."""
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


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def problem(nz, nk, dperp, ec, seed):
    geom = q1d.GeometryQ1D(nz, 1.0, nk, nk, dperp)
    z = L.centered_coords(nz, 1.0)
    mu = 1.0
    vb, wb, zb = synth.gaussian_bump(seed)
    zb = zb * nz / 256.0
    vext = 0.5 * (0.0175 * 256 / nz) ** 2 * z ** 2 + vb * np.exp(-(z - zb) ** 2 / (2 * wb ** 2))
    delta = np.full(nz, 0.5 + 0j)
    E, kp2, pid, phi = q1d.eigenstates(geom, vext - mu, delta, ec=ec)
    geom.set_states(kp2)
    return geom, mu, vext, E, kp2, pid, phi


def make_ctx(geom, mu, ecreg, n, prec=0, dt=0.005):
    from paper_2602_08982_amd import tdslda as T
    lat = T.lattice_q1d(geom.nz, geom.dz, geom.Lx, geom.Ly)
    return T.Context(lat, T.functional_slda(mu, ecreg), T.run_config(precision=prec, dt=dt), n)


@pytest.mark.parametrize("nz,nk,dperp,ec", [(16, 8, 1.0, None), (64, 6, 1.3, 6.0), (256, 4, 2.0, 4.0)])
@pytest.mark.parametrize("prec", [0, 1])
def test_q1d_td(nz, nk, dperp, ec, prec):
    geom, mu, vext, E, kp2, pid, phi = problem(nz, nk, dperp, ec, seed=3)
    counts = np.bincount(pid)
    ecreg = 0.5 * np.pi ** 2 if ec is None else ec
    lam = F.lambda_c(vext, mu, ecreg)
    # the bump is removed at t = 0
    z = L.centered_coords(nz, 1.0)
    v0 = 0.5 * (0.0175 * 256 / nz) ** 2 * z ** 2
    sysm = td.TDSystem(geom, F.Functional(F.SLDA), mu, v0, lam, F.fermi_weight(E), F.fermi_weight(-E))
    ref = td.evolve(sysm, phi, 0.005, 10)
    ctx = make_ctx(geom, mu, ecreg, len(E), prec)
    ctx.set_external(v0, freeze_regulator=False)
    ctx.set_regulator(lam)
    ctx.load_states(phi, E, kp2)
    ctx.abm_step(10)
    d = ctx.densities()
    r, t_, n, j = geom.full_densities(ref, sysm.wu, sysm.wv)
    tol = 1e-10 if prec == 0 else 1e-5
    assert rel(d["rho"], r) < tol
    assert rel(d["nu"], n) < tol
    assert rel(d["tau"], t_) < tol
    assert np.abs(d["j"][2] - j[2]).max() < tol * np.abs(t_).max()
    e = ctx.energy()
    o = td.observables(sysm, ref)
    for k in ("kin", "pot", "pair", "potext", "N", "total"):
        sc = abs(o[k]) if o[k] != 0 else o["EFG"]  # each term against its own size
        assert abs(e[k] - o[k]) / sc < tol, (k, e[k], o[k])
    if prec == 0:
        assert np.abs(ctx.get_states() - ref).max() < 1e-9
    ctx.close()


def test_q1d_apply_hbdg():
    geom, mu, vext, E, kp2, pid, phi = problem(64, 4, 1.0, 5.0, seed=5)
    U = synth.uniform_field(9, 64, -0.3, 0.3)
    delta = synth.complex_normal(10, 64, 0.3)
    x = synth.complex_normal(11, phi.shape)
    ref = geom.apply_h(x, U + vext - mu, delta)
    ctx = make_ctx(geom, mu, 5.0, len(E))
    ctx.set_external(vext, freeze_regulator=True)
    ctx.load_states(phi, E, kp2)
    ctx.set_fields(U, delta)
    xd = torch.from_numpy(x.reshape(len(E), 2, -1)).cuda()
    yd = torch.zeros_like(xd)
    ctx.apply_hbdg(xd, yd, len(E))
    torch.cuda.synchronize()
    out = yd.cpu().numpy().reshape(x.shape)
    assert np.abs(out - ref).max() / np.abs(ref).max() < 1e-12
    ctx.close()


def test_q1d_many_states_parity():
    """2,304 problems of N_z = 16 (36,864 states: more than 64 state groups,
    so the per-site reduction takes the one-workgroup-per-site path and the
    graph-free hot path uses the transform-free density pass): densities and
    states after 5 steps against the oracle to 1e-10 (FP64)."""
    geom, mu, vext, E, kp2, pid, phi = problem(16, 48, 1.0, None, seed=4)
    assert len(E) > 64 * 512
    ecreg = 0.5 * np.pi ** 2
    lam = F.lambda_c(vext, mu, ecreg)
    z = L.centered_coords(16, 1.0)
    v0 = 0.5 * (0.0175 * 16) ** 2 * z ** 2
    sysm = td.TDSystem(geom, F.Functional(F.SLDA), mu, v0, lam, F.fermi_weight(E), F.fermi_weight(-E))
    ref = td.evolve(sysm, phi, 0.005, 5)
    ctx = make_ctx(geom, mu, ecreg, len(E), 0)
    try:
        ctx.set_external(v0, freeze_regulator=False)
        ctx.set_regulator(lam)
        ctx.load_states(phi, E, kp2)
        ctx.abm_step(5)
        d = ctx.densities()
        r, t_, n, j = geom.full_densities(ref, sysm.wu, sysm.wv)
        assert rel(d["rho"], r) < 1e-10
        assert rel(d["nu"], n) < 1e-10
        assert np.abs(ctx.get_states() - ref).max() < 1e-9
    finally:
        ctx.close()
