"""Parity of the general-functional (A != 1) quasi-1D path with the oracle:
the operator of Eq. h_sigma with the symmetrised kinetic term of Eq.
kinop-alpha and the current-potential anticommutator (Eqs. Ad_dx, d_dxA),
in linear mode with spatially varying alpha and A_z, and the self-consistent
SLDA evolution at A = 1.094 (alpha = A, A_z = (1 - A) j / rho, the current
term of U, the regulator with A) of current-carrying states.

Bars: FP64 1e-10 relative (operator 1e-12), FP32-mixed 1e-5 relative;
energy terms relative to their own magnitude."""
import numpy as np
import pytest

from oracle import lattice as L, functional as F, td, q1d
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


def problem(nz, nk, dperp, ec, seed, boost=2):
    """Static states of a trapped quasi-1D problem with a bump (A = 1
    diagonalisation), given a pair momentum by the gauge rotation
    u <- e^{i q z / 2} u, v <- e^{-i q z / 2} v with q = 2 pi boost / L
    (boost even: periodic), so that the evolution carries currents."""
    geom = q1d.GeometryQ1D(nz, 1.0, nk, nk, dperp)
    z = L.centered_coords(nz, 1.0)
    mu = 1.0
    vb, wb, zb = synth.gaussian_bump(seed)
    zb = zb * nz / 256.0
    vext = 0.5 * (0.0175 * 256 / nz) ** 2 * z ** 2 + vb * np.exp(-(z - zb) ** 2 / (2 * wb ** 2))
    E, kp2, pid, phi = q1d.eigenstates(geom, vext - mu, np.full(nz, 0.5 + 0j), ec=ec)
    geom.set_states(kp2)
    th = np.pi * boost * np.arange(nz) / nz
    phi = phi.copy()
    phi[:, 0] *= np.exp(1j * th)
    phi[:, 1] *= np.exp(-1j * th)
    v0 = 0.5 * (0.0175 * 256 / nz) ** 2 * z ** 2
    return geom, mu, vext, v0, E, kp2, phi


def make_ctx(geom, mu, ecreg, n, prec, A=1.0, dt=0.005):
    from paper_2602_08982_amd import tdslda as T
    lat = T.lattice_q1d(geom.nz, geom.dz, geom.Lx, geom.Ly)
    return T.Context(lat, T.functional_slda(mu, ecreg, A=A), T.run_config(precision=prec, dt=dt), n)


def _general_fields(nz, seed):
    U = synth.uniform_field(seed, nz, -0.3, 0.3)
    delta = synth.complex_normal(seed + 1, nz, 0.3)
    alpha = 1.0 + 0.25 * synth.uniform_field(seed + 2, nz)
    az = 0.3 * synth.uniform_field(seed + 3, nz)
    return U, delta, alpha, az


@pytest.mark.parametrize("prec", [0, 1])
def test_general_operator_linear_mode(prec):
    geom, mu, vext, v0, E, kp2, phi = problem(64, 4, 1.0, 5.0, seed=5)
    U, delta, alpha, az = _general_fields(64, 90)
    x = synth.complex_normal(95, phi.shape)
    zero = np.zeros(64)
    ref = geom.apply_h(x, U + vext - mu, delta, alpha, [zero, zero, az])
    ctx = make_ctx(geom, mu, 5.0, len(E), prec)
    try:
        ctx.set_external(vext, freeze_regulator=True)
        ctx.load_states(phi, E, kp2)
        ctx.set_fields(U, delta)
        ctx.set_current_fields(alpha, az)
        dt = torch.complex128 if prec == 0 else torch.complex64
        xd = torch.from_numpy(x.reshape(len(E), 2, -1)).to(dt).cuda()
        yd = torch.zeros_like(xd)
        ctx.apply_hbdg(xd, yd, len(E))
        torch.cuda.synchronize()
        out = yd.cpu().numpy().astype(np.complex128).reshape(x.shape)
        assert np.abs(out - ref).max() / np.abs(ref).max() < (1e-12 if prec == 0 else 3e-6)
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_general_td_linear_mode(prec):
    """Frozen general fields: Taylor start-up + 10 AB4AM5 steps of every
    state against the oracle's evolution with the same operator."""
    geom, mu, vext, v0, E, kp2, phi = problem(64, 4, 1.0, 5.0, seed=6)
    U, delta, alpha, az = _general_fields(64, 100)
    zero = np.zeros(64)
    frozen = (U + vext - mu, delta, alpha, [zero, zero, az])
    sysm = td.TDSystem(geom, None, mu, vext, np.zeros(64), F.fermi_weight(E), F.fermi_weight(-E), frozen=frozen)
    ref = td.evolve(sysm, phi, 0.005, 10)
    ctx = make_ctx(geom, mu, 5.0, len(E), prec)
    try:
        ctx.set_external(vext, freeze_regulator=True)
        ctx.set_fields(U, delta)
        ctx.set_current_fields(alpha, az)
        ctx.load_states(phi, E, kp2)
        ctx.abm_step(10)
        got = ctx.get_states()
        assert rel(got, ref) < (1e-10 if prec == 0 else 1e-5)
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_general_td_selfconsistent(prec):
    """SLDA at A = 1.094 (the general functional), states carrying a pair
    momentum in a trap whose bump is removed at t = 0: Taylor start-up + 10
    steps; rho, tau, nu, j, every energy term and (FP64) the states against
    the oracle.  The regulator is computed on the device with A."""
    nz, nk, dperp, ec = 64, 6, 1.3, 6.0
    geom, mu, vext, v0, E, kp2, phi = problem(nz, nk, dperp, ec, seed=3)
    fun = F.Functional(F.SLDA, force_a1=False)
    lam = F.lambda_c(v0, mu, ec, A=fun.A)
    sysm = td.TDSystem(geom, fun, mu, v0, lam, F.fermi_weight(E), F.fermi_weight(-E))
    ref = td.evolve(sysm, phi, 0.005, 10)
    ctx = make_ctx(geom, mu, ec, len(E), prec, A=fun.A)
    try:
        ctx.set_external(v0, freeze_regulator=True)
        ctx.load_states(phi, E, kp2)
        ctx.abm_step(10)
        d = ctx.densities()
        r, t_, n, j = geom.full_densities(ref, sysm.wu, sysm.wv)
        tol = 1e-10 if prec == 0 else 1e-5
        assert np.abs(j[2]).max() > 1e-3 * np.abs(r).max()  # the currents are there
        assert rel(d["rho"], r) < tol
        assert rel(d["nu"], n) < tol
        assert rel(d["tau"], t_) < tol
        assert rel(d["j"][2], j[2]) < tol
        e = ctx.energy()
        o = td.observables(sysm, ref)
        for k in ("kin", "pot", "pair", "curr", "potext", "N", "total"):
            assert abs(e[k] - o[k]) <= tol * max(abs(o[k]), 1e-12 * o["EFG"]), (k, e[k], o[k])
        if prec == 0:
            assert rel(ctx.get_states(), ref) < 1e-10
    finally:
        ctx.close()


