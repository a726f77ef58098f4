"""Parity of the quasi-2D kernel set with the oracle's quasi-2D mode (Sec.
3.1, quasi-2D item): one x-y BdG problem per |k_z| class, all classes in one
flat batch of states with their k_z^2 and multiplicities, the 2D Laplacian
of every state in one workgroup."""
import numpy as np
import pytest

from oracle import bdg, functional as F, td, q2d
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


def problem(nx, ny, nz, ec, seed, d=(1.0, 1.2, 1.0)):
    """Static states of a trap with a Gaussian obstacle (removed at t = 0)."""
    geom = q2d.GeometryQ2D(nx, ny, nz, *d)
    X, Y = geom.static.coords()
    mu = 1.0
    vb, wb, xb = synth.gaussian_bump(seed)
    wb = wb * nx / 256.0 + 0.8
    trap = 0.5 * (0.6 / nx) ** 2 * (X ** 2 + Y ** 2)
    vs = trap + vb * np.exp(-((X - 0.1 * xb * nx / 256.0) ** 2 + Y ** 2) / (2 * wb * wb))
    delta = 0.5 + 0.05 * synth.uniform_field(seed + 1, geom.shape)
    E, kz2, mult, phi = q2d.eigenstates(geom, vs - mu, delta + 0j, ec=ec)
    geom.set_states(kz2)
    return geom, mu, trap, E, kz2, mult, phi


def make_ctx(geom, mu, ecreg, n, prec=0, dt=0.005):
    from paper_2602_08982_amd import tdslda as T
    lat = T.lattice_q2d(geom.nx, geom.ny, geom.nz, (geom.dx, geom.dy, geom.dz))
    return T.Context(lat, T.functional_slda(mu, ecreg), T.run_config(precision=prec, dt=dt), n)


@pytest.mark.parametrize("nx,ny,nz,ec", [(8, 8, 4, None), (12, 12, 6, 4.0), (24, 16, 6, 3.0)])
@pytest.mark.parametrize("prec", [0, 1])
def test_q2d_td(nx, ny, nz, ec, prec):
    """Self-consistent evolution after the obstacle is removed: densities,
    energy terms and (FP64) the states after 10 steps against the oracle."""
    geom, mu, trap, E, kz2, mult, phi = problem(nx, ny, nz, ec, seed=3)
    assert len(np.unique(kz2)) > 1 and np.any(mult == 2) and np.any(mult == 1)
    ecreg = 0.5 * np.pi ** 2 if ec is None else ec
    lam = F.lambda_c(trap, mu, ecreg)
    sysm = td.TDSystem(geom, F.Functional(F.SLDA), mu, trap, lam, mult * F.fermi_weight(E),
                       mult * F.fermi_weight(-E))
    ref = td.evolve(sysm, phi, 0.005, 10)
    ctx = make_ctx(geom, mu, ecreg, len(E), prec)
    try:
        ctx.set_external(trap, freeze_regulator=False)
        ctx.set_regulator(lam)
        ctx.load_states(phi, E, kz2)
        ctx.set_multiplicity(mult)
        ctx.abm_step(10)
        d = ctx.densities()
        r, t_, n, j = geom.full_densities(ref, sysm.wu, sysm.wv)
        tol = 1e-10 if prec == 0 else 1e-5
        assert rel(d["rho"], r) < tol
        assert rel(d["nu"], n) < tol
        assert rel(d["tau"], t_) < tol
        for a in range(2):
            assert np.abs(d["j"][a] - j[a]).max() < tol * np.abs(t_).max()
        assert np.abs(d["j"][2]).max() == 0.0
        e = ctx.energy()
        o = td.observables(sysm, ref)
        for k in ("kin", "pot", "pair", "potext", "N", "total"):
            sc = abs(o[k]) if o[k] != 0 else o["EFG"]  # each term against its own size
            assert abs(e[k] - o[k]) / sc < tol, (k, e[k], o[k])
        if prec == 0:
            assert np.abs(ctx.get_states() - ref).max() < 1e-9
    finally:
        ctx.close()


@pytest.mark.parametrize("nx,ny", [(16, 16), (24, 16)])
def test_q2d_apply_hbdg(nx, ny):
    """H phi of random states with random fields, each state with its own
    k_z^2 (FP64, to 1e-12 of the largest entry)."""
    geom, mu, trap, E, kz2, mult, phi = problem(nx, ny, 4, 2.0, seed=5)
    U = synth.uniform_field(9, geom.shape, -0.3, 0.3)
    delta = synth.complex_normal(10, geom.shape, 0.3)
    x = synth.complex_normal(11, phi.shape)
    ref = geom.apply_h(x, U + trap - mu, delta)
    ctx = make_ctx(geom, mu, 2.0, len(E))
    try:
        ctx.set_external(trap, freeze_regulator=True)
        ctx.load_states(phi, E, kz2)
        ctx.set_fields(U, delta)
        xd = torch.from_numpy(x.reshape(len(E), 2, -1)).cuda()
        yd = torch.zeros_like(xd)
        ctx.apply_hbdg(xd, yd, len(E))
        torch.cuda.synchronize()
        out = yd.cpu().numpy().reshape(x.shape)
        assert np.abs(out - ref).max() / np.abs(ref).max() < 1e-12
    finally:
        ctx.close()


def test_q2d_plane_waves_vortex():
    """Device plane-wave start (every (l_x, l_y) and |k_z| class) with a
    vortex imprint, then 8 steps in a trap, against the oracle."""
    from paper_2602_08982_amd import tdslda as T
    geom = q2d.GeometryQ2D(12, 12, 6, 1.0, 1.0, 1.0)
    lat = T.lattice_q2d(12, 12, 6, 1.0)
    mu, u0, d0 = 1.0, 0.0, 0.5
    kidx = np.array([(a, b, m) for a in range(12) for b in range(12) for m in range(4)], np.int32)
    E, kz2, mult, phi = q2d.plane_wave_states(geom, kidx, u0 - mu, d0)
    geom.set_states(kz2)
    X, Y = geom.static.coords()
    trap = 0.5 * 0.08 ** 2 * (X ** 2 + Y ** 2)
    ec = 0.5 * np.pi ** 2
    vort = np.array([[0.3, -0.2, 1.0]])
    th = q2d_vortex_theta(geom, vort)
    phi = bdg.imprint_phase(phi, th)
    lam = F.lambda_c(trap, mu, ec)
    sysm = td.TDSystem(geom, F.Functional(F.SLDA), mu, trap, lam, mult * F.fermi_weight(E),
                       mult * F.fermi_weight(-E))
    ref = td.evolve(sysm, phi, 0.005, 8)
    ctx = T.Context(lat, T.functional_slda(mu, ec), T.run_config(dt=0.005), len(kidx))
    try:
        ctx.set_external(trap, freeze_regulator=True)
        ctx.init_plane_waves(kidx, u0, d0)
        ctx.imprint_vortices(vort)
        assert np.abs(ctx.get_states() - phi).max() < 1e-13
        ctx.abm_step(8)
        assert np.abs(ctx.get_states() - ref).max() < 1e-9
        e = ctx.energy()
        o = td.observables(sysm, ref)
        for k in ("kin", "pot", "pair", "total", "N"):
            sc = abs(o[k]) if o[k] != 0 else o["EFG"]  # each term against its own size
            assert abs(e[k] - o[k]) / sc < 1e-10, (k, e[k], o[k])
    finally:
        ctx.close()


def q2d_vortex_theta(geom, vort):
    X, Y = geom.static.coords()
    return sum(q * np.arctan2(Y - y0, X - x0) for x0, y0, q in vort)


def test_q2d_refusals():
    """A != 1, quantum friction, the general operator and an unknown shape
    are refused with EINVAL; multiplicities only between a load and the
    first step."""
    from paper_2602_08982_amd import tdslda as T
    lat = T.lattice_q2d(8, 8, 4, 1.0)
    with pytest.raises(T.TdsldaError):
        T.Context(lat, T.functional_slda(1.0, 4.0, A=1.094), T.run_config(), 4)
    with pytest.raises(T.TdsldaError):
        T.Context(T.lattice_q2d(10, 10, 4, 1.0), T.functional_slda(1.0, 4.0), T.run_config(), 4)
    geom, mu, trap, E, kz2, mult, phi = problem(8, 8, 4, 2.0, seed=7)
    ctx = make_ctx(geom, mu, 2.0, len(E))
    try:
        with pytest.raises(T.TdsldaError):
            ctx.set_multiplicity(mult)  # nothing loaded
        ctx.set_external(trap)
        ctx.load_states(phi, E, kz2)
        with pytest.raises(T.TdsldaError):
            ctx.set_multiplicity(mult[:-1])
        with pytest.raises(T.TdsldaError):
            ctx.set_friction(alpha=0.1)
        ctx.set_multiplicity(mult)
        ctx.abm_step(1)
        with pytest.raises(T.TdsldaError):
            ctx.set_multiplicity(mult)
        ctx.set_fields(*ctx.get_fields())
        with pytest.raises(T.TdsldaError):
            ctx.set_current_fields(alpha=np.full(geom.shape, 1.1))
    finally:
        ctx.close()


def test_q2d_bench_size_sampled():
    """The 64 x 64, N_z = 64 workload of the benchmark in its own launch
    configuration (135,168 states: more grid rows than one launch dimension
    holds, so the per-state passes stride over states), FP32-mixed:
    sampled start states against the oracle's plane-wave start with the
    vortex, H phi of sampled states with the device's fields against the
    oracle's operator, then 4 steps with the particle number and the norms
    kept."""
    from paper_2602_08982_amd import tdslda as T
    from paper_2602_08982_amd import workloads as W
    cfg = W.Q2D
    vort = [(-0.95, -0.81, 1.0)]
    ctx, kidx = W.setup_q2d(cfg, vort)
    try:
        nst = len(kidx)
        assert nst == 64 * 64 * 33 > 65535
        geom = q2d.GeometryQ2D(64, 64, 64, 1.0, 1.0, 1.0)
        rng = np.random.default_rng(5)
        pick = np.sort(np.concatenate([[0, nst - 1], rng.choice(nst, 62, replace=False)]))
        E, kz2, mult, phi = q2d.plane_wave_states(geom, kidx[pick], cfg["u0"] - cfg["mu"], cfg["delta0"])
        phi = bdg.imprint_phase(phi, q2d_vortex_theta(geom, np.array(vort)))
        xd = torch.empty((nst, 2, 64 * 64), dtype=torch.complex64, device="cuda")
        states = ctx.get_states()
        assert np.abs(states[pick] - phi).max() < 2e-7
        U, delta = ctx.get_fields()
        X, Y = geom.static.coords()
        vext = 0.5 * cfg["omega"] ** 2 * (X ** 2 + Y ** 2)
        geom.set_states(kz2)
        ref = geom.apply_h(phi, U + vext - cfg["mu"], delta)
        xs = torch.from_numpy(states[pick].reshape(len(pick), 2, -1).astype(np.complex64)).cuda()
        ys = torch.zeros_like(xs)
        # apply_hbdg takes k_z^2 of the loaded state with the same index: put
        # the sampled states at their own indices of a full-size input
        xd.zero_()
        xd[torch.from_numpy(pick).cuda()] = xs
        yd = torch.zeros_like(xd)
        ctx.apply_hbdg(xd, yd, nst)
        torch.cuda.synchronize()
        out = yd[torch.from_numpy(pick).cuda()].cpu().numpy().reshape(ref.shape)
        assert np.abs(out - ref).max() / np.abs(ref).max() < 2e-6
        del xd, yd, xs, ys
        e0 = ctx.energy()
        ctx.abm_step(4)
        e1 = ctx.energy()
        assert abs(e1["N"] - e0["N"]) / e0["N"] < 1e-6
        st, chk = ctx.check()
        assert chk["norm"] < 1e-5
    finally:
        ctx.close()
