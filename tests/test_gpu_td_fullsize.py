"""Time-dependent parity with the FP64 oracle at the lattice shapes the
benchmark times (32^3 FP64, 48^3 FP64, 48^3 FP32-mixed) and at 24^3.

The kernels are templated on the lattice shape: the slab tiling of the
(y,z) transforms, the radix-3 48-point lines, the density-group sizes and
the lazy normalisation all differ between 8^3 and these shapes, so every
integrator pass (Taylor start-up, predictor, corrector, full pass) is run
here at the benchmarked instantiations and compared element by element
with the oracle on the same seeded inputs:

  - self-consistent fields: a seeded sample of the benchmark's own start
    (plane-wave states of the uniform H, trap switched on, vortex imprint;
    Secs. 2.3, 3.3, 4.5.1), Taylor start-up + 1 step, then 3 more steps in
    one call (so the full pass that fuses f_k, the next predictor and the
    partial corrector runs twice);
  - linear mode (fields frozen at random values) per shape;
  - more states than one density group (256 FP64 / 128 FP32), so the
    multi-group fixed-order reduction runs, from a stationary start.

Bars (written in each test): FP64 1e-10 relative, FP32-mixed 1e-5
relative; energy terms relative to their own magnitude.
"""
import numpy as np
import pytest

from oracle import lattice as L, bdg, densities as D, functional as F, td
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FP64, FP32 = 0, 1


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


def harmonic(lat, omega):
    X, Y, Z = lat.coords()
    wx, wy, wz = omega
    return 0.5 * (wx ** 2 * X ** 2 + wy ** 2 * Y ** 2 + wz ** 2 * Z ** 2)


# trap and vortices of the benchmarked workloads: 32^3 one vortex in an
# isotropic trap, 48^3 a vortex pair in the elongated trap; 24^3 uses the
# 32^3 parameters
def workload(n):
    if n == 48:
        (x1, y1), (x2, y2) = synth.vortex_pair(4)
        return (0.08, 0.08, 0.02), [(x1, y1, 1.0), (x2, y2, -1.0)]
    dx, dy = synth.vortex_offset(2)
    return (0.05, 0.05, 0.05), [(dx, dy, 1.0)]


MU, U0, DELTA0, DT = 1.0, 0.0, 0.5, 0.005


def sample_kidx(n, nst, seed):
    """nst distinct lattice momenta (seeded) of an n^3 grid."""
    g = synth.rng(seed)
    flat = np.sort(g.choice(n ** 3, size=nst, replace=False))
    return np.stack([flat // (n * n), (flat // n) % n, flat % n], axis=1).astype(np.int32)


class Case:
    """One seeded self-consistent workload: oracle system + initial states."""

    def __init__(self, n, nst, seed):
        self.n, self.nst = n, nst
        self.lat = L.Lattice(n, n, n)
        omega, self.vort = workload(n)
        self.vext = harmonic(self.lat, omega)
        self.kidx = sample_kidx(n, nst, seed)
        self.ec = 0.5 * np.pi ** 2
        E, phi = bdg.plane_wave_states(self.lat, self.kidx, U0 - MU, DELTA0)
        self.E = E
        self.phi0 = bdg.imprint_phase(phi, bdg.vortex_phase(self.lat, self.vort))
        lam = F.lambda_c(self.vext, MU, self.ec)
        self.sys = td.TDSystem(td.Geometry3D(self.lat), F.Functional(F.SLDA), MU, self.vext, lam,
                               F.fermi_weight(E), F.fermi_weight(-E))

    def gpu_context(self, prec, selfstart):
        t = T()
        run = t.run_config(precision=prec, dt=DT, selfstart=selfstart)
        ctx = t.Context(t.lattice_3d((self.n,) * 3), t.functional_slda(MU, self.ec), run, self.nst)
        ctx.set_external(self.vext, freeze_regulator=True)
        # the benchmark's device generators: plane waves, then the imprint
        ctx.init_plane_waves(self.kidx, U0, DELTA0)
        ctx.imprint_vortices(self.vort)
        return ctx

    def reference(self, selfstart, checkpoints):
        """Oracle states and observables after each checkpoint step."""
        out = {}
        phi, hist, _ = td.start(self.sys, self.phi0, DT, "AB4AM5", selfstart)
        for s in range(1, max(checkpoints) + 1):
            phi, hist = td.abm_step(self.sys, phi, hist, DT)
            if s in checkpoints:
                dens = D.spin_symmetric(phi, self.sys.wu, self.sys.wv, self.lat)
                out[s] = (phi.copy(), dens, td.observables(self.sys, phi))
        return out


_cache = {}


def cached(key, make):
    if key not in _cache:
        _cache[key] = make()
    return _cache[key]


def compare(ctx, lat, ref, tol, states, label):
    phi_ref, (r, t_, n, j), o = ref
    d = ctx.densities()
    assert rel(d["rho"], r) < tol, (label, "rho", rel(d["rho"], r))
    assert rel(d["tau"], t_) < tol, (label, "tau", rel(d["tau"], t_))
    assert rel(d["nu"], n) < tol, (label, "nu", rel(d["nu"], n))
    jn = np.sqrt(sum(np.sum(np.abs(c) ** 2) for c in j))
    for c in range(3):
        # each current component against the norm of the whole current
        assert np.linalg.norm(d["j"][c] - j[c]) / jn < tol, (label, "j", c)
    e = ctx.energy()
    for k in ("kin", "pot", "pair", "curr", "potext", "total", "N"):
        assert abs(e[k] - o[k]) <= tol * abs(o[k]), (label, k, e[k], o[k])
    if states:
        st = ctx.get_states()
        err = np.abs(st - phi_ref).max() / np.abs(phi_ref).max()
        assert err < tol, (label, "states", err)


# ---------------------------------------------------------------------------
# self-consistent fields, Taylor start-up, bench workload sample
SC = [(32, FP64), (48, FP64), (48, FP32), (24, FP64), (24, FP32)]


@pytest.mark.parametrize("n,prec", SC, ids=[f"{n}^3-{'fp64' if p == FP64 else 'fp32'}" for n, p in SC])
def test_td_selfconsistent_fullsize(n, prec):
    """Taylor start-up + 1 AB4AM5 step, then 3 steps in one call: states
    (FP64), rho, tau, nu, j and every energy term against the oracle."""
    print(f"# td parity {n}^3 prec={prec}: oracle", flush=True)
    case = cached(("case", n, 16), lambda: Case(n, 16, 100 + n))
    ref = cached(("ref", n, 16, 1), lambda: case.reference(1, (1, 4)))
    print(f"# td parity {n}^3 prec={prec}: device", flush=True)
    tol = 1e-10 if prec == FP64 else 1e-5
    ctx = case.gpu_context(prec, selfstart=1)
    try:
        ctx.abm_step(1)
        compare(ctx, case.lat, ref[1], tol, prec == FP64, "step 1")
        ctx.abm_step(3)
        compare(ctx, case.lat, ref[4], tol, prec == FP64, "step 4")
    finally:
        ctx.close()


# ---------------------------------------------------------------------------
# linear mode: fields frozen
LIN = [(32, FP64), (48, FP64), (48, FP32), (24, FP64)]


@pytest.mark.parametrize("n,prec", LIN, ids=[f"{n}^3-{'fp64' if p == FP64 else 'fp32'}" for n, p in LIN])
def test_td_linear_mode_fullsize(n, prec):
    """Random frozen U, Delta; random states; Taylor start-up + 3 steps in
    one call: the states against the oracle's integrator on the same
    frozen operator."""
    lat = L.Lattice(n, n, n)
    nst = 6
    mu = 0.4

    def make():
        U = synth.uniform_field(200 + n, lat.shape, -0.3, 0.3)
        delta = synth.complex_normal(201 + n, lat.shape, 0.2)
        phi = D.normalize(synth.complex_normal(202 + n, (nst, 2) + lat.shape), lat.dV)
        sysl = td.TDSystem(td.Geometry3D(lat), None, mu, np.zeros(lat.shape), np.zeros(lat.shape),
                           np.zeros(nst), np.ones(nst), frozen=(U - mu, delta))
        return U, delta, phi, td.evolve(sysl, phi, DT, 3)

    print(f"# linear mode {n}^3 prec={prec}: oracle", flush=True)
    U, delta, phi, ref = cached(("lin", n), make)
    t = T()
    run = t.run_config(precision=prec, dt=DT, selfstart=1)
    ctx = t.Context(t.lattice_3d((n,) * 3), t.functional_slda(mu, 10.0), run, nst)
    try:
        ctx.load_states(phi, np.ones(nst))
        ctx.set_fields(U, delta)
        ctx.abm_step(3)
        st = ctx.get_states()
        tol = 1e-10 if prec == FP64 else 1e-5
        err = np.abs(st - ref).max() / np.abs(ref).max()
        assert err < tol, err
    finally:
        ctx.close()


# ---------------------------------------------------------------------------
# more states than one density group
MANY = [(32, FP64, 300), (48, FP32, 136)]


@pytest.mark.parametrize("n,prec,nst", MANY, ids=[f"{n}^3-{'fp64' if p == FP64 else 'fp32'}-{k}"
                                                 for n, p, k in MANY])
def test_td_many_states_fullsize(n, prec, nst):
    """nst > states per density group (256 FP64, 128 FP32): stationary
    start, then 2 steps in one call; densities, energy terms and (FP64)
    states against the oracle."""
    print(f"# many states {n}^3 prec={prec} nst={nst}: oracle", flush=True)
    case = Case(n, nst, 300 + n)
    ref = case.reference(0, (2,))
    print(f"# many states {n}^3 prec={prec} nst={nst}: device", flush=True)
    tol = 1e-10 if prec == FP64 else 1e-5
    ctx = case.gpu_context(prec, selfstart=0)
    try:
        ctx.abm_step(2)
        compare(ctx, case.lat, ref[2], tol, prec == FP64, "step 2")
    finally:
        ctx.close()
