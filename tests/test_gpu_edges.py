"""Edge cases of the HIP path through the C ABI: a single state, state counts
that leave partial workgroups and partial density groups (3D and quasi-1D,
where the quasi-1D F / CORR / FULL passes take <H>_n inside the pass), a
zero-step call, and the argument checks (counts outside [1, capacity],
negative step counts, out-of-order calls)."""
import numpy as np
import pytest

from oracle import lattice as L, densities as D, td, q1d
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


def linear_3d_ctx(lat, mu, nst, prec):
    t = T()
    lt = t.Lattice(t.MODE_3D, *lat.n, *lat.d, 0.0, 0.0)
    return t.Context(lt, t.functional_slda(mu, 10.0), t.run_config(precision=prec, dt=0.01), nst)


@pytest.mark.parametrize("nst", [1, 2, 65])
@pytest.mark.parametrize("prec", [0, 1])
def test_linear_3d_state_counts(nst, prec):
    """Frozen fields (linear mode), 6^3: one state, two states and 65 (one
    more than a density group) against the oracle's integrator."""
    lat = L.Lattice(6, 6, 6, 1.2, 1.2, 1.2)
    mu = 0.3
    U = synth.uniform_field(11, lat.shape, -0.3, 0.3)
    delta = synth.complex_normal(12, lat.shape, 0.3)
    phi = D.normalize(synth.complex_normal(13, (nst, 2) + lat.shape), lat.dV)
    zero = np.zeros(lat.shape)
    sysl = td.TDSystem(td.Geometry3D(lat), None, mu, zero, zero, np.zeros(nst), np.ones(nst),
                       frozen=(U - mu, delta))
    ref = td.evolve(sysl, phi, 0.01, 6)
    ctx = linear_3d_ctx(lat, mu, nst, prec)
    ctx.load_states(phi, np.ones(nst))
    ctx.set_fields(U, delta)
    ctx.abm_step(6)
    st = ctx.get_states()
    ctx.close()
    tol = 1e-11 if prec == 0 else 1e-5
    assert np.abs(st - ref).max() < tol * np.abs(ref).max()


@pytest.mark.parametrize("nst", [1, 3, 37])
@pytest.mark.parametrize("prec", [0, 1])
def test_linear_q1d_state_counts(nst, prec):
    """Frozen fields, quasi-1D N_z = 64 with per-state k_perp^2: one state,
    three, and 37 (a partial workgroup of the fused passes) against the
    oracle's integrator on the same frozen operator."""
    nz = 64
    geom = q1d.GeometryQ1D(nz, 1.0, 4, 4, 1.5)
    kp2 = synth.uniform_field(21, (nst,), 0.0, 2.0)
    geom.set_states(kp2)
    mu = 0.3
    U = synth.uniform_field(22, (nz,), -0.3, 0.3)
    delta = synth.complex_normal(23, (nz,), 0.3)
    phi = D.normalize(synth.complex_normal(24, (nst, 2, nz)), geom.dV)
    zero = np.zeros(nz)
    sysl = td.TDSystem(geom, None, mu, zero, zero, np.zeros(nst), np.ones(nst), frozen=(U - mu, delta))
    ref = td.evolve(sysl, phi, 0.01, 6)
    t = T()
    ctx = t.Context(t.lattice_q1d(nz, 1.0, geom.Lx, geom.Ly), t.functional_slda(mu, 10.0),
                    t.run_config(precision=prec, dt=0.01), nst)
    ctx.load_states(phi, np.ones(nst), kp2)
    ctx.set_fields(U, delta)
    ctx.abm_step(6)
    st = ctx.get_states()
    ctx.close()
    tol = 1e-11 if prec == 0 else 1e-5
    assert np.abs(st - ref).max() < tol * np.abs(ref).max()


def test_zero_steps_and_argument_errors():
    """abm_step(0) runs only the start-up (3 Taylor steps for AB4AM5, not
    counted as steps) and a second abm_step(0) changes nothing; counts
    outside [1, capacity] and negative step counts return EINVAL; calls
    before a load return EORDER."""
    t = T()
    lat = L.Lattice(6, 6, 6, 1.2, 1.2, 1.2)
    mu = 0.3
    nst = 3
    U = synth.uniform_field(11, lat.shape, -0.3, 0.3)
    delta = synth.complex_normal(12, lat.shape, 0.3)
    phi = D.normalize(synth.complex_normal(13, (nst, 2) + lat.shape), lat.dV)
    ctx = linear_3d_ctx(lat, mu, nst, 0)
    with pytest.raises(t.TdsldaError) as ei:
        ctx.abm_step(1)
    assert ei.value.status == t.EORDER
    with pytest.raises(t.TdsldaError) as ei:
        ctx.load_states(phi[:0], np.ones(0))
    assert ei.value.status == t.EINVAL
    big = np.concatenate([phi, phi[:1]])
    with pytest.raises(t.TdsldaError) as ei:
        ctx.load_states(big, np.ones(nst + 1))
    assert ei.value.status == t.EINVAL
    ctx.load_states(phi, np.ones(nst))
    ctx.set_fields(U, delta)
    with pytest.raises(t.TdsldaError) as ei:
        ctx.abm_step(-1)
    assert ei.value.status == t.EINVAL
    ctx.abm_step(0)
    n, steps, time = ctx.info()
    assert (n, steps) == (nst, 0) and abs(time - 3 * 0.01) < 1e-15
    a = ctx.get_states()
    ctx.abm_step(0)
    assert np.array_equal(ctx.get_states(), a)
    x = torch.zeros(nst * 2 * int(np.prod(lat.n)) * 2, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    for bad_n in (0, nst + 1):
        with pytest.raises(t.TdsldaError) as ei:
            ctx.apply_hbdg(x, y, bad_n)
        assert ei.value.status == t.EINVAL
    ctx.close()


def test_unsupported_shapes():
    """Shapes without a kernel instance are refused at creation (EINVAL)."""
    t = T()
    for lt in (t.Lattice(t.MODE_3D, 10, 10, 10, 1.0, 1.0, 1.0, 0.0, 0.0), t.lattice_q1d(32, 1.0, 4.0, 4.0)):
        with pytest.raises(t.TdsldaError) as ei:
            t.Context(lt, t.functional_slda(0.3, 10.0), t.run_config(), 4)
        assert ei.value.status == t.EINVAL
