"""Batched quasi-1D mode on the GPU: static states of every transverse
problem from the device eigensolver against the oracle, the HIP-graph
advance against the eagerly launched one, the launch-shape tuner, and the
full-size batched workload (2,304 problems, N_z = 256)."""
import numpy as np
import pytest

from oracle import q1d as Q, functional as F
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
    tdslda.load_library()
    return tdslda


def small_case(nz=64, nk=4, dperp=2.0, seed=3):
    from paper_2602_08982_amd import workloads as W
    cfg = dict(W.Q1D, nz=nz, nk=nk)
    vt, vs = W.q1d_potentials(cfg, synth.gaussian_bump(seed))
    kp2 = W.q1d_kperp2(nk, dperp)
    hstatic = vs - cfg["mu"]
    delta = np.full(nz, cfg["delta0"])
    return cfg, vt, hstatic, delta, kp2


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("prec", [0, 1])
def test_q1d_static_states_match_oracle(prec):
    """Device eigensolver + selection (0 < E < E_c) of 16 problems at N_z=64:
    per-problem counts equal the oracle's dense eigh counts exactly, and the
    densities of the loaded states match the oracle's (FP64 1e-10, FP32-mixed
    states 1e-5)."""
    t = T()
    cfg, vt, hstatic, delta, kp2 = small_case()
    nz, nk, dperp = cfg["nz"], cfg["nk"], 2.0
    lat = t.lattice_q1d(nz, 1.0, nk * dperp, nk * dperp)
    counts, total = t.q1d_count(lat, kp2, hstatic, delta, cfg["ecut"])
    # oracle, problem by problem in the same k_perp^2 order
    geom = Q.GeometryQ1D(nz, 1.0, nk, nk, dperp)
    ref_counts, Es, kps, phis = [], [], [], []
    for kp in kp2:
        H = Q.dense_h_1d(hstatic, delta, nz, 1.0, kp)
        E, W_ = np.linalg.eigh(H)
        sel = np.nonzero((E > 0) & (E < cfg["ecut"]))[0]
        ref_counts.append(sel.size)
        Es.append(E[sel])
        kps.append(np.full(sel.size, kp))
        phis.append(W_[:, sel].T.reshape(sel.size, 2, nz))
    assert counts.tolist() == ref_counts
    assert total == sum(ref_counts)
    E = np.concatenate(Es)
    phi = np.concatenate(phis)
    geom.set_states(np.concatenate(kps))
    rho, tau, nu, j = geom.full_densities(phi, F.fermi_weight(E), F.fermi_weight(-E))
    run = t.run_config(precision=prec)
    ctx = t.Context(lat, t.functional_slda(cfg["mu"], cfg["ecut"]), run, int(total))
    try:
        ctx.set_external(vt, freeze_regulator=True)
        assert ctx.q1d_load_static(kp2, hstatic, delta, cfg["ecut"]) == total
        d = ctx.densities()
        tol = 1e-10 if prec == 0 else 1e-5
        assert rel(d["rho"], rho) < tol
        assert rel(d["nu"], nu) < tol
        assert rel(d["tau"], tau) < tol
    finally:
        ctx.close()


def _q1d_ctx(t, prec, nz=64, nk=4):
    cfg, vt, hstatic, delta, kp2 = small_case(nz=nz, nk=nk)
    lat = t.lattice_q1d(nz, 1.0, nk * 2.0, nk * 2.0)
    _, total = t.q1d_count(lat, kp2, hstatic, delta, cfg["ecut"])
    ctx = t.Context(lat, t.functional_slda(cfg["mu"], cfg["ecut"]), t.run_config(precision=prec), int(total))
    ctx.set_external(vt, freeze_regulator=True)
    ctx.q1d_load_static(kp2, hstatic, delta, cfg["ecut"])
    return ctx


def _3d_ctx(t):
    from test_gpu_parity import config1, make_ctx
    lat, mu, ec, E, phi, sysm = config1()
    ctx = make_ctx(lat, mu, ec, len(E))
    ctx.set_external(np.zeros(lat.shape), freeze_regulator=True)
    ctx.load_states(phi, E)
    return ctx


@pytest.mark.parametrize("kind", ["q1d_fp32", "q1d_fp64", "3d_fp64"])
def test_graph_advance_equals_eager(kind):
    """abm_graph(k) (one recorded launch) gives bit-identical states to
    abm_step(k), on three consecutive advances with eager work (a read-out)
    and synchronisation between them."""
    t = T()
    make = (lambda: _q1d_ctx(t, 1)) if kind == "q1d_fp32" else \
        (lambda: _q1d_ctx(t, 0)) if kind == "q1d_fp64" else (lambda: _3d_ctx(t))
    a, b = make(), make()
    try:
        a.abm_step(0)
        b.abm_step(0)
        for k in (4, 3, 5):
            a.abm_step(k)
            rec_ms, run_ms = b.abm_graph(k)
            assert rec_ms >= 0 and run_ms >= 0
            sa, sb = a.get_states(), b.get_states()
            assert np.array_equal(sa, sb)
            assert a.info()[1] == b.info()[1]
    finally:
        a.close()
        b.close()


def test_graph_needs_started_integrator():
    t = T()
    ctx = _q1d_ctx(t, 1)
    try:
        with pytest.raises(t.TdsldaError) as e:
            ctx.abm_graph(2)
        assert e.value.status == t.EORDER
    finally:
        ctx.close()


def test_autotune_keeps_the_result():
    """The tuner picks workgroup sizes from {64, 128, 256} for the four
    quasi-1D kernel classes; evolving with the tuned shapes agrees with the
    default shapes to FP64 rounding (the shapes change only summation order)."""
    t = T()
    a, b = _q1d_ctx(t, 0), _q1d_ctx(t, 0)
    try:
        a.abm_step(0)
        b.abm_step(0)
        tuned = b.autotune()
        assert len(tuned) == 4
        assert all(tb in (64, 128, 256) and ms > 0 for tb, ms in tuned)
        a.abm_step(6)
        b.abm_step(6)
        assert rel(b.get_states(), a.get_states()) < 1e-12
    finally:
        a.close()
        b.close()
    c = _3d_ctx(t)
    try:
        assert c.autotune() == []  # fixed shapes in 3D
    finally:
        c.close()


def test_batched_q1d_fullsize():
    """The full batched workload (2,304 problems, N_z = 256, FP32-mixed):
    the corner problem's kept count is in [32, 48] after the d_perp bisection;
    sampled problems' counts equal the oracle's dense eigh; after tuning, a
    graph-recorded advance conserves N and keeps the states normalised."""
    t = T()
    from paper_2602_08982_amd import workloads as W
    cfg = W.Q1D
    ctx, info = W.setup_q1d(cfg, seed=7)
    try:
        assert info["nproblems"] == 2304
        assert 32 <= info["corner_count"] <= 48
        vt, vs = W.q1d_potentials(cfg, synth.gaussian_bump(7))
        hstatic = vs - cfg["mu"]
        delta = np.full(cfg["nz"], cfg["delta0"])
        kp2, counts = info["kperp2"], info["counts"]
        for p in (0, int(np.argmin(kp2)), 1234, int(np.argmax(kp2))):
            H = Q.dense_h_1d(hstatic, delta, cfg["nz"], cfg["dz"], kp2[p])
            E = np.linalg.eigvalsh(H)
            assert counts[p] == int(np.sum((E > 0) & (E < cfg["ecut"])))
        ctx.abm_step(0)
        tuned = ctx.autotune()
        assert len(tuned) == 4
        e0 = ctx.energy()
        ctx.abm_graph(8)
        e1 = ctx.energy()
        assert abs(e1["N"] - e0["N"]) / e0["N"] < 1e-5
        st, chk = ctx.check()
        assert chk["norm"] < 1e-4
        assert np.isfinite(e1["total"])
    finally:
        ctx.close()


def test_graph_advance_with_friction_equals_eager():
    """The recorded advance includes the quantum-friction passes: abm_graph
    and abm_step give bit-identical states with all three terms on."""
    t = T()
    a, b = _q1d_ctx(t, 0), _q1d_ctx(t, 0)
    try:
        for c in (a, b):
            N0 = c.energy()["N"]
            c.set_friction(alpha=5.0, beta=5.0, gamma=0.1, rho0=0.05, N_req=1.01 * N0)
            c.abm_step(0)
        for k in (3, 4):
            a.abm_step(k)
            b.abm_graph(k)
            assert np.array_equal(a.get_states(), b.get_states())
    finally:
        a.close()
        b.close()
