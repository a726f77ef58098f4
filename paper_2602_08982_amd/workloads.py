"""Synthetic trapped-gas workloads of the benchmark (host-side set-up only:
lattice momenta to start from, external potentials, vortex positions).
The states themselves are generated and evolved by libtdslda.

  plain_fp64_32 : 32^3, dx = 1, V_ext = omega^2 r^2 / 2 (omega = 0.05), one
                  vortex along z at the centre + a seeded offset in
                  [-2, 2)^2, all 32,768 plane-wave states of the uniform H
                  (U = 0, Delta = 0.5, mu = 1), complex128.
  mixed_fp32_48 : 48^3, dx = 1, V_ext = (w_perp^2 (x^2 + y^2) + w_z^2 z^2)/2
                  with w_perp = 0.08, w_z = 0.02, a seeded vortex pair, the
                  8,192 plane-wave states with the smallest |xi_k| (16,384
                  quasiparticle states of both signs), complex64.
  q2d_64        : quasi-2D, 64 x 64 x-y lattice, dx = 1, N_z = 64 plane waves
                  along z (33 |k_z| classes), V_ext = omega^2 (x^2 + y^2)/2
                  with omega = 0.05, one vortex line at the centre + a seeded
                  offset, all 135,168 plane-wave states (every x-y momentum in
                  every class), complex64 with FP64 sums.
"""
import numpy as np

from . import tdslda as T


def centered(n, d):
    return (np.arange(n) - n // 2) * float(d)


def all_kidx(n):
    nx, ny, nz = n
    return np.array(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"),
                    dtype=np.int32).reshape(3, -1).T.copy()


def lowest_xi_kidx(n, d, mu, u0, count):
    """The `count` lattice momenta with the smallest |k^2/2 + u0 - mu|;
    ties broken by the lexicographic order of the integer indices."""
    kid = all_kidx(n)
    m = np.where(kid < np.array(n) // 2, kid, kid - np.array(n))
    k2 = sum((2 * np.pi * m[:, a] / (n[a] * d[a])) ** 2 for a in range(3))
    xi = np.abs(0.5 * k2 + u0 - mu)
    order = np.lexsort((kid[:, 2], kid[:, 1], kid[:, 0], xi))
    return kid[np.sort(order[:count])]


def harmonic(n, d, omega):
    X, Y, Z = np.meshgrid(*[centered(a, b) for a, b in zip(n, d)], indexing="ij")
    wx, wy, wz = omega
    return 0.5 * (wx ** 2 * X ** 2 + wy ** 2 * Y ** 2 + wz ** 2 * Z ** 2)


PLAIN = dict(name="plain_fp64_32", n=(32, 32, 32), d=(1.0, 1.0, 1.0), mu=1.0, u0=0.0, delta0=0.5,
             omega=(0.05, 0.05, 0.05), precision=T.FP64, dt=0.005, nstates=32768)
MIXED = dict(name="mixed_fp32_48", n=(48, 48, 48), d=(1.0, 1.0, 1.0), mu=1.0, u0=0.0, delta0=0.5,
             omega=(0.08, 0.08, 0.02), precision=T.FP32_MIXED, dt=0.005, nstates=8192)


def setup(cfg, vortices, stream=None, precision=None, integrator=T.AB4AM5, A=1.0):
    """Create a context, switch on the trap (regulator frozen with V_+ =
    V_ext), generate the plane-wave states on the device and imprint the
    vortices.  A != 1 evolves the same start with the general functional.
    Returns (ctx, kidx)."""
    n, d = cfg["n"], cfg["d"]
    prec = cfg["precision"] if precision is None else precision
    ec = 0.5 * (np.pi / d[0]) ** 2
    if cfg["nstates"] == n[0] * n[1] * n[2]:
        kidx = all_kidx(n)
    else:
        kidx = lowest_xi_kidx(n, d, cfg["mu"], cfg["u0"], cfg["nstates"])
    run = T.run_config(precision=prec, integrator=integrator, dt=cfg["dt"], selfstart=1, stream=stream)
    ctx = T.Context(T.lattice_3d(n, d), T.functional_slda(cfg["mu"], ec, A=A), run, len(kidx))
    ctx.set_external(harmonic(n, d, cfg["omega"]), freeze_regulator=True)
    ctx.init_plane_waves(kidx, cfg["u0"], cfg["delta0"])
    if len(vortices):
        ctx.imprint_vortices(vortices)
    return ctx, kidx


# ---------------------------------------------------------------------------
# Batched quasi-1D workload: N_z = 256, dz = 1, transverse momenta on a
# 48 x 48 grid (2,304 independent problems), FP32 states with FP64 sums.
Q1D = dict(name="batched_q1d_256", nz=256, dz=1.0, nk=48, mu=1.0, delta0=0.5, omega_z=0.0175, ecut=12.0,
           precision=T.FP32_MIXED, dt=0.005, corner_range=(32, 48))


def q1d_kperp2(nk, dperp):
    """k_perp^2 of every problem: k = 2 pi m / (nk dperp), m in [-nk/2, nk/2),
    x index slow (no de-duplication of equal k_perp^2)."""
    m = np.arange(nk) - nk // 2
    k = 2.0 * np.pi * m / (nk * dperp)
    return (k[:, None] ** 2 + k[None, :] ** 2).ravel()


def q1d_potentials(cfg, bump):
    """(V_trap, V_static = V_trap + bump) on the centred z lattice."""
    z = centered(cfg["nz"], cfg["dz"])
    vt = 0.5 * cfg["omega_z"] ** 2 * z * z
    vb, wb, zb = bump
    return vt, vt + vb * np.exp(-((z - zb) ** 2) / (2.0 * wb * wb))


def q1d_dperp(cfg, hstatic, lo=0.3, hi=3.0, iters=40):
    """Transverse spacing d_perp by bisection on the corner problem (largest
    k_perp^2) so that its kept-state count lies in cfg['corner_range'];
    the count grows with d_perp."""
    lat = T.lattice_q1d(cfg["nz"], cfg["dz"], 1.0, 1.0)
    delta = np.full(cfg["nz"], cfg["delta0"])
    want_lo, want_hi = cfg["corner_range"]

    def count(d):
        kc = 2.0 * (np.pi * (cfg["nk"] // 2) * 2.0 / (cfg["nk"] * d)) ** 2
        _, tot = T.q1d_count(lat, [kc], hstatic, delta, cfg["ecut"])
        return tot

    a, b = lo, hi
    for _ in range(iters):
        m = 0.5 * (a + b)
        c = count(m)
        if c < want_lo:
            a = m
        elif c > want_hi:
            b = m
        else:
            return m, c
    raise RuntimeError("no d_perp gives a corner count in range")


def setup_q1d(cfg, seed, stream=None, precision=None, nk=None, A=1.0):
    """Create the batched quasi-1D context: static states of every problem
    (bump on, U = 0, Delta = delta0) loaded on the device, trap-only V_ext
    for the evolution (bump removed at t = 0), regulator frozen with
    E_c = ecut.  A != 1 evolves the same states with the general functional
    (alpha = A, current potential).  Returns (ctx, info)."""
    import synth
    nk = cfg["nk"] if nk is None else nk
    bump = synth.gaussian_bump(seed)
    vt, vs = q1d_potentials(cfg, bump)
    hstatic = vs - cfg["mu"]
    dperp, corner = q1d_dperp(dict(cfg, nk=nk), hstatic)
    kp2 = q1d_kperp2(nk, dperp)
    delta = np.full(cfg["nz"], cfg["delta0"])
    lat = T.lattice_q1d(cfg["nz"], cfg["dz"], nk * dperp, nk * dperp)
    counts, total = T.q1d_count(lat, kp2, hstatic, delta, cfg["ecut"])
    prec = cfg["precision"] if precision is None else precision
    run = T.run_config(precision=prec, integrator=T.AB4AM5, dt=cfg["dt"], selfstart=1, stream=stream)
    ctx = T.Context(lat, T.functional_slda(cfg["mu"], cfg["ecut"], A=A), run, int(total))
    ctx.set_external(vt, freeze_regulator=True)
    n = ctx.q1d_load_static(kp2, hstatic, delta, cfg["ecut"])
    assert n == total
    info = dict(dperp=dperp, corner_count=int(corner), nproblems=int(kp2.size), states=int(total),
                count_min=int(counts.min()), count_mean=float(counts.mean()), count_max=int(counts.max()),
                histogram=np.histogram(counts, bins=8)[0].tolist(), bump=bump, kperp2=kp2, counts=counts)
    return ctx, info


# ---------------------------------------------------------------------------
# Quasi-2D workload: the geometry of the static quasi-2D configuration (64 x
# 64 x-y lattice, 64 plane waves along z) evolved in time.
Q2D = dict(name="q2d_64", n=(64, 64), nz=64, d=(1.0, 1.0, 1.0), mu=1.0, u0=0.0, delta0=0.5, omega=0.05,
           precision=T.FP32_MIXED, dt=0.005)


def q2d_kidx(cfg):
    """Every x-y lattice momentum in every |k_z| class m = 0 .. N_z/2,
    class-major."""
    nx, ny = cfg["n"]
    m, a, b = np.meshgrid(np.arange(cfg["nz"] // 2 + 1), np.arange(nx), np.arange(ny), indexing="ij")
    return np.stack([a.ravel(), b.ravel(), m.ravel()], axis=1).astype(np.int32)


def setup_q2d(cfg, vortices, stream=None, precision=None, integrator=T.AB4AM5):
    """Quasi-2D context: trap on (regulator frozen with V_+ = V_ext),
    plane-wave states of every class generated on the device, vortices
    imprinted.  Returns (ctx, kidx)."""
    nx, ny = cfg["n"]
    d = cfg["d"]
    prec = cfg["precision"] if precision is None else precision
    ec = 0.5 * (np.pi / d[0]) ** 2
    kidx = q2d_kidx(cfg)
    run = T.run_config(precision=prec, integrator=integrator, dt=cfg["dt"], selfstart=1, stream=stream)
    ctx = T.Context(T.lattice_q2d(nx, ny, cfg["nz"], d), T.functional_slda(cfg["mu"], ec), run, len(kidx))
    X, Y = np.meshgrid(centered(nx, d[0]), centered(ny, d[1]), indexing="ij")
    ctx.set_external(0.5 * cfg["omega"] ** 2 * (X ** 2 + Y ** 2), freeze_regulator=True)
    ctx.init_plane_waves(kidx, cfg["u0"], cfg["delta0"])
    if len(vortices):
        ctx.imprint_vortices(vortices)
    return ctx, kidx


# ---------------------------------------------------------------------------
# Spin-imbalanced batched quasi-1D workload (ASLDA at p != 0): N_z = 64,
# dz = 1, transverse momenta on a 24 x 24 grid, trap omega_z = 0.07,
# mu_a = 1.3, mu_b = 0.5 (a Zeeman split above the pairing gap), static
# states of the A = 1 reduced problem with U = 0, Delta = 0.3, both branches
# with |E| < 6, FP32 states with FP64 sums.
Q1D_ASLDA = dict(name="batched_q1d_aslda_64", nz=64, dz=1.0, nk=24, dperp=2.0, mu_a=1.3, mu_b=0.5, delta0=0.3,
                 omega_z=0.07, ecut=6.0, precision=T.FP32_MIXED, dt=0.005)


def setup_q1d_aslda(cfg, stream=None, precision=None):
    """Create the spin-imbalanced batched quasi-1D context: both branches of
    every problem from the device eigensolver, trap V_ext, regulator frozen
    with the spin averages.  Returns (ctx, info)."""
    kp2 = q1d_kperp2(cfg["nk"], cfg["dperp"])
    z = centered(cfg["nz"], cfg["dz"])
    vt = 0.5 * cfg["omega_z"] ** 2 * z * z
    delta = np.full(cfg["nz"], cfg["delta0"])
    L_perp = cfg["nk"] * cfg["dperp"]
    lat = T.lattice_q1d(cfg["nz"], cfg["dz"], L_perp, L_perp)
    ha, hb = vt - cfg["mu_a"], vt - cfg["mu_b"]
    counts, total = T.q1d_count_spin(lat, kp2, ha, hb, delta, cfg["ecut"])
    prec = cfg["precision"] if precision is None else precision
    run = T.run_config(precision=prec, integrator=T.AB4AM5, dt=cfg["dt"], selfstart=1, stream=stream)
    ctx = T.Context(lat, T.functional_aslda(cfg["mu_a"], cfg["mu_b"], cfg["ecut"]), run, int(total))
    ctx.set_external(vt, freeze_regulator=True)
    n = ctx.q1d_load_static_spin(kp2, ha, hb, delta, cfg["ecut"])
    assert n == total
    return ctx, dict(nproblems=int(kp2.size), states=int(total), count_min=int(counts.min()),
                     count_max=int(counts.max()))


# ---------------------------------------------------------------------------
# Spin-imbalanced 3D workload (ASLDA at p != 0): the 32^3 trapped gas of the
# headline with mu_a = 1.4, mu_b = 0.6 (a Zeeman split above the start's
# pairing gap), the 16,384 momenta with the smallest |xi| of the uniform
# start, both branches of each (32,768 states), FP64.
ASLDA3D = dict(name="aslda_fp64_32", n=(32, 32, 32), d=(1.0, 1.0, 1.0), mu_a=1.4, mu_b=0.6, u0=0.0, delta0=0.3,
               omega=(0.05, 0.05, 0.05), precision=T.FP64, dt=0.005, nmomenta=16384)


def setup_aslda3d(cfg, stream=None, precision=None):
    """Create the spin-imbalanced 3D context: trap on (regulator frozen with
    the spin averages), both branches of the uniform start generated on the
    device.  Returns (ctx, kidx)."""
    n, d = cfg["n"], cfg["d"]
    prec = cfg["precision"] if precision is None else precision
    ec = 0.5 * (np.pi / d[0]) ** 2
    mubar = 0.5 * (cfg["mu_a"] + cfg["mu_b"])
    kidx = lowest_xi_kidx(n, d, mubar, cfg["u0"], cfg["nmomenta"])
    run = T.run_config(precision=prec, integrator=T.AB4AM5, dt=cfg["dt"], selfstart=1, stream=stream)
    ctx = T.Context(T.lattice_3d(n, d), T.functional_aslda(cfg["mu_a"], cfg["mu_b"], ec), run, 2 * len(kidx))
    ctx.set_external(harmonic(n, d, cfg["omega"]), freeze_regulator=True)
    ctx.init_plane_waves(kidx, cfg["u0"], cfg["delta0"])
    return ctx, kidx
