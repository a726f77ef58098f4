"""Pins of the oracle's static quasi-2D solver (Alg. MapK + linear mixing +
Eq. update-mu): the dense BdG matrix against the uniform dispersion, the
uniform fixed point against the scalar lattice k-sum, and the fixed-N
solve with an obstacle."""
import numpy as np
import pytest

from oracle import lattice as L, functional as F, uniform as UN, static as ST
import synth

FUN = F.Functional(F.SLDA)
EC = 0.5 * np.pi ** 2


@pytest.mark.parametrize("kz_index", [0, 1, 2])
def test_q2d_matrix_uniform_dispersion(kz_index):
    """P2 (quasi-2D): with constant hfield c and Delta d the eigenvalues of
    the dense matrix are +-sqrt((k_perp^2/2 + k_z^2/2 + c)^2 + d^2) over the
    x-y lattice momenta (Nyquist kept)."""
    g = ST.GeometryQ2D(6, 4, 4, 1.0, 1.3, 0.9)
    c, d = -0.7, 0.45
    kz = g.kz[kz_index]
    E = np.linalg.eigvalsh(ST.build_h(g, np.full(g.shape, c), np.full(g.shape, d), kz))
    kx, ky = L.kgrid(6, 1.0), L.kgrid(4, 1.3)
    xi = 0.5 * (kx[:, None] ** 2 + ky[None, :] ** 2) + 0.5 * kz * kz + c
    Ek = np.sqrt(xi ** 2 + d * d).ravel()
    ref = np.sort(np.concatenate([Ek, -Ek]))
    assert np.abs(E - ref).max() < 1e-12


def test_q2d_multiplicities_cover_the_kz_grid():
    g = ST.GeometryQ2D(4, 4, 8)
    kz_all = np.abs(L.kgrid(8, 1.0))
    for kz, w in zip(g.kz, g.mult):
        assert np.sum(np.isclose(kz_all, kz)) == w


def test_uniform_fixed_point_matches_lattice_k_sum():
    """P12: without an external potential, at fixed mu, the static solve
    from a uniform guess converges to a uniform state, and that state is the
    solution of the scalar k-sum over the N_x x N_y x N_z lattice with the
    same regulator (oracle.uniform.lattice_uniform) to 1e-9."""
    g = ST.GeometryQ2D(6, 6, 4)
    mu = 1.0
    vext = np.zeros(g.shape)
    U, D, mu_out, it, ok = ST.solve(g, FUN, vext, np.full(g.shape, -0.2), np.full(g.shape, 0.3), mu, EC,
                                    mix=0.5, tol=1e-11, maxit=400)
    assert ok
    assert np.ptp(U) < 1e-10 and np.ptp(np.real(D)) < 1e-10
    lam = float(F.lambda_c(np.array(U.mean()), mu, EC))
    lat = L.Lattice(6, 6, 4)
    Uk, Dk = UN.lattice_uniform(lat, FUN, mu, lam, delta_guess=float(np.real(D.mean())), U_guess=float(U.mean()))
    assert abs(Uk - U.mean()) < 1e-9
    assert abs(Dk - np.real(D.mean())) < 1e-9


def test_fixed_n_solve_with_obstacle():
    """Fixed-N mode with a trap and one Gaussian obstacle: the iteration
    converges to r < 1e-8, N equals N_req, and the converged potentials are
    a fixed point of MapK (one more application moves them by < 1e-7)."""
    g = ST.GeometryQ2D(8, 8, 4)
    X, Y = g.coords()
    amp, wid, cen = synth.obstacles(5, 8.0)
    vext = 0.5 * 0.4 ** 2 * (X ** 2 + Y ** 2) + amp[0] * 0.5 * np.exp(
        -((X - cen[0, 0] / 4) ** 2 + (Y - cen[0, 1] / 4) ** 2) / (2 * (wid[0] / 4) ** 2))
    # N_req from the same trap at mu = 1 without the obstacle, a few iterations
    U0, D0 = np.full(g.shape, -0.2), np.full(g.shape, 0.25)
    _, _, _, _, N_req = ST.map_k(g, FUN, 0.5 * 0.4 ** 2 * (X ** 2 + Y ** 2), U0, D0, 1.0, EC)
    hist = []
    U, D, mu, it, ok = ST.solve(g, FUN, vext, U0, D0, 0.8, EC, mix=0.5, a_mu=0.5, N_req=N_req, tol=1e-8,
                                maxit=600, history=hist)
    assert ok, hist[-1]
    Uo, Do, rho, nu, N = ST.map_k(g, FUN, vext, U, D, mu, EC)
    assert abs(N - N_req) / N_req < 1e-7
    assert np.abs(Uo - U).max() < 1e-7 and np.abs(Do - D).max() < 1e-7


def test_broyden_terminates_on_linear_maps():
    """The modified Broyden mixing with w0 -> 0 and a history as long as the
    dimension is Anderson mixing, whose iterates on a linear map p -> A p + b
    reach the fixed point in at most dim + 1 steps (they are GMRES's): the
    error is still > 1e-5 after dim steps and < 1e-9 after dim + 1, for two
    mixing parameters; linear mixing is far from converged by then.  With no
    history the step is linear mixing exactly."""
    rng = np.random.default_rng(0)
    n = 10
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(rng.uniform(-0.9, 0.9, n)) @ Q.T + 0.05 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    ps = np.linalg.solve(np.eye(n) - A, b)
    for mix in (0.5, 1.0):
        B = ST.Broyden(n, mix, w0=1e-10)
        p = np.zeros(n)
        errs = []
        for _ in range(n + 1):
            p = B.step(p, A @ p + b)
            errs.append(np.linalg.norm(p - ps) / np.linalg.norm(ps))
        assert errs[n - 1] > 1e-5 and errs[n] < 1e-9, errs
        q = np.zeros(n)
        for _ in range(n + 1):
            q = q + mix * (A @ q + b - q)
        assert np.linalg.norm(q - ps) / np.linalg.norm(ps) > 1e-2
    B0 = ST.Broyden(0, 0.3)
    p, Kp = rng.standard_normal(n), rng.standard_normal(n)
    for _ in range(3):
        assert np.array_equal(B0.step(p, Kp), p + 0.3 * (Kp - p))


def test_broyden_solve_reaches_the_linear_mixing_fixed_point():
    """Fixed-N solve with a trap and an obstacle: modified Broyden mixing
    (history 8) converges to the same potentials, mu and N as linear mixing
    (both to r < 1e-10) in fewer iterations."""
    g = ST.GeometryQ2D(8, 8, 4)
    X, Y = g.coords()
    amp, wid, cen = synth.obstacles(5, 8.0)
    trap = 0.5 * 0.4 ** 2 * (X ** 2 + Y ** 2)
    vext = trap + amp[0] * 0.5 * np.exp(
        -((X - cen[0, 0] / 4) ** 2 + (Y - cen[0, 1] / 4) ** 2) / (2 * (wid[0] / 4) ** 2))
    U0, D0 = np.full(g.shape, -0.2), np.full(g.shape, 0.25)
    _, _, _, _, N_req = ST.map_k(g, FUN, trap, U0, D0, 1.0, EC)
    kw = dict(mix=0.5, a_mu=0.5, N_req=N_req, tol=1e-10, maxit=800)
    Ul, Dl, mul, itl, okl = ST.solve(g, FUN, vext, U0, D0, 0.8, EC, **kw)
    Ub, Db, mub, itb, okb = ST.solve(g, FUN, vext, U0, D0, 0.8, EC, broyden=8, **kw)
    assert okl and okb
    assert itb < itl, (itb, itl)
    assert np.abs(Ub - Ul).max() < 1e-8 and np.abs(Db - Dl).max() < 1e-8 and abs(mub - mul) < 1e-8


def test_q1d_static_classes_cover_the_transverse_grid():
    """The quasi-1D classes (|k_y|, |k_z|) with multiplicities w_y w_z cover
    every transverse momentum pair of the N_y x N_z plane-wave grid once."""
    g = ST.GeometryQ1DStatic(6, 4, 8, 1.0, 1.2, 0.9)
    ky, kz = L.kgrid(4, 1.2), L.kgrid(8, 0.9)
    kp = np.sqrt(ky[:, None] ** 2 + kz[None, :] ** 2).ravel()
    assert g.mult.sum() == kp.size
    # each distinct |k_perp| carries as many pairs as the classes that share it
    for k in np.unique(np.round(kp, 10)):
        assert np.isclose(g.mult[np.isclose(g.kz, k)].sum(), np.sum(np.isclose(kp, k)))


def test_q1d_static_is_the_q2d_one_for_y_independent_fields():
    """Exact mode reduction (Sec. 3.1): for fields that do not depend on y,
    the quasi-2D map (an N_y-site y lattice, spectral D2) and the quasi-1D
    map (N_y plane waves along y, same L_y) give the same densities and
    potentials, and a fixed-N solve of a trap in x converges to the same
    fields and mu in both geometries."""
    nx, ny, nz = 8, 4, 4
    g2 = ST.GeometryQ2D(nx, ny, nz, 1.0, 1.5, 1.0)
    g1 = ST.GeometryQ1DStatic(nx, ny, nz, 1.0, 1.5, 1.0)
    x = g1.coords()[0]
    vx = 0.5 * 0.3 ** 2 * x ** 2
    U1 = 0.1 * synth.uniform_field(51, nx)
    D1 = 0.4 + 0.1 * synth.uniform_field(52, nx)
    mu = 0.9
    b = lambda f: np.repeat(f[:, None], ny, axis=1)
    o1 = ST.map_k(g1, FUN, vx, U1, D1, mu, EC)
    o2 = ST.map_k(g2, FUN, b(vx), b(U1), b(D1), mu, EC)
    for a1, a2 in zip(o1[:4], o2[:4]):
        assert np.abs(b(a1) - a2).max() < 1e-12 * max(1.0, np.abs(a2).max())
    assert o1[4] == pytest.approx(o2[4], rel=1e-13)
    N_req = 0.9 * o1[4]
    s1 = ST.solve(g1, FUN, vx, np.zeros(nx), np.full(nx, 0.5), mu, EC, N_req=N_req, maxit=400)
    s2 = ST.solve(g2, FUN, b(vx), np.zeros((nx, ny)), np.full((nx, ny), 0.5), mu, EC, N_req=N_req, maxit=400)
    assert s1[4] and s2[4]
    assert np.abs(b(s1[0]) - s2[0]).max() < 1e-7 and np.abs(b(s1[1]) - s2[1]).max() < 1e-7
    assert s1[2] == pytest.approx(s2[2], abs=1e-7)
