"""Uniform-system solutions: the continuum SLDA state at p = 0 and the
self-consistent uniform state on a periodic lattice.

Both are scalar problems; they serve as pins for the lattice machinery and
as plane-wave starting points (the paper's uniform-system solution used to
start TD runs quickly, Sec. 4.5.1).

Part of the oracle: test infrastructure only (tests, the smoke check and
the benchmark's CPU baseline use it; the product path never does).
"""
import numpy as np
from scipy import integrate, optimize

from . import functional as F
from . import lattice as L


def continuum_slda(fun, ec_over_ef=100.0, kF=1.0):
    """Homogeneous spin-symmetric superfluid in the continuum with the
    regularised functional.  States with A k^2/2 + U - mu < E_c are kept
    (k < k_c, the same k_c as in Lambda_c; V_+ = U, the static iteration
    order).  Solves the number and gap equations for (mu, Delta) at total
    density n = kF^3 / (3 pi^2).  Returns dict with E/E_FG, Delta/eF, mu/eF."""
    n = kF ** 3 / (3 * np.pi ** 2)
    ef = 0.5 * kF ** 2
    ec = ec_over_ef * ef
    A = fun.A

    def parts(mu, d):
        U = fun.B * F.eF(n) - d ** 2 / (3 * fun.C * n ** (2.0 / 3.0))
        kc = np.sqrt(2 * (ec + mu - U) / A)
        xi = lambda k: 0.5 * A * k * k + U - mu
        E = lambda k: np.sqrt(xi(k) ** 2 + d ** 2)
        v2 = lambda k: 0.5 * (1 - xi(k) / E(k))
        k0 = np.sqrt(max(2 * (mu - U) / A, 0.0))
        pts = [k0] if 0 < k0 < kc else None
        q = lambda g: integrate.quad(g, 0, kc, points=pts, limit=400, epsabs=0, epsrel=1e-12)[0]
        rho_s = q(lambda k: k * k * v2(k)) / (2 * np.pi ** 2)
        nu = q(lambda k: k * k * d / (2 * E(k))) / (2 * np.pi ** 2)
        tau_s = q(lambda k: k ** 4 * v2(k)) / (2 * np.pi ** 2)
        lam = float(F.lambda_c(U, mu, ec, A))
        ig = n ** (1.0 / 3.0) / fun.C - lam
        return U, rho_s, nu, tau_s, ig

    def eqs(x):
        mu, d = x
        U, rho_s, nu, tau_s, ig = parts(mu, d)
        return [2 * rho_s / n - 1.0, (d * ig + nu) / ef]

    mu, d = optimize.fsolve(eqs, [0.4 * ef, 0.5 * ef], xtol=1e-13)
    U, rho_s, nu, tau_s, ig = parts(mu, d)
    g = 1.0 / ig
    edens = A * tau_s + 0.6 * fun.B * n * F.eF(n) + g * nu * nu
    return dict(E_over_EFG=edens / (0.6 * n * ef), delta_over_eF=d / ef, mu_over_eF=mu / ef,
                residual=max(abs(v) for v in eqs([mu, d])))


def lattice_uniform(lat, fun, mu, lam, delta_guess=0.5, U_guess=0.0):
    """Self-consistent uniform state on the lattice at fixed mu, T = 0, with
    every lattice momentum kept (one E>0 state per k): find constant (U,
    Delta) such that the densities of the plane-wave eigenstates reproduce
    them through the functional.  lam is the (constant) frozen regulator.
    Returns (U, Delta)."""
    k2 = lat.k2.ravel()

    def out(x):
        U, d = x
        xi = 0.5 * k2 + U - mu
        E = np.sqrt(xi ** 2 + d ** 2)
        rho = np.sum(0.5 * (1 - xi / E)) / lat.V
        nu = np.sum(d / (2 * E)) / lat.V
        Uo, Do, _ = F.potentials(np.array([rho]), np.array([nu]), np.array([lam]), fun)
        return np.array([Uo[0] - U, np.real(Do[0]) - d])

    sol = optimize.fsolve(out, [U_guess, delta_guess], xtol=1e-15)
    for _ in range(3):   # polish with Newton from fsolve's answer
        sol = optimize.fsolve(out, sol, xtol=1e-16)
    return float(sol[0]), float(sol[1])


def free_gas_lattice_count(n, d, mu):
    """Brute-force count over lattice momenta of an n^3 box: number of
    occupied k (k^2/2 < mu) per spin and the sum of k^2/2 over them."""
    k = L.kgrid(n, d)
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    e = 0.5 * (kx ** 2 + ky ** 2 + kz ** 2)
    occ = e < mu
    return int(np.count_nonzero(occ)), float(np.sum(e[occ]))
