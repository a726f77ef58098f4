"""Time integration of the TDSLDA equations (paper Sec. 3.3).

Equation of motion with the instantaneous-energy shift (Eqs.
shorttdproblem-mod and ABM-f):

    d phi_n / dt = f(phi)_n = -i [ H(phi) - <H>_n ] phi_n,
    <H>_n = int phi_n^dagger H(phi) phi_n dV,

where H(phi) is built from the densities of all states.  Integrators:
AB3AM4, AB4AM5 and AB5AM5 (Eqs. AB3-AB5, AM4-AM5) in the memory schedule of
Alg. AB4AM5, started either from a stationary history or by the Taylor
predictor-corrector of Eq. Taylor-exp.

Part of the oracle: test infrastructure only (tests, the smoke check and
the benchmark's CPU baseline use it; the product path never does).
"""
import numpy as np
from math import factorial

from . import bdg
from . import densities as D
from . import functional as F
from . import lattice as L

# Adams-Bashforth predictors (Eqs. AB3, AB4, AB5): weights of f_{k-1}, f_{k-2}, ...
AB = {
    3: np.array([23.0, -16.0, 5.0]) / 12.0,
    4: np.array([55.0, -59.0, 37.0, -9.0]) / 24.0,
    5: np.array([1901.0, -2774.0, 2616.0, -1274.0, 251.0]) / 720.0,
}
# Adams-Moulton correctors (Eqs. AM4, AM5): weights of f(phi^p), f_{k-1}, f_{k-2}, ...
AM = {
    4: np.array([9.0, 19.0, -5.0, 1.0]) / 24.0,
    5: np.array([251.0, 646.0, -264.0, 106.0, -19.0]) / 720.0,
}
SCHEMES = {"AB3AM4": (3, 4), "AB4AM5": (4, 5), "AB5AM5": (5, 5)}


def history_depth(scheme):
    """Number of stored f buffers: AB5AM5 keeps five, AB4AM5 four, AB3AM4
    three (Sec. 3.3), plus the buffer of phi itself."""
    p, c = SCHEMES[scheme]
    return max(len(AB[p]), len(AM[c]) - 1)


class Geometry3D:
    """Full 3D mode: states live on the whole lattice."""

    def __init__(self, lat):
        self.lat = lat
        self.dV = lat.dV          # measure of the state normalisation
        self.dV_energy = lat.dV   # measure of energy / particle-number integrals
        self.shape = lat.shape

    def apply_h(self, phi, hfield, delta, alpha=None, avec=None):
        if alpha is None and avec is None:
            return bdg.apply_h(phi, hfield, delta, self.lat)
        return bdg.apply_h_general(phi, hfield, delta, 1.0 if alpha is None else alpha, avec, self.lat)

    def rho_nu(self, phi, wu, wv):
        return D.local_densities(phi, wu, wv)

    def rho_nu_j(self, phi, wu, wv):
        rho, _, nu, j = D.spin_symmetric(phi, wu, wv, self.lat)
        return rho, nu, j

    def friction_sources(self, phi, wu, wv):
        """What the dissipative fields of the quantum-friction evolution need
        (Sec. 5.2, correcting the initial state by a time-dependent approach)
        on the full 3D lattice:
          div j = sum_d D1_d j_d (D1 with the Nyquist mode zeroed, as j itself),
          B'    = -1/2 sum_n (f_v - f_u) [u lap v^* + v^* lap u]
                  (lap = the full spectral Laplacian of Eq. D2; the weights of nu),
          N     = int rho_+ d^3r.
        Returns (div_j, B', N)."""
        lat = self.lat
        rho, _, _, j = D.spin_symmetric(phi, wu, wv, lat)
        div_j = np.zeros(lat.shape)
        for d in range(3):
            div_j += np.real(L.spectral_derivative(j[d], lat.k[d], d, 1))
        w = (np.asarray(wv, float) - np.asarray(wu, float)).reshape(-1, 1, 1, 1)
        Bp = np.zeros(lat.shape, complex)
        for s in range(0, phi.shape[0], D.CHUNK):
            u, v = phi[s:s + D.CHUNK, 0], phi[s:s + D.CHUNK, 1]
            lu, lv = L.laplacian(u, lat), L.laplacian(v, lat)
            Bp += -0.5 * np.sum(w[s:s + D.CHUNK] * (u * np.conj(lv) + np.conj(v) * lu), axis=0)
        N = self.dV_energy * np.sum(2.0 * rho)
        return div_j, Bp, N

    def full_densities(self, phi, wu, wv):
        return D.spin_symmetric(phi, wu, wv, self.lat)


class Friction:
    """Dissipative mean fields (quantum friction) of Sec. 5.2, correcting
    the initial state by a time-dependent approach, added to U and Delta at
    every field build:
        U_diss     = -(alpha / rho0) div j,
        Delta_diss = Delta [beta sin(theta_nu - theta_B') + i gamma~],
        gamma~     = gamma (N - N_req) / N_req   (0 without N_req),
    theta_nu = arg nu, theta_B' = arg B' with B' from the geometry's
    friction_sources.  rho0 is a reference density (a parameter here)."""

    def __init__(self, alpha=0.0, beta=0.0, gamma=0.0, rho0=1.0, N_req=None):
        self.alpha, self.beta, self.gamma = float(alpha), float(beta), float(gamma)
        self.rho0, self.N_req = float(rho0), N_req

    def terms(self, geom, phi, wu, wv, nu, delta):
        div_j, Bp, N = geom.friction_sources(phi, wu, wv)
        Ud = -self.alpha / self.rho0 * div_j
        gt = 0.0 if self.N_req is None else self.gamma * (N - self.N_req) / self.N_req
        Dd = delta * (self.beta * np.sin(np.angle(nu) - np.angle(Bp)) + 1j * gt)
        return Ud, Dd


class TDSystem:
    """Everything the right-hand side f needs besides the states.

    mu: chemical potential (fixed in TD); vext: external potential (static
    after t=0); lam: frozen regulator Lambda_c(r) (reading: computed once,
    never refreshed, so that U is the exact derivative of the energy);
    wu, wv: frozen thermal weights f(E_n), f(-E_n) (Sec. 2.5).
    frozen=(hfield, delta) switches to linear mode (fields not rebuilt);
    friction (a Friction) adds the dissipative fields.
    dext: external pairing potential Delta_ext(r) (Sec. 2.2, Eq. E_tot; None
    = 0).  The off-diagonal of H is Delta + Delta_ext (Eq. HpsiEpsi and its
    time-dependent form), in linear mode too; Delta itself stays -g nu."""

    def __init__(self, geom, fun, mu, vext, lam, wu, wv, frozen=None, friction=None, dext=None):
        self.geom, self.fun, self.mu = geom, fun, float(mu)
        self.friction = friction
        self.dext = None if dext is None else np.asarray(dext, complex)
        self.vext = np.asarray(vext, float)
        self.lam = np.asarray(lam, float)
        self.wu = np.asarray(wu, float)
        self.wv = np.asarray(wv, float)
        self.frozen = frozen
        self.n_f_evals = 0

    def fields(self, phi):
        """Densities -> potentials -> (hfield = U + V_ext - mu, the
        off-diagonal field Delta + Delta_ext, alpha, A_vec).  alpha and
        A_vec are None for the A = 1 functional (Eq. h_sigma_A1); with
        A != 1 the current j enters every field build (alpha = A, A_vec =
        (1 - A) j / rho and the current term of U).  frozen = (hfield,
        Delta) or (hfield, Delta, alpha, A_vec)."""
        if self.frozen is not None:
            hf, de = self.frozen[0], self.frozen[1]
            al = self.frozen[2] if len(self.frozen) > 2 else None
            av = self.frozen[3] if len(self.frozen) > 3 else None
            return hf, (de if self.dext is None else de + self.dext), al, av
        al = av = None
        if self.fun.A != 1.0:
            if self.friction is not None:
                raise NotImplementedError("quantum friction is written for the A = 1 functional")
            rho, nu, j = self.geom.rho_nu_j(phi, self.wu, self.wv)
            U, delta, al, av = F.potentials_general(rho, nu, j, self.lam, self.fun)
        else:
            rho, nu = self.geom.rho_nu(phi, self.wu, self.wv)
            U, delta, _ = F.potentials(rho, nu, self.lam, self.fun)
        if self.friction is not None:
            Ud, Dd = self.friction.terms(self.geom, phi, self.wu, self.wv, nu, delta)
            U, delta = U + Ud, delta + Dd
        if self.dext is not None:
            delta = delta + self.dext
        return U + self.vext - self.mu, delta, al, av

    def expect(self, phi, hphi):
        ax = tuple(range(1, phi.ndim))
        return self.geom.dV * np.real(np.sum(np.conj(phi) * hphi, axis=ax))

    def f(self, phi):
        """f(phi) of Eq. ABM-f for normalised phi."""
        self.n_f_evals += 1
        hphi = self.geom.apply_h(phi, *self.fields(phi))
        e = self.expect(phi, hphi)
        return -1j * (hphi - _bc(e, phi) * phi)

    def normalize(self, phi):
        return D.normalize(phi, self.geom.dV)


def _bc(x, phi):
    return np.asarray(x).reshape((-1,) + (1,) * (phi.ndim - 1))


def abm_step(sys, phi, hist, dt, scheme="AB4AM5"):
    """One step of the predictor-corrector in the order of Alg. AB4AM5
    (the AB3AM4 and AB5AM5 variants follow the same pattern):

      p   = phi + dt * sum_j b_j f_{k-j}                      (predictor)
      c   = phi + dt * sum_{j>=1} a_j f_{k-j}                 (corrector part)
      p  <- p / |p|;  phi_new = c + dt a_0 f(p)
      phi_new <- phi_new / |phi_new|;  f_k = f(phi_new)

    hist[0] = f_{k-1}, hist[1] = f_{k-2}, ...  Returns (phi_new, hist)."""
    pb, cb = SCHEMES[scheme]
    b, a = AB[pb], AM[cb]
    p = phi + dt * sum(b[j] * hist[j] for j in range(len(b)))
    c = phi + dt * sum(a[j + 1] * hist[j] for j in range(len(a) - 1))
    p = sys.normalize(p)
    phi_new = c + dt * a[0] * sys.f(p)
    phi_new = sys.normalize(phi_new)
    fk = sys.f(phi_new)
    return phi_new, [fk] + list(hist[:-1])


def taylor_apply(sys, phi, fields, shift, tau, r):
    """sum_{k=0}^{r} (-i tau)^k / k! (H - shift)^k phi with H fixed by fields
    (the tuple TDSystem.fields returns)."""
    term = phi
    out = phi.copy()
    for k in range(1, r + 1):
        hterm = sys.geom.apply_h(term, *fields) - _bc(shift, phi) * term
        term = (-1j * tau / k) * hterm
        out = out + term
    return out


def taylor_step(sys, phi, dt, r=5):
    """One start-up step by the Taylor predictor-corrector of Eq. Taylor-exp.

    Readings where the paper is silent: the operator is the shifted one,
    H - <H>_n, with <H>_n taken on the state the H is built from (phi at t
    for the half step, the mid-point state for the full step), so the start
    matches the phases of the shifted ABM trajectory; both the mid-point and
    the end state are renormalised, as the ABM steps are."""
    fl = sys.fields(phi)
    e0 = sys.expect(phi, sys.geom.apply_h(phi, *fl))
    phim = sys.normalize(taylor_apply(sys, phi, fl, e0, 0.5 * dt, r))
    flm = sys.fields(phim)
    em = sys.expect(phim, sys.geom.apply_h(phim, *flm))
    return sys.normalize(taylor_apply(sys, phi, flm, em, dt, r))


def start(sys, phi0, dt, scheme="AB4AM5", selfstart=1, r=5):
    """Initialise the multistep history.

    selfstart = 0: the states are taken as stationary, every history slot
    holds f(phi_0) (zero for an exact stationary state).
    selfstart = 1: Hd - 1 Taylor steps (Hd = history depth: 3 for AB4AM5)
    give phi_1 ... phi_{Hd-1}; the history is f of those states.
    Returns (phi, hist, n_startup_steps)."""
    hd = history_depth(scheme)
    phi0 = sys.normalize(phi0)
    if selfstart == 0:
        f0 = sys.f(phi0)
        return phi0, [f0] * hd, 0
    phis = [phi0]
    for _ in range(hd - 1):
        phis.append(taylor_step(sys, phis[-1], dt, r))
    hist = [sys.f(p) for p in reversed(phis)]
    return phis[-1], hist, hd - 1


def evolve(sys, phi0, dt, nsteps, scheme="AB4AM5", selfstart=1, r=5, callback=None):
    """Start-up followed by nsteps ABM steps.  callback(step, phi) is called
    after every step.  Returns the final states."""
    phi, hist, _ = start(sys, phi0, dt, scheme, selfstart, r)
    for s in range(nsteps):
        phi, hist = abm_step(sys, phi, hist, dt, scheme)
        if callback is not None:
            callback(s + 1, phi)
    return phi


def observables(sys, phi):
    """Energy terms of Sec. 3.2 (the external pairing energy included),
    particle number N = int rho_+ dV and the free-gas normalisation
    E_FG = 3/5 N eF of the uniform system with the same mean density."""
    g = sys.geom
    rho, tau, nu, j = g.full_densities(phi, sys.wu, sys.wv)
    terms = F.energy_terms(rho, tau, j, nu, sys.lam, sys.vext, sys.fun, g.dV_energy, dext=sys.dext)
    N = g.dV_energy * np.sum(2.0 * rho)
    vol = g.dV_energy * np.prod(rho.shape)
    terms["N"] = N
    terms["EFG"] = 0.6 * N * F.eF(N / vol)
    return terms


def gram(phi, dV):
    """Overlap matrix int phi_n^dagger phi_m dV."""
    A = phi.reshape(phi.shape[0], -1)
    return dV * (np.conj(A) @ A.T)
