"""SLDA-type energy density functional, pairing field and regularisation
(paper Sec. 2.4 and 2.6), written for the spin-symmetric case.

Notation: rho is the density of ONE spin component (rho_a = rho_b = rho),
rho_p = rho_a + rho_b = 2 rho is the total density (Sec. 2.4, rho_+),
tau and j are per spin component, nu is the anomalous density.

Part of the oracle: test infrastructure only (tests, the smoke check and
the benchmark's CPU baseline use it; the product path never does).
"""
import numpy as np

SLDA = "slda"
BDG = "bdg"

C_SLDA = -11.11          # C(p) of the ASLDA parametrisation
RHO_FLOOR = 1e-14        # guard in rho^(1/3), rho^(-2/3)


def aslda_A(p):
    """A_a(p) of the ASLDA parametrisation (Sec. 2.4, ASLDA item)."""
    return 1.094 + 0.156 * p * (1 - 2 * p ** 2 / 3 + p ** 4 / 5) - 0.532 * p ** 2 * (1 - p ** 2 + p ** 4 / 3)


def aslda_B(p, force_a1=False):
    """B(p) of the ASLDA parametrisation.  B is defined through A_a and A_b;
    with the A_sigma = 1 option the same formula is evaluated with
    A_a = A_b = 1 (reading: forcing A=1 recomputes B, which keeps the
    equation of state the formula encodes)."""
    if force_a1:
        Aa = Ab = 1.0
    else:
        Aa, Ab = aslda_A(p), aslda_A(-p)
    return 2.0 ** (2.0 / 3.0) * (0.357 + 0.642 * p ** 2
                                 - Aa * ((1 + p) / 2) ** (5.0 / 3.0)
                                 - Ab * ((1 - p) / 2) ** (5.0 / 3.0))


class Functional:
    """Constants of the functional in the spin-symmetric limit.

    kind = SLDA: A, B, C from ASLDA at p = 0 (optionally A forced to 1).
    kind = BDG:  A = 1, B = 0 and the bare coupling 1/g = 1/(4 pi a_s)
                 (Eq. HBdG)."""

    def __init__(self, kind=SLDA, force_a1=True, a_s=None):
        self.kind = kind
        if kind == SLDA:
            self.A = 1.0 if force_a1 else aslda_A(0.0)
            self.B = aslda_B(0.0, force_a1=force_a1)
            self.C = C_SLDA
            self.inv_g_bdg = None
        elif kind == BDG:
            if a_s is None:
                raise ValueError("BdG functional needs a_s")
            self.A, self.B, self.C = 1.0, 0.0, None
            self.inv_g_bdg = 1.0 / (4.0 * np.pi * a_s)
        else:
            raise ValueError(kind)


def eF(rho_p):
    """Fermi energy of the total density, (3 pi^2 rho_+)^(2/3) / 2."""
    return 0.5 * (3.0 * np.pi ** 2 * rho_p) ** (2.0 / 3.0)


def lambda_c(vplus, mu, ec, A=1.0):
    """Regulator Lambda_c of Eq. Creg, evaluated pointwise.

    k_0 and k_c solve A k_0^2/2 + V_+ - mu = 0 and A k_c^2/2 + V_+ - mu = E_c.
    Where k_0^2 < 0 (mu below V_+) the paper is silent; the analytic
    continuation k_0 = i kappa is used, which turns the bracket into
    1 + (kappa/k_c) arctan(kappa/k_c)."""
    vplus = np.asarray(vplus, dtype=float)
    k0sq = 2.0 * (mu - vplus) / A
    kcsq = 2.0 * (ec + mu - vplus) / A
    if np.any(kcsq <= 0):
        raise ValueError("E_c below the local band bottom")
    kc = np.sqrt(kcsq)
    br = np.empty_like(kc)
    pos = k0sq > 0
    k0 = np.sqrt(np.where(pos, k0sq, 1.0))
    kap = np.sqrt(np.where(pos, 1.0, -k0sq))
    br_pos = 1.0 - k0 / (2 * kc) * np.log((kc + k0) / (kc - k0))
    br_neg = 1.0 + kap / kc * np.arctan(kap / kc)
    br = np.where(pos, br_pos, br_neg)
    return kc / (2.0 * np.pi ** 2 * A) * br


def inv_geff(rho, lam, fun):
    """1/g_eff = rho_+^(1/3)/C - Lambda_c (Eq. Creg, SLDA), or
    1/(4 pi a_s) - Lambda_c (BdG).

    Reading of the garbled Eq. Creg naming: the regularised coupling is the
    bare one minus the regulator, with C = -11.11 finite; the regulator is
    frozen (computed once, passed in)."""
    if fun.kind == BDG:
        return fun.inv_g_bdg - lam
    rho_p = np.maximum(2.0 * rho, RHO_FLOOR)
    return rho_p ** (1.0 / 3.0) / fun.C - lam


def potentials(rho, nu, lam, fun):
    """Mean field U and pairing field Delta from the densities.

    Delta = -g_eff nu (Eq. Delta with the regularised coupling).  U is the
    functional derivative dE/drho_sigma of the A=1 energy density with the
    regulator frozen: U = B eF(rho_+) - |Delta|^2 / (3 C rho_+^(2/3)); for the
    BdG functional U = 0 (B = 0, coupling independent of density).
    Returns (U, Delta, g_eff)."""
    g = 1.0 / inv_geff(rho, lam, fun)
    delta = -g * nu
    if fun.kind == BDG:
        U = np.zeros_like(rho)
    else:
        rho_p = np.maximum(2.0 * rho, RHO_FLOOR)
        U = fun.B * eF(2.0 * rho) - np.abs(delta) ** 2 / (3.0 * fun.C * rho_p ** (2.0 / 3.0))
    return U, delta, g


def potentials_general(rho, nu, j, lam, fun):
    """Potentials of the SLDA-type functional with A != 1 (Sec. 2.3, the
    functional derivatives of Eq. h_sigma) in the spin-symmetric case, per
    spin component:
        alpha = 2 dE/dtau_sigma = A,
        A_vec = dE/dj_sigma     = (1 - A) j / rho,
        U     = dE/drho_sigma   = B eF(rho_+) - |Delta|^2 / (3 C rho_+^(2/3))
                                  - (1 - A) |j|^2 / (2 rho^2),
        Delta = -g_eff nu,
    from the intrinsic part (A/2)(tau - j^2/rho) and the centre-of-mass part
    j^2/(2 rho) of the energy density (Eqs. sldae-functional,
    sldae-functional-CM).  j: three arrays (per spin).  Returns (U, Delta,
    alpha, A_vec)."""
    U, delta, _ = potentials(rho, nu, lam, fun)
    rho_s = np.maximum(rho, RHO_FLOOR / 2)
    jsq = sum(np.abs(c) ** 2 for c in j)
    c = 1.0 - fun.A
    U = U - c * jsq / (2.0 * rho_s ** 2)
    avec = [c * jc / rho_s for jc in j]
    return U, delta, fun.A, avec


def energy_density(rho, tau, jsq, nu, lam, fun):
    """SLDA-type energy density (Eqs. sldae-functional-generic, -CM, and the
    intrinsic part) for the spin-symmetric case, with the regularised
    coupling in the pairing term:

        sum_sigma A/2 (tau - j^2/rho) + 3/5 B rho_+ eF(rho_+) + g_eff |nu|^2
        + sum_sigma j^2 / (2 rho)

    rho, tau are per spin; jsq = |j_sigma|^2 per spin."""
    g = 1.0 / inv_geff(rho, lam, fun)
    rho_s = np.maximum(rho, RHO_FLOOR / 2)
    kin = 2.0 * 0.5 * fun.A * (tau - jsq / rho_s)
    pot = 0.6 * fun.B * (2.0 * rho) * eF(2.0 * rho)
    pair = g * np.abs(nu) ** 2
    cm = 2.0 * jsq / (2.0 * rho_s)
    return kin + pot + pair + cm


def energy_terms(rho, tau, j, nu, lam, vext, fun, dV, dext=None):
    """Energy contributions of Sec. 3.2 (spin-symmetric, j = (jx, jy, jz)
    per spin): E_kin, E_pot, E_pair, E_curr, E_pot.ext, the external
    pairing energy E_pair.ext = -int (Delta_ext nu^* + c.c.) (zero without
    dext) and their sum.  E_pair = -int Delta^* nu, which equals
    int g_eff |nu|^2."""
    U, delta, g = potentials(rho, nu, lam, fun)
    jsq = sum(np.abs(c) ** 2 for c in j)
    rho_s = np.maximum(rho, RHO_FLOOR / 2)
    e_kin = dV * np.sum(2.0 * 0.5 * fun.A * (tau - jsq / rho_s))
    e_pot = dV * np.sum(0.6 * fun.B * (2.0 * rho) * eF(2.0 * rho))
    e_pair = -dV * np.sum(np.real(np.conj(delta) * nu))
    e_curr = dV * np.sum(2.0 * jsq / (2.0 * rho_s))
    e_ext = dV * np.sum(vext * 2.0 * rho)
    e_pext = 0.0 if dext is None else -2.0 * dV * np.sum(np.real(dext * np.conj(nu)))
    tot = e_kin + e_pot + e_pair + e_curr + e_ext + e_pext
    return dict(kin=e_kin, pot=e_pot, pair=e_pair, curr=e_curr, potext=e_ext, pairext=e_pext, total=tot)


def fermi_weight(E, T=0.0):
    """f_beta(E) = 1/(exp(E/T)+1); at T = 0 the step theta(-E) with f(0)=1/2."""
    E = np.asarray(E, dtype=float)
    if T == 0.0:
        return np.where(E < 0, 1.0, np.where(E > 0, 0.0, 0.5))
    x = np.clip(E / T, -700, 700)
    return 1.0 / (np.exp(x) + 1.0)
