"""Static self-consistent solve of the quasi-2D problem (test infrastructure:
only tests/, the smoke check and the benchmark's CPU leg use the oracle).

Geometry (Sec. 3.1, quasi-2D item): an N_x x N_y periodic lattice in the x-y
plane and plane waves exp(i k_z z) / sqrt(L_z) along z, with the N_z lattice
momenta k_z = 2 pi m / (N_z dz), m in [-N_z/2, N_z/2).  Equal |k_z| give the
same BdG problem, so the N_z/2 + 1 distinct |k_z| are diagonalised once and
weighted by their multiplicity (1 for m = 0 and m = -N_z/2, 2 otherwise).

The map K of Alg. MapK (H -> eigenpairs -> densities -> potentials), the
linear and modified Broyden mixing of the potentials, the fixed-N
chemical-potential update of
Eq. update-mu and the convergence test (the largest change of the
potentials relative to eF_ref, and of N relative to N_req) are written out
plainly: dense matrices, numpy.linalg.eigh, FP64.
"""
import numpy as np

from . import functional as F
from . import lattice as L


class GeometryQ2D:
    def __init__(self, nx, ny, nz, dx=1.0, dy=1.0, dz=1.0):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy, self.dz = float(dx), float(dy), float(dz)
        self.M = self.nx * self.ny
        self.shape = (self.nx, self.ny)
        self.Lz = self.nz * self.dz
        self.dA = self.dx * self.dy
        # -1/2 (D2_x (x) 1 + 1 (x) D2_y) on the flat index ix*N_y + iy (Eq. D2)
        d2x = L.d2_matrix(self.nx, self.dx)
        d2y = L.d2_matrix(self.ny, self.dy)
        self.K = -0.5 * (np.kron(d2x, np.eye(self.ny)) + np.kron(np.eye(self.nx), d2y))
        m = np.arange(0, self.nz // 2 + 1)
        self.kz = 2.0 * np.pi * m / (self.nz * self.dz)
        self.mult = np.where((m == 0) | (m == self.nz // 2), 1.0, 2.0)
        self.Lperp = self.Lz  # length of the plane-wave directions (densities carry 1/Lperp)

    def coords(self):
        x = (np.arange(self.nx) - self.nx // 2) * self.dx
        y = (np.arange(self.ny) - self.ny // 2) * self.dy
        return np.meshgrid(x, y, indexing="ij")


class GeometryQ1DStatic:
    """Quasi-1D static geometry (Sec. 3.1, quasi-1D item): an N_x-site
    periodic lattice along x and plane waves exp(i (k_y y + k_z z)) /
    sqrt(L_y L_z) in y and z, N_y and N_z lattice momenta (spacings dy, dz).
    Problems depend on k_perp^2 = k_y^2 + k_z^2 only; the distinct (|k_y|,
    |k_z|) pairs are diagonalised once with multiplicity w_y w_z (1 for the
    zero and Nyquist momenta, 2 otherwise), and the densities carry
    1 / (L_y L_z).  The first stage of releasing symmetry constraints
    (Sec. 5.2): a problem with translational symmetry in y and z."""

    def __init__(self, nx, ny, nz, dx=1.0, dy=1.0, dz=1.0):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy, self.dz = float(dx), float(dy), float(dz)
        self.M = self.nx
        self.shape = (self.nx,)
        self.dA = self.dx
        self.Lperp = self.ny * self.dy * self.nz * self.dz
        self.K = -0.5 * L.d2_matrix(self.nx, self.dx)
        my = np.arange(0, self.ny // 2 + 1)
        mz = np.arange(0, self.nz // 2 + 1)
        wy = np.where((my == 0) | (my == self.ny // 2), 1.0, 2.0)
        wz = np.where((mz == 0) | (mz == self.nz // 2), 1.0, 2.0)
        ky = 2.0 * np.pi * my / (self.ny * self.dy)
        kz = 2.0 * np.pi * mz / (self.nz * self.dz)
        # build_h adds k^2/2 of the class momentum: k = |k_perp|
        self.kz = np.sqrt(ky[:, None] ** 2 + kz[None, :] ** 2).ravel()
        self.mult = (wy[:, None] * wz[None, :]).ravel()

    def coords(self):
        return ((np.arange(self.nx) - self.nx // 2) * self.dx,)


def build_h(geom, hfield, delta, kz):
    """2M x 2M BdG matrix of one k_z (Eq. HpsiEpsi, spin-symmetric reduced
    form): h = K + diag(hfield) + k_z^2 / 2 with hfield = V_ext + U - mu."""
    h = geom.K + np.diag(np.ravel(hfield) + 0.5 * kz * kz)
    d = np.diag(np.ravel(delta))
    return np.block([[h, d], [np.conj(d), -h]])


def densities(geom, hfield, delta):
    """rho (per spin) and nu of the T = 0 state: every E > 0 eigenpair of
    every plane-wave class, v occupied (f(-E) = 1, f(E) = 0), states
    normalised on the lattice (eigenvectors / sqrt(dx dy), quasi-1D
    / sqrt(dx)), and the 1 / L_z (quasi-1D 1 / (L_y L_z)) of the plane
    waves."""
    rho = np.zeros(geom.M)
    nu = np.zeros(geom.M, dtype=complex)
    for kz, w in zip(geom.kz, geom.mult):
        E, W = np.linalg.eigh(build_h(geom, hfield, delta, kz))
        sel = E > 0
        u = W[:geom.M, sel] / np.sqrt(geom.dA)
        v = W[geom.M:, sel] / np.sqrt(geom.dA)
        rho += w * np.sum(np.abs(v) ** 2, axis=1)
        nu += w * np.sum(u * np.conj(v), axis=1)
    return (rho / geom.Lperp).reshape(geom.shape), (nu / geom.Lperp).reshape(geom.shape)


def map_k(geom, fun, vext, U, delta, mu, ec):
    """One application of Alg. MapK.  The regulator uses V_+ = V_ext + U_in
    (the static iteration order).  Returns (U_out, Delta_out, rho, nu, N)
    with N = int rho_+ d^3r = L_z sum 2 rho dx dy (quasi-1D:
    L_y L_z sum 2 rho dx)."""
    lam = F.lambda_c(vext + U, mu, ec)
    rho, nu = densities(geom, vext + U - mu, delta)
    Uo, Do, _ = F.potentials(rho, nu, lam, fun)
    N = geom.Lperp * geom.dA * np.sum(2.0 * rho)
    return Uo, Do, rho, nu, N


class Broyden:
    """Modified Broyden mixing of a real vector p (the Broyden option of
    Sec. 3.2, which follows the variant for strongly interacting systems of
    Baran et al., Phys. Rev. C 78, 014318 (2008), built on Johnson's
    modified method).  With F_i = K[p_i] - p_i and the last m normalised
    differences dF_k = (F_{k+1} - F_k) / |F_{k+1} - F_k|,
    dp_k = (p_{k+1} - p_k) / |F_{k+1} - F_k|:
        a_kl  = w0^2 delta_kl + dF_k . dF_l      (weights w_k = 1)
        gamma = a^{-1} c,  c_k = dF_k . F_i
        p_{i+1} = p_i + m_p F_i - sum_l gamma_l (m_p dF_l + dp_l).
    m = 0 is linear mixing.  With w0 -> 0 and m >= the dimension this is
    Anderson mixing, which on a linear map reaches the fixed point in at most
    dim + 1 steps (its iterates are GMRES's)."""

    def __init__(self, m, mix, w0=0.01):
        self.m, self.mix, self.w0 = int(m), float(mix), float(w0)
        self.dF, self.dp = [], []
        self.prev = None

    def step(self, p, Kp):
        p = np.asarray(p, float)
        F = np.asarray(Kp, float) - p
        if self.m > 0 and self.prev is not None:
            p0, F0 = self.prev
            dF = F - F0
            n = np.linalg.norm(dF)
            inv = 1.0 / n if n > 0 else 0.0  # an unchanged residual: a zero row (gamma 0)
            self.dF.append(dF * inv)
            self.dp.append((p - p0) * inv)
            if len(self.dF) > self.m:
                self.dF.pop(0)
                self.dp.pop(0)
        self.prev = (p, F)
        out = p + self.mix * F
        if self.m > 0 and self.dF:
            DF = np.array(self.dF)
            a = self.w0 ** 2 * np.eye(len(self.dF)) + DF @ DF.T
            gamma = np.linalg.solve(a, DF @ F)
            for g, dF, dp in zip(gamma, self.dF, self.dp):
                out = out - g * (self.mix * dF + dp)
        return out


def solve(geom, fun, vext, U, delta, mu, ec, mix=0.5, a_mu=0.5, N_req=None, tol=1e-8, eF_ref=0.5,
          maxit=500, history=None, broyden=0, w0=0.01):
    """Iterate p = (U, Delta) to the fixed point of K: linear mixing
    p_{n+1} = m K[p_n] + (1 - m) p_n (broyden = 0) or the modified Broyden
    mixing above with the last `broyden` differences.  In fixed-N mode
    (N_req given) Eq. update-mu is a step of K: with linear mixing mu takes
    its output unmixed; with Broyden mixing mu is a component of p.  Converged when
    max(|U_out - U_in|_inf, |Delta_out - Delta_in|_inf) / eF_ref < tol and
    (fixed N) |N - N_req| / N_req < tol.  Returns (U, Delta, mu, iterations,
    converged)."""
    U = np.array(U, float)
    delta = np.array(delta, complex)
    mixer = Broyden(broyden, mix, w0)
    n = U.size
    for it in range(1, maxit + 1):
        Uo, Do, rho, nu, N = map_k(geom, fun, vext, U, delta, mu, ec)
        r = max(np.abs(Uo - U).max(), np.abs(Do - delta).max()) / eF_ref
        rn = 0.0 if N_req is None else abs(N - N_req) / N_req
        if history is not None:
            history.append((r, rn, mu, N))
        if r < tol and rn < tol:
            return Uo, Do, mu, it, True
        mu_out = mu if N_req is None else mu + a_mu / N_req * (N_req - N)
        if broyden:
            # mu is part of p here: Eq. update-mu is the last step of K
            p = np.concatenate([U.ravel(), delta.real.ravel(), delta.imag.ravel(), [mu]])
            Kp = np.concatenate([np.ravel(Uo), np.real(Do).ravel(), np.imag(Do).ravel(), [mu_out]])
            q = mixer.step(p, Kp)
            U = q[:n].reshape(U.shape)
            delta = (q[n:2 * n] + 1j * q[2 * n:3 * n]).reshape(U.shape)
            mu = q[3 * n]
        else:
            U = mix * Uo + (1.0 - mix) * U
            delta = mix * Do + (1.0 - mix) * delta
            mu = mu_out
    return U, delta, mu, maxit, False
