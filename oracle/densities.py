"""Densities of the reduced BdG problem (paper Sec. 2.2-2.3).

A set of n quasiparticle states is an array phi of shape (n, 2, *grid):
phi[:, 0] = u_{n,a}, phi[:, 1] = v_{n,b}.  Integrals use dV, so states are
normalised as int (|u|^2 + |v|^2) dV = 1.

Derivative conventions (reading of the paper's Nyquist rule for the
kinetic density): j is built from the paper's odd-derivative rule with the
Nyquist mode zeroed.  tau gives the Nyquist mode its full weight k_N^2 =
(pi/dx)^2, so int tau dV = sum_k k^2 |phi_k|^2 matches the D^(2) kinetic
operator in H exactly (energy conservation); the Nyquist momentum is taken
symmetrically, i.e. |d f|^2 is averaged over k_N = -pi/dx and +pi/dx, which
gives per axis

    |d_x f|^2  ->  |D1_x f|^2 + (pi/dx)^2 |c_x|^2,
    c_x(y, z) = (1/N_x) sum_l (-1)^l f(l, y, z)   (the Nyquist amplitude),

and keeps tau invariant under f -> f^*, so the general and the
spin-symmetric forms of the densities agree point by point.

Part of the oracle: test infrastructure only (tests, the smoke check and
the benchmark's CPU baseline use it; the product path never does).
"""
import numpy as np
from . import lattice as L

CHUNK = 256


def norms(phi, dV):
    """int (|u|^2 + |v|^2) dV for every state."""
    ax = tuple(range(1, phi.ndim))
    return dV * np.sum(np.abs(phi) ** 2, axis=ax)


def normalize(phi, dV):
    return phi / np.sqrt(norms(phi, dV)).reshape((-1,) + (1,) * (phi.ndim - 1))


def grad_sq(f, lat):
    """Kinetic-density integrand sum_d |d_d f|^2 of fields f (..., nx, ny, nz)
    in the symmetric-Nyquist convention stated in the module docstring."""
    out = np.zeros(f.shape)
    gz = L.gradient(f, lat, zero_nyquist=True)
    for a in range(3):
        axis = f.ndim - 3 + a
        n = f.shape[axis]
        sgn = ((-1.0) ** np.arange(n)).reshape([n if i == axis else 1 for i in range(f.ndim)])
        c = np.sum(sgn * f, axis=axis, keepdims=True) / n
        out += np.abs(gz[a]) ** 2 + (np.pi / lat.d[a]) ** 2 * np.abs(c) ** 2
    return out


def local_densities(phi, wu, wv):
    """rho and nu of the spin-symmetric form (Eqs. nab3D and the anomalous
    density): rho = sum |v|^2 f(-E) + |u|^2 f(E), nu = sum u v^* (f(-E)-f(E)).
    wu = f(E_n), wv = f(-E_n)."""
    shp = (-1,) + (1,) * (phi.ndim - 2)
    wu = np.asarray(wu, float).reshape(shp)
    wv = np.asarray(wv, float).reshape(shp)
    u, v = phi[:, 0], phi[:, 1]
    rho = np.sum(wv * np.abs(v) ** 2 + wu * np.abs(u) ** 2, axis=0)
    nu = np.sum((wv - wu) * u * np.conj(v), axis=0)
    return rho, nu


def spin_symmetric(phi, wu, wv, lat):
    """All four densities of the spin-symmetric case (Eqs. nab3D-jab3D),
    summed over the supplied (E_n > 0) states.  Returns rho, tau, nu, j[3],
    all per spin component."""
    rho = np.zeros(lat.shape)
    tau = np.zeros(lat.shape)
    nu = np.zeros(lat.shape, complex)
    j = [np.zeros(lat.shape) for _ in range(3)]
    wu = np.asarray(wu, float)
    wv = np.asarray(wv, float)
    for s in range(0, phi.shape[0], CHUNK):
        p = phi[s:s + CHUNK]
        a, b = wu[s:s + CHUNK], wv[s:s + CHUNK]
        r, n = local_densities(p, a, b)
        rho += r
        nu += n
        shp = (-1, 1, 1, 1)
        A, B = a.reshape(shp), b.reshape(shp)
        u, v = p[:, 0], p[:, 1]
        tau += np.sum(B * grad_sq(v, lat) + A * grad_sq(u, lat), axis=0)
        gz_u = L.gradient(u, lat, zero_nyquist=True)
        gz_v = L.gradient(v, lat, zero_nyquist=True)
        for c in range(3):
            j[c] += np.sum(B * np.imag(v * np.conj(gz_v[c])) - A * np.imag(u * np.conj(gz_u[c])), axis=0)
    return rho, tau, nu, j


def general(phi, fE, fmE, lat):
    """Densities of the reduced problem with both spin branches explicit
    (Eqs. na3D-jb3D), summed over every supplied state (both signs of E).
    fE = f(E_n), fmE = f(-E_n).  Returns dict of rho_a, rho_b, tau_a, tau_b,
    nu, j_a[3], j_b[3]."""
    shp = (-1, 1, 1, 1)
    fE = np.asarray(fE, float).reshape(shp)
    fmE = np.asarray(fmE, float).reshape(shp)
    u, v = phi[:, 0], phi[:, 1]
    gz_u = L.gradient(u, lat, zero_nyquist=True)
    gz_v = L.gradient(v, lat, zero_nyquist=True)
    out = dict(
        rho_a=np.sum(np.abs(u) ** 2 * fE, axis=0),
        rho_b=np.sum(np.abs(v) ** 2 * fmE, axis=0),
        tau_a=np.sum(grad_sq(u, lat) * fE, axis=0),
        tau_b=np.sum(grad_sq(v, lat) * fmE, axis=0),
        nu=0.5 * np.sum(u * np.conj(v) * (fmE - fE), axis=0),
        j_a=[-np.sum(np.imag(u * np.conj(g)) * fE, axis=0) for g in gz_u],
        j_b=[np.sum(np.imag(v * np.conj(g)) * fmE, axis=0) for g in gz_v],
    )
    return out
