"""Reduced 2x2 BdG operator of the spin-symmetric problem (paper Sec. 2.3,
Eq. HpsiEpsi) with the A_sigma = 1 single-particle Hamiltonian
(Eq. h_sigma_A1): h = -1/2 nabla^2 + U + V_ext.

    H (u, v) = ( (h - mu) u + Delta v ,  Delta^* u - (h - mu)^* v )

For real U and V_ext, (h - mu)^* = h - mu.  The field hfield = U + V_ext - mu
is passed as one real array.

Part of the oracle: test infrastructure only (tests, the smoke check and
the benchmark's CPU baseline use it; the product path never does).
"""
import numpy as np
from . import lattice as L


def apply_h(phi, hfield, delta, lat):
    """H applied to every state of phi (shape (n, 2, nx, ny, nz)), with the
    spectral Laplacian (Eq. derivative-spectral, full -k^2)."""
    u, v = phi[:, 0], phi[:, 1]
    lap_u = L.laplacian(u, lat)
    lap_v = L.laplacian(v, lat)
    hu = -0.5 * lap_u + hfield * u + delta * v
    hv = np.conj(delta) * u - (-0.5 * lap_v + hfield * v)
    return np.stack([hu, hv], axis=1)


def kinetic_alpha(f, alpha, lat):
    """-1/2 div(alpha grad f) in the symmetrised form of Eq. kinop-alpha,
    summed over the three axes: -1/4 [lap(alpha f) + alpha lap f - f lap alpha],
    every Laplacian spectral with the full -k^2 (Eq. D2)."""
    return -0.25 * (L.laplacian(alpha * f, lat) + alpha * L.laplacian(f, lat) - f * L.laplacian(alpha, lat))


def current_term(f, avec, lat):
    """-(i/2) {A, grad} f = -(i/2) sum_d [A_d d_d f + d_d (A_d f)] (the
    current-potential term of Eq. h_sigma), each first derivative the
    spectral D1 with the Nyquist mode zeroed (Sec. 3.1; matrix forms of
    Eqs. Ad_dx and d_dxA)."""
    out = np.zeros(f.shape, complex)
    for d in range(3):
        axis = f.ndim - 3 + d
        out += avec[d] * L.spectral_derivative(f, lat.k[d], axis, 1)
        out += L.spectral_derivative(avec[d] * f, lat.k[d], axis, 1)
    return -0.5j * out


def apply_h_general(phi, hfield, delta, alpha, avec, lat):
    """H of Eq. HpsiEpsi with the general single-particle Hamiltonian of
    Eq. h_sigma (spin-symmetric: one alpha, one current potential A):

        h = -1/2 div(alpha grad) + hfield - (i/2) {A, grad},
        H (u, v) = ( h u + Delta v,  Delta^* u - h^* v ),
        -h^* v = 1/2 div(alpha grad) v - hfield v - (i/2) {A, grad} v

    (the kinetic and current parts are real operators, hence the same sign
    of the current term in both rows).  alpha: scalar or field; avec: three
    real fields (or None)."""
    alpha = np.broadcast_to(np.asarray(alpha, float), lat.shape)
    u, v = phi[:, 0], phi[:, 1]
    ku, kv = kinetic_alpha(u, alpha, lat), kinetic_alpha(v, alpha, lat)
    hu = ku + hfield * u + delta * v
    hv = np.conj(delta) * u - (kv + hfield * v)
    if avec is not None:
        hu = hu + current_term(u, avec, lat)
        hv = hv + current_term(v, avec, lat)
    return np.stack([hu, hv], axis=1)


def dense_h_general(hfield, delta, alpha, avec, lat):
    """2M x 2M matrix of apply_h_general from the dense matrices of Eqs. D1
    and D2 (Kronecker products per axis): the kinetic part as
    1/2 [D2 diag(alpha) + diag(alpha) D2 - diag(D2 alpha)] per axis (Eq.
    kinop-alpha), the current part as diag(A_d) D1_d + D1_d diag(A_d) (Eqs.
    Ad_dx, d_dxA)."""
    n = lat.n
    eye = [np.eye(m) for m in n]

    def axis_op(Dm, d):
        mats = [eye[0], eye[1], eye[2]]
        mats[d] = Dm
        return np.kron(np.kron(mats[0], mats[1]), mats[2])
    a = np.ravel(np.broadcast_to(np.asarray(alpha, float), lat.shape))
    A = np.diag(a)
    K = np.zeros((lat.M, lat.M))
    for d in range(3):
        D2 = axis_op(L.d2_matrix(n[d], lat.d[d]), d)
        K += -0.25 * (D2 @ A + A @ D2 - np.diag(D2 @ a))
    C = np.zeros((lat.M, lat.M), complex)
    if avec is not None:
        for d in range(3):
            D1 = axis_op(L.d1_matrix(n[d], lat.d[d]), d)
            Ad = np.diag(np.ravel(avec[d]))
            C += -0.5j * (Ad @ D1 + D1 @ Ad)
    h = K + np.diag(np.ravel(hfield))
    dm = np.diag(np.ravel(delta))
    return np.block([[h + C, dm], [np.conj(dm), -h + C]])


def dense_h(hfield, delta, lat):
    """2M x 2M matrix of H in the ordering (u, v), built from the dense
    derivative matrices of Eq. D2 and diagonal matrices for the local
    fields (Sec. 3.2, matrix form of local fields)."""
    K = -0.5 * L.dense_laplacian(lat)
    h = K + np.diag(np.ravel(hfield))
    d = np.diag(np.ravel(delta))
    return np.block([[h, d], [np.conj(d), -h]])


def eigenstates(hfield, delta, lat):
    """Diagonalise the dense H.  Returns (E, phi) with E ascending and phi of
    shape (2M, 2, nx, ny, nz), normalised so int (|u|^2+|v|^2) dV = 1."""
    H = dense_h(hfield, delta, lat)
    E, W = np.linalg.eigh(H)
    M = lat.M
    phi = W.T.reshape((2 * M, 2) + lat.shape) / np.sqrt(lat.dV)
    return E, phi


def plane_wave_states(lat, kidx, hshift, delta0):
    """Eigenstates of the uniform H (constant U, Delta): for lattice momentum
    k, xi = k^2/2 + hshift with hshift = U - mu, E = sqrt(xi^2 + |Delta|^2),
    positive branch u = sqrt((1 + xi/E)/2), v = sqrt((1 - xi/E)/2) Delta^*/|Delta|,
    times exp(i k.r)/sqrt(V) with r measured from the lattice corner.

    kidx: integer array (n, 3) of k-grid indices.  Returns (E, phi)."""
    kidx = np.asarray(kidx)
    kx = lat.k[0][kidx[:, 0]]
    ky = lat.k[1][kidx[:, 1]]
    kz = lat.k[2][kidx[:, 2]]
    xi = 0.5 * (kx ** 2 + ky ** 2 + kz ** 2) + hshift
    ad = abs(delta0)
    E = np.sqrt(xi ** 2 + ad ** 2)
    uk = np.sqrt(0.5 * (1.0 + xi / E))
    vk = np.sqrt(0.5 * (1.0 - xi / E)) * (np.conj(delta0) / ad if ad > 0 else 1.0)
    rx = np.arange(lat.n[0]) * lat.d[0]
    ry = np.arange(lat.n[1]) * lat.d[1]
    rz = np.arange(lat.n[2]) * lat.d[2]
    ph = (np.exp(1j * kx[:, None, None, None] * rx[None, :, None, None])
          * np.exp(1j * ky[:, None, None, None] * ry[None, None, :, None])
          * np.exp(1j * kz[:, None, None, None] * rz[None, None, None, :])) / np.sqrt(lat.V)
    phi = np.stack([uk[:, None, None, None] * ph, vk[:, None, None, None] * ph], axis=1)
    return E, phi


def vortex_phase(lat, vortices):
    """Phase field theta(x, y) = sum_j q_j atan2(y - y_j, x - x_j) of straight
    vortex lines along z, in centred coordinates.  vortices: list of
    (x_j, y_j, q_j)."""
    X, Y, _ = lat.coords()
    th = np.zeros(lat.shape)
    for (x0, y0, q) in vortices:
        th += q * np.arctan2(Y - y0, X - x0)
    return th


def imprint_phase(phi, theta):
    """Vortex imprint (a phase e^{i theta} on Delta): Delta is derived
    from the states in TD, so the phase goes onto the states as the local
    gauge rotation of both fermion fields by theta/2: u_n <- e^{i theta/2} u_n,
    v_n <- e^{-i theta/2} v_n for every state.  This multiplies nu = sum u v^*
    (and hence Delta) by e^{i theta}, leaves rho unchanged, and commutes with
    the partner map (u, v) -> (v^*, -u^*) of the spin-symmetric reduction
    (Sec. 2.3), so the imprinted E > 0 states still stand for a complete set
    closed under that map.  (e^{i theta/2} changes sign across a branch line
    of theta; the imprinted states carry that sign change.)"""
    out = phi.copy()
    out[:, 0] = np.exp(0.5j * theta) * phi[:, 0]
    out[:, 1] = np.exp(-0.5j * theta) * phi[:, 1]
    return out
