"""Pins of the external pairing potential Delta_ext in the oracle (Sec. 2.2,
Eq. E_tot; Sec. 2.3, Eq. HpsiEpsi; Sec. 3.2, external pairing energy).

  - the BdG off-diagonal is Delta + Delta_ext: the uniform spectrum becomes
    +-sqrt(xi^2 + |Delta + Delta_ext|^2) (textbook uniform BCS with the
    total pairing field);
  - the off-diagonal field the evolution uses equals -dE/dnu^* of the
    total energy including E_pair.ext (central differences);
  - with a complete set of states the quantity minimised in Eq. E_tot,
    Omega = E_total - mu N (E_total including E_pair.ext), is conserved
    under the evolution at fixed mu; a pairing source does not conserve N,
    so E_total alone is not, and neither is Omega without E_pair.ext or
    with the sign of Delta_ext flipped in H only (a planted mistake).
"""
import numpy as np
import pytest

from oracle import lattice as L, bdg, densities as D, functional as F, td
import synth


def test_uniform_dispersion_with_dext():
    lat = L.Lattice(4, 4, 6, 1.0, 1.2, 0.9)
    mu, U0, d0 = 0.8, -0.1, 0.3
    dext = 0.1 + 0.2j
    nst = 2
    sys_ = td.TDSystem(td.Geometry3D(lat), None, mu, np.zeros(lat.shape), np.zeros(lat.shape),
                       np.zeros(nst), np.ones(nst), frozen=(np.full(lat.shape, U0 - mu), np.full(lat.shape, d0 + 0j)),
                       dext=np.full(lat.shape, dext))
    hf, de = sys_.fields(None)[:2]
    E = np.linalg.eigvalsh(bdg.dense_h(hf, de, lat))
    xi = 0.5 * lat.k2.ravel() + U0 - mu
    ek = np.sqrt(xi ** 2 + abs(d0 + dext) ** 2)
    ref = np.sort(np.concatenate([ek, -ek]))
    assert np.abs(E - ref).max() < 1e-12
    # and not the dispersion without Delta_ext
    ek0 = np.sqrt(xi ** 2 + d0 ** 2)
    assert np.abs(E - np.sort(np.concatenate([ek0, -ek0]))).max() > 1e-2


def _system(n=6, seed=40, dext_amp=0.08):
    lat = L.Lattice(n, n, n)
    fun = F.Functional(F.SLDA)
    mu = 1.0
    eta = synth.uniform_field(seed, lat.shape)
    E, phi = bdg.eigenstates(np.full(lat.shape, -mu), 0.5 * np.exp(1j * 0.05 * eta), lat)
    pos = E > 0
    lam = F.lambda_c(np.zeros(lat.shape), mu, 0.5 * np.pi ** 2)
    dext = dext_amp * synth.complex_normal(seed + 1, lat.shape)
    return lat, fun, mu, lam, E[pos], phi[pos], dext


def test_offdiagonal_field_is_energy_derivative():
    """-dE_total/dnu^* (central differences in nu at fixed rho, tau, j) is
    the off-diagonal field Delta + Delta_ext that the evolution applies."""
    lat, fun, mu, lam, E, phi, dext = _system(4, 41)
    sys_ = td.TDSystem(td.Geometry3D(lat), fun, mu, np.zeros(lat.shape), lam, F.fermi_weight(E),
                       F.fermi_weight(-E), dext=dext)
    rho, tau, nu, j = D.spin_symmetric(D.normalize(phi, lat.dV), sys_.wu, sys_.wv, lat)
    off = sys_.fields(D.normalize(phi, lat.dV))[1]
    tot = lambda x: F.energy_terms(rho, tau, j, x, lam, np.zeros(lat.shape), fun, lat.dV, dext=dext)["total"]
    h = 1e-7
    for site in [(0, 0, 0), (1, 2, 3), (3, 1, 0)]:
        e = np.zeros(lat.shape)
        e[site] = h
        dr = (tot(nu + e) - tot(nu - e)) / (2 * h)
        di = (tot(nu + 1j * e) - tot(nu - 1j * e)) / (2 * h)
        deriv = -0.5 * (dr + 1j * di) / lat.dV
        assert abs(deriv - off[site]) < 1e-6 * abs(off[site]), (site, deriv, off[site])


class _FlippedDext(td.TDSystem):
    """Planted mistake: H uses Delta - Delta_ext while the energy keeps
    E_pair.ext as defined."""

    def fields(self, phi):
        hf, de, al, av = super().fields(phi)
        return hf, de - 2.0 * self.dext, al, av


def _drift(sys_, phi0, steps=20, dt=0.005):
    phi, hist, _ = td.start(sys_, phi0, dt, "AB4AM5", 1)
    o0 = td.observables(sys_, phi)
    for _ in range(steps):
        phi, hist = td.abm_step(sys_, phi, hist, dt)
    o1 = td.observables(sys_, phi)
    return o0, o1


def test_energy_with_dext_is_conserved():
    lat, fun, mu, lam, E, phi, dext = _system()
    args = (td.Geometry3D(lat), fun, mu, np.zeros(lat.shape), lam, F.fermi_weight(E), F.fermi_weight(-E))
    o0, o1 = _drift(td.TDSystem(*args, dext=dext), phi)
    efg = o0["EFG"]
    omega = lambda o: o["total"] - mu * o["N"]
    # Delta_ext moves energy between the terms and changes N ...
    assert abs(o1["pairext"] - o0["pairext"]) / efg > 1e-4
    assert abs(o1["N"] - o0["N"]) / o0["N"] > 1e-4
    # ... Omega with E_pair.ext is conserved, without it is not
    assert abs(omega(o1) - omega(o0)) / efg < 1e-9
    assert abs(o1["total"] - o0["total"]) / efg > 1e-4
    assert abs((omega(o1) - o1["pairext"]) - (omega(o0) - o0["pairext"])) / efg > 1e-4
    # the planted sign mistake in H breaks conservation
    f0, f1 = _drift(_FlippedDext(*args, dext=dext), phi)
    assert abs(omega(f1) - omega(f0)) / efg > 1e-6
