"""Pins of the functional (Sec. 2.4, 2.6) against the paper's printed
values, closed forms and definitions."""
import numpy as np
import pytest

from oracle import functional as F
from oracle import uniform as UN
import synth


def test_aslda_constants_at_p0():
    """A(0) = 1.094, and B(0) from its defining formula; the A=1 reading."""
    assert F.aslda_A(0.0) == pytest.approx(1.094)
    assert F.aslda_B(0.0) == pytest.approx(2 ** (2 / 3) * 0.357 - 1.094, abs=1e-12)
    assert F.aslda_B(0.0, force_a1=True) == pytest.approx(-0.4332978244, abs=1e-9)
    # A_b(p) = A_a(-p): B is even in p
    assert F.aslda_B(0.3) == pytest.approx(F.aslda_B(-0.3), abs=1e-14)


@pytest.mark.parametrize("force_a1", [False, True])
def test_uniform_slda_reproduces_printed_values(force_a1):
    """P5: the continuum uniform solution of the regularised functional gives
    E/E_FG = 0.39(1) and Delta/eF = 0.51(1) (ASLDA at p=0).  With A forced to
    1 and B recomputed the equation of state is kept (E/E_FG) while the gap
    moves to about 0.48."""
    fun = F.Functional(F.SLDA, force_a1=force_a1)
    r = UN.continuum_slda(fun, ec_over_ef=100.0)
    assert r["residual"] < 1e-10
    assert abs(r["E_over_EFG"] - 0.39) < 0.015
    if not force_a1:
        assert abs(r["delta_over_eF"] - 0.51) < 0.015
    else:
        assert 0.45 < r["delta_over_eF"] < 0.51


def test_uniform_slda_converges_in_cutoff():
    fun = F.Functional(F.SLDA, force_a1=False)
    a = UN.continuum_slda(fun, ec_over_ef=50.0)
    b = UN.continuum_slda(fun, ec_over_ef=400.0)
    assert abs(a["E_over_EFG"] - b["E_over_EFG"]) < 2e-3
    assert abs(a["delta_over_eF"] - b["delta_over_eF"]) < 1e-2


def test_lambda_c_limits():
    """Lambda_c -> k_c/(2 pi^2 A) for k_c >> k_0, is continuous through
    k_0 = 0, and the analytic continuation matches a numerically continued
    bracket for small imaginary k_0."""
    mu, ec = 1.0, 1e6
    lam = F.lambda_c(0.0, mu, ec)
    kc = np.sqrt(2 * (ec + mu))
    assert lam == pytest.approx(kc / (2 * np.pi ** 2), rel=1e-3)
    eps = 1e-9
    a = F.lambda_c(mu - eps, mu, 10.0)
    b = F.lambda_c(mu + eps, mu, 10.0)
    assert a == pytest.approx(b, rel=1e-7)
    # complex evaluation of the bracket at k0 = i kappa
    vplus, ecs = 1.3, 7.0
    kc = np.sqrt(2 * (ecs + mu - vplus))
    k0 = 1j * np.sqrt(2 * (vplus - mu))
    br = 1 - k0 / (2 * kc) * np.log((kc + k0) / (kc - k0))
    assert abs(br.imag) < 1e-14
    assert F.lambda_c(vplus, mu, ecs) == pytest.approx(kc / (2 * np.pi ** 2) * br.real, rel=1e-13)


@pytest.mark.parametrize("kind", [F.SLDA, F.BDG])
def test_potentials_are_functional_derivatives(kind):
    """P6: U = dE/drho_sigma and Delta = -dE/dnu^* of the energy density by
    central differences (Sec. 2.3 definitions of the potentials)."""
    fun = F.Functional(kind, force_a1=True, a_s=-0.7) if kind == F.BDG else F.Functional(kind)
    n = 12
    rho = 0.02 + 0.05 * synth.uniform_field(11, n, 0, 1)
    tau = 0.3 * synth.uniform_field(12, n, 0, 1)
    nu = 0.01 * synth.complex_normal(13, n)
    lam = 0.1 + 0.05 * synth.uniform_field(14, n, 0, 1)
    U, delta, _ = F.potentials(rho, nu, lam, fun)
    e = lambda r, x: F.energy_density(r, tau, np.zeros(n), x, lam, fun)
    h = 1e-6 * rho
    # E depends on rho_a + rho_b; d/drho of the symmetric form is 2 dE/drho_a
    dU = (e(rho + h, nu) - e(rho - h, nu)) / (2 * h) / 2
    assert np.allclose(dU, U, rtol=1e-7, atol=1e-10)
    hn = 1e-7
    dr = (e(rho, nu + hn) - e(rho, nu - hn)) / (2 * hn)
    di = (e(rho, nu + 1j * hn) - e(rho, nu - 1j * hn)) / (2 * hn)
    assert np.allclose(-0.5 * (dr + 1j * di), delta, rtol=1e-6, atol=1e-12)


def test_fermi_weights():
    assert np.array_equal(F.fermi_weight([-1.0, 0.0, 2.0]), [1.0, 0.5, 0.0])
    T = 0.3
    E = np.linspace(-2, 2, 9)
    assert np.allclose(F.fermi_weight(E, T) + F.fermi_weight(-E, T), 1.0)
