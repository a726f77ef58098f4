"""Pins of the oracle's lattice machinery against the paper's closed forms
(Sec. 3.1: k-grid, Eq. derivative-spectral, Eqs. D1 and D2)."""
import numpy as np
import pytest

from oracle import lattice as L
import synth


@pytest.mark.parametrize("n,d", [(4, 1.0), (6, 0.7), (8, 1.0), (12, 1.3), (32, 1.0), (48, 0.5)])
def test_fft_derivative_equals_dense_D1_D2(n, d):
    """P1: the FFT derivative with the Nyquist mode zeroed is D^(1) of
    Eq. D1; with the full -k^2 it is D^(2) of Eq. D2."""
    k = L.kgrid(n, d)
    f = synth.complex_normal(n, (n,))
    d1 = L.d1_matrix(n, d) @ f
    d2 = L.d2_matrix(n, d) @ f
    scale = np.abs(f).max() / d ** 2 * n
    assert np.abs(d1 - L.spectral_derivative(f, k, 0, 1)).max() < 1e-13 * scale
    assert np.abs(d2 - L.spectral_derivative(f, k, 0, 2)).max() < 1e-13 * scale


def test_kgrid_layout():
    k = L.kgrid(8, 0.5)
    L8 = 8 * 0.5
    assert np.allclose(k[:4], 2 * np.pi / L8 * np.arange(4))
    assert np.allclose(k[4:], 2 * np.pi / L8 * (np.arange(4, 8) - 8))
    assert np.isclose(k[4], -np.pi / 0.5)  # Nyquist carries -pi/dx


def test_derivatives_of_plane_waves_and_trig():
    """Exact on band-limited functions: d/dx sin(2 pi m x / L) and the
    second derivative of a Nyquist wave (-1)^l (which D1 maps to 0)."""
    n, d = 16, 0.25
    x = np.arange(n) * d
    Lx = n * d
    k = L.kgrid(n, d)
    for m in (1, 3, 7):
        q = 2 * np.pi * m / Lx
        f = np.sin(q * x)
        assert np.allclose(L.spectral_derivative(f, k, 0, 1).real, q * np.cos(q * x), atol=1e-12)
        assert np.allclose(L.spectral_derivative(f, k, 0, 2).real, -q * q * f, atol=1e-11)
    ny = (-1.0) ** np.arange(n)
    assert np.abs(L.d1_matrix(n, d) @ ny).max() < 1e-12
    assert np.allclose(L.d2_matrix(n, d) @ ny, -(np.pi / d) ** 2 * ny, atol=1e-10)


def test_D1_squared_differs_from_D2_only_by_nyquist():
    n, d = 8, 1.0
    D1, D2 = L.d1_matrix(n, d), L.d2_matrix(n, d)
    ny = (-1.0) ** np.arange(n) / np.sqrt(n)
    diff = D2 - D1 @ D1
    # the difference is -(pi/d)^2 times the projector on the Nyquist mode
    assert np.allclose(diff, -(np.pi / d) ** 2 * np.outer(ny, ny), atol=1e-12)


def test_dense_laplacian_matches_spectral():
    lat = L.Lattice(4, 6, 8, 1.0, 0.8, 1.2)
    f = synth.complex_normal(5, lat.shape)
    a = (L.dense_laplacian(lat) @ f.ravel()).reshape(lat.shape)
    b = L.laplacian(f[None], lat)[0]
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
