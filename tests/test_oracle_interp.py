"""Pins of the lattice interpolation (Sec. 5.2, refining lattice
resolution): at the stored lattice points the interpolant returns the stored
values (the paper's own statement), and a trigonometric polynomial below the
Nyquist mode of the source lattice is reproduced exactly everywhere."""
import numpy as np
import pytest

from oracle import interp as I
import synth



def test_identity_on_the_same_lattice_and_at_shared_points():
    f = synth.uniform_field(3, (6, 8), -1.0, 1.0)
    assert np.abs(I.to_lattice(f, 1.5, 1.0, 6, 8, 1.5, 1.0) - f).max() < 1e-13
    # a lattice twice as fine contains every source point at even indices
    g = I.to_lattice(f, 1.5, 1.0, 12, 16, 0.75, 0.5)
    assert np.abs(g[::2, ::2] - f).max() < 1e-13


@pytest.mark.parametrize("dst", [(16, 16, 0.75, 0.75), (9 * 2, 10, 12.0 / 18, 1.2)])
def test_band_limited_function_is_reproduced(dst):
    """12 x 12 source with spacing 1 (box 12): f = sum of modes with |l|, |m|
    below 6 (random real amplitudes and phases) is interpolated onto other
    lattices of the same box without error."""
    g = np.random.default_rng(4)
    modes = [(int(a), int(b)) for a, b in g.integers(-5, 6, size=(7, 2))]
    amp, ph = g.uniform(0.2, 1.0, 7), g.uniform(0, 2 * np.pi, 7)
    Lb = 12.0

    def f(x, y):
        out = np.full(np.shape(x), 0.3)
        for (l, m), a, p in zip(modes, amp, ph):
            out = out + a * np.cos(2 * np.pi * (l * x + m * y) / Lb + p)
        return out

    X, Y = np.meshgrid(np.arange(12) * 1.0, np.arange(12) * 1.0, indexing="ij")
    nx2, ny2, dx2, dy2 = dst
    X2, Y2 = np.meshgrid(np.arange(nx2) * dx2, np.arange(ny2) * dy2, indexing="ij")
    got = I.to_lattice(f(X, Y), 1.0, 1.0, nx2, ny2, dx2, dy2)
    assert np.abs(got - f(X2, Y2)).max() < 1e-12
