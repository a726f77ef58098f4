"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

Only random draws live here (numpy PCG64 streams); this module holds none of
the method's arithmetic, so the oracle and the HIP path receive the same
random numbers and compute everything else on their own.
"""
import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_field(seed, shape, lo=-1.0, hi=1.0):
    """iid U[lo, hi) values of the given shape."""
    return rng(seed).uniform(lo, hi, size=shape)


def complex_normal(seed, shape, scale=1.0):
    """iid complex normal values (real and imaginary parts N(0, scale^2))."""
    g = rng(seed)
    return scale * (g.standard_normal(shape) + 1j * g.standard_normal(shape))


def vortex_offset(seed, half_width=2.0):
    """Continuous offset (dx, dy) ~ U[-w, w)^2 of a single vortex core."""
    g = rng(seed)
    return tuple(float(x) for x in g.uniform(-half_width, half_width, size=2))


def vortex_pair(seed, radius=8.0, min_sep=4.0):
    """Two core positions, uniform in the disk r < radius, at least min_sep
    apart (rejection sampling)."""
    g = rng(seed)
    pts = []
    while len(pts) < 2:
        x, y = g.uniform(-radius, radius, size=2)
        if x * x + y * y >= radius * radius:
            continue
        if pts and np.hypot(x - pts[0][0], y - pts[0][1]) < min_sep:
            continue
        pts.append((float(x), float(y)))
    return pts


def gaussian_bump(seed):
    """Amplitude V_b = -U(0.1, 0.3), width w_b ~ U(4, 10), centre
    z_b ~ U(-40, 40) of the quasi-1D density bump."""
    g = rng(seed)
    vb = -g.uniform(0.1, 0.3)
    wb = g.uniform(4.0, 10.0)
    zb = g.uniform(-40.0, 40.0)
    return float(vb), float(wb), float(zb)


def obstacles(seed, box):
    """1-4 Gaussian obstacles: amplitudes U(0.5, 3), widths U(2, 8) sites,
    centres uniform in the box [-box/2, box/2)^2."""
    g = rng(seed)
    K = int(g.integers(1, 5))
    amp = g.uniform(0.5, 3.0, size=K)
    wid = g.uniform(2.0, 8.0, size=K)
    cen = g.uniform(-box / 2.0, box / 2.0, size=(K, 2))
    return amp, wid, cen
