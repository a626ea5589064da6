"""Seeded random vectors (numpy PCG64 via ``default_rng``)."""
import numpy as np


def real_normal(seed, shape):
    """N(0,1) float64 array drawn from ``default_rng(seed)``."""
    return np.random.default_rng(seed).standard_normal(shape)


def complex_normal(seed, shape):
    """Complex128 array whose real parts are drawn first, then the imaginary
    parts, both N(0,1), from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im
