"""Pins of the oracle's Adam step: the first step moves each parameter by
lr g / (|g| + eps) (bias correction cancels the moment weights), and a
constant gradient gives the geometric-series moments."""

import numpy as np

from oracle import ref64


def test_first_step_and_constant_gradient_moments():
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = ref64.adam_step(p0, g, np.zeros(50), np.zeros(50), 1e-2, 0.9, 0.999, 1e-8, 1)
    assert np.allclose(p1, p0 - 1e-2 * g / (np.abs(g) + 1e-8), atol=1e-14)
    p, m, v = p0, np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        p, m, v = ref64.adam_step(p, g, m, v, 1e-3, 0.9, 0.999, 1e-8, t)
    assert np.allclose(m, (1 - 0.9 ** 7) * g, atol=1e-14)
    assert np.allclose(v, (1 - 0.999 ** 7) * g * g, atol=1e-14)
    # with the moments bias-corrected, every step moves by lr g / (|g| + eps)
    assert np.allclose(p, p0 - 7e-3 * g / (np.abs(g) + 1e-8), atol=1e-12)
