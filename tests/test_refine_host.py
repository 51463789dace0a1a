"""Host-side pieces of the refinement study: Fourier truncation and the error measure."""
import math

import numpy as np

from paper_2605_20140_amd import refine as R


def _mode(N, q, phase=0.3):
    x = np.arange(N) * (6.0 / N)
    X1, X2, X3 = np.meshgrid(x, x, x, indexing="ij")
    return np.cos(2 * math.pi * (q[0] * X1 + q[1] * X2 + q[2] * X3) / 6.0 + phase)


def test_truncation_keeps_low_modes_exactly():
    for q in [(0, 0, 0), (1, -2, 3), (7, 7, -7), (-5, 0, 2)]:
        u = 2.0 + _mode(64, q)
        np.testing.assert_allclose(R.downsample(u), 2.0 + _mode(16, q), atol=1e-12)


def test_truncation_drops_high_modes():
    for q in [(8, 0, 0), (0, 9, 1), (20, -3, 0)]:
        np.testing.assert_allclose(R.downsample(_mode(64, q)), 0.0, atol=1e-12)


def test_relative_error():
    a = np.ones((16, 16, 16))
    assert R.rel_error(a, a, 6.0) == 0.0
    assert math.isclose(R.rel_error(a, 2 * a, 6.0), 0.5)
    assert math.isclose(R.norm(a, 6.0), (6.0 / 16) ** 1.5 * 64.0)
