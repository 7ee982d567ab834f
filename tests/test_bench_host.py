"""Host-side helpers of bench.py's measurement sections (no GPU): the 3D
block restriction and spectral Helmholtz projection used by the storage
precision study, and the equal-error interpolation rule they feed."""

import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _grid(n):
    x = (np.arange(n) + 0.5) * 2 * math.pi / n
    return np.meshgrid(x, x, x, indexing="ij")   # z, y, x


def test_restrict_3d_is_the_block_mean():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3, 12, 12, 12))
    r = bench._restrict_3d(a, 3)
    assert r.shape == (3, 4, 4, 4)
    for c, z, y, x in ((0, 0, 0, 0), (2, 3, 1, 2), (1, 2, 3, 3)):
        assert np.isclose(r[c, z, y, x], a[c, 3 * z:3 * z + 3, 3 * y:3 * y + 3, 3 * x:3 * x + 3].mean())
    assert bench._restrict_3d(a, 1) is a
    # block means keep the mean of every component
    assert np.allclose(r.mean(axis=(1, 2, 3)), a.mean(axis=(1, 2, 3)))


def test_solenoidal_3d_keeps_curls_and_removes_gradients():
    n = 16
    z, y, x = _grid(n)
    curl = np.stack([np.sin(z) + np.cos(2 * y), np.sin(x), np.sin(3 * x)])  # divergence-free
    grad = np.stack([np.cos(x) * np.sin(2 * y), 2 * np.sin(x) * np.cos(2 * y), 0 * x])      # grad(sin x sin 2y)
    assert np.abs(bench._solenoidal_3d(curl) - curl).max() < 1e-12
    assert np.abs(bench._solenoidal_3d(grad)).max() < 1e-12
    mix = curl + grad + 0.25                                     # a constant mean is divergence-free
    assert np.abs(bench._solenoidal_3d(mix) - (curl + 0.25)).max() < 1e-12
    p = bench._solenoidal_3d(mix)
    assert np.abs(bench._solenoidal_3d(p) - p).max() < 1e-12   # a projection


def test_relative_error():
    a = np.ones((3, 2, 2, 2))
    assert bench._rel(a, a) == 0.0
    assert math.isclose(bench._rel(2 * a, a), 1.0)
