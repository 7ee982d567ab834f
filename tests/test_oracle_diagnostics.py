"""Closed forms for the FP64 diagnostics on sampled trigonometric fields."""

import math

import numpy as np
import pytest

import inputs
from oracle import diagnostics, scheme


@pytest.mark.parametrize("n", [16, 64, 75])
def test_taylor_green_closed_forms(n):
    """u = (sin x cos y, -cos x sin y), rho = 1, on [0, 2pi)^2 sampled at cell centres.

    Midpoint sums of cos^2 over n equispaced points are exact (n > 2), so
    kinetic = 1/2 int |u|^2 = pi^2; the centred difference of sin is
    (sin dx / dx) cos, so the discrete vorticity is 2 (sin dx/dx) sin x sin y,
    the enstrophy 2 pi^2 (sin dx/dx)^2 and the discrete divergence vanishes.
    """
    p = scheme.params_for_grid(2, n, 0.01)
    f = scheme.init(np.ones((n, n)), inputs.taylor_green(n), p)
    d = diagnostics.of_state(f, p)
    s = math.sin(p.dx) / p.dx
    assert d["mass"] == pytest.approx(4 * math.pi ** 2, rel=1e-14)
    assert d["kinetic"] == pytest.approx(math.pi ** 2, rel=1e-13)
    assert d["enstrophy"] == pytest.approx(2 * math.pi ** 2 * s * s, rel=1e-13)
    assert d["div_l2"] < 1e-12
    assert abs(d["mom"][0]) < 1e-13 and abs(d["mom"][1]) < 1e-13
    assert d["nonfinite"] == 0


def test_abc_closed_forms():
    """ABC with A = B = C = 1: each velocity component has mean square 1, so
    kinetic = 1/2 * 3 * (2pi)^3; curl u = u and the centred difference scales
    each mode by sin(dx)/dx, so enstrophy = (sin dx/dx)^2 * kinetic."""
    n = 12
    p = scheme.params_for_grid(3, n, 0.01)
    f = scheme.init(np.ones((n, n, n)), inputs.abc_flow(n), p)
    d = diagnostics.of_state(f, p)
    s = math.sin(p.dx) / p.dx
    vol = (2 * math.pi) ** 3
    assert d["kinetic"] == pytest.approx(1.5 * vol, rel=1e-13)
    assert d["enstrophy"] == pytest.approx(s * s * 1.5 * vol, rel=1e-13)
    assert d["div_l2"] < 1e-12


def test_nonfinite_count():
    p = scheme.params_for_grid(2, 8, 0.01)
    f = scheme.init(np.ones((8, 8)), inputs.taylor_green(8), p)
    f[1, 3, 2, 5] = np.nan
    f[0, 0, 7, 7] = np.inf
    f[2, 1, 7, 7] = np.nan
    assert diagnostics.of_state(f, p)["nonfinite"] == 2
