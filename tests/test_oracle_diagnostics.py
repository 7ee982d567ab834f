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


@pytest.mark.parametrize("n", [16, 64, 100])
def test_divergent_field_closed_forms_2d(n):
    """u = (sin x, 0) with rho = 1 + eps cos y on [0, 2pi)^2 at cell centres
    (n a multiple of 4).  The centred difference of sin is (sin dx / dx) cos,
    so div_h u = s cos x with s = sin(dx)/dx, and the midpoint sum of cos^2
    over a period is n/2:
        div_l2  = sqrt(dx^2 * n * (n/2) * s^2) = s pi sqrt(2)
        max_u   = max_i |sin x_i| = cos(dx/2)     (x_i = (i + 1/2) dx)
        rho_min = 1 - eps cos(dx/2), rho_max = 1 + eps cos(dx/2)
        mass    = (2 pi)^2,  kinetic = 1/2 int rho |u|^2 = pi^2
    (the eps cos y sin^2 x cross term sums to zero).  A dropped square root,
    cell volume or difference factor changes div_l2 by a factor that depends
    on n, so each parametrised size fails on its own."""
    eps = 0.1
    p = scheme.params_for_grid(2, n, 0.01)
    x = (np.arange(n) + 0.5) * p.dx
    u0 = np.zeros((2, n, n))
    u0[0] = np.sin(x)[None, :]
    rho0 = np.broadcast_to(1 + eps * np.cos(x)[:, None], (n, n)).copy()
    f = scheme.init(rho0, u0, p)
    d = diagnostics.of_state(f, p)
    s = math.sin(p.dx) / p.dx
    c = math.cos(p.dx / 2)
    assert d["div_l2"] == pytest.approx(s * math.pi * math.sqrt(2), rel=1e-13)
    assert d["max_u"] == pytest.approx(c, rel=1e-14)
    assert d["rho_min"] == pytest.approx(1 - eps * c, rel=1e-14)
    assert d["rho_max"] == pytest.approx(1 + eps * c, rel=1e-14)
    assert d["mass"] == pytest.approx(4 * math.pi ** 2, rel=1e-14)
    assert d["kinetic"] == pytest.approx(math.pi ** 2, rel=1e-13)
    # u_x depends on x only: no vorticity
    assert d["enstrophy"] < 1e-24


def test_divergent_field_closed_forms_3d():
    """u = (sin x, 0, 2 sin z), rho = 1 on [0, 2pi)^3 (n = 12):
    div_h u = s (cos x + 2 cos z); the cross term sums to zero, so
    dV sum (div_h u)^2 = s^2 dx^3 (n^3/2 + 4 n^3/2) = 5/2 s^2 (2pi)^3;
    max |u|^2 = cos^2(dx/2) (1 + 4)."""
    n = 12
    p = scheme.params_for_grid(3, n, 0.01)
    x = (np.arange(n) + 0.5) * p.dx
    u0 = np.zeros((3, n, n, n))
    u0[0] = np.sin(x)[None, None, :]
    u0[2] = 2 * np.sin(x)[:, None, None]
    f = scheme.init(np.ones((n, n, n)), u0, p)
    d = diagnostics.of_state(f, p)
    s = math.sin(p.dx) / p.dx
    assert d["div_l2"] == pytest.approx(math.sqrt(2.5 * s * s * (2 * math.pi) ** 3), rel=1e-13)
    assert d["max_u"] == pytest.approx(math.sqrt(5) * math.cos(p.dx / 2), rel=1e-14)
    assert d["rho_min"] == pytest.approx(1.0, abs=1e-15) and d["rho_max"] == pytest.approx(1.0, abs=1e-15)
