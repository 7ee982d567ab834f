"""The oracle in the parameter plane of Fig. 2 (Section 5.1), Taylor-Green
vortex, L2 error on u_x.

The paper does not give the viscosity of these runs, so only its qualitative
statements about Fig. 2 are pinned, at nu = 0.01 with the density well
prepared:
* reducing the diffusion on rho (alpha_rho (1/omega_rho - 1/2), the density
  diffusivity of Section 3) reduces the error;
* the error is nearly constant along an isoline of that diffusivity (the
  three pairs of Section 5.1 lie on one);
* at the corner omega_rho -> 2 with small alpha_rho the runs lose stability.
Fig. 3's statement (an optimum of omega_q near 1.15) does not show at this
viscosity: the error is flat to 1% over omega_q in [1, 1.6], so it stays
unpinned.
"""

import math

import numpy as np
import pytest

import inputs
from oracle import scheme


def _tg_error(n, T, omega_rho, alpha_rho, omega_q=1.0, nu=0.01):
    dx = 2 * math.pi / n
    p = scheme.Params(dim=2, dx=dx, dt=dx * dx / 8, nu=nu, omega_rho=omega_rho, omega_q=omega_q,
                      alpha_rho=alpha_rho)
    u0 = inputs.taylor_green(n)
    rho0 = inputs.well_prepared_density(inputs.taylor_green_pressure(n), dx)
    steps = round(T / p.dt)
    rho, q, _ = scheme.simulate(u0, p, steps, rho0)
    e = q[0] / rho - u0[0] * math.exp(-2 * nu * steps * p.dt)
    return math.sqrt(dx * dx * np.sum(e * e))


def test_less_density_diffusion_smaller_error():
    """48 cells, t = 1, omega_q = 1: along omega_rho = 1 the error grows with
    alpha_rho; the three isoline pairs agree within 1%; a smaller diffusivity
    at another omega_rho gives a smaller error than the isoline."""
    errs = [_tg_error(48, 1.0, 1.0, a) for a in (0.0125, 0.05, 0.1, 0.25)]
    assert all(b > 1.5 * a for a, b in zip(errs, errs[1:])), errs
    iso = [_tg_error(48, 1.0, w, a) for w, a in ((1.0, 1 / 20), (6 / 5, 3 / 40), (3 / 2, 3 / 20))]
    assert max(iso) / min(iso) < 1.01, iso
    assert _tg_error(48, 1.0, 1.6, 0.0125) < 0.5 * min(iso)


def test_unstable_corner():
    """75 cells, t = 1: at omega_rho = 1.95 the run with alpha_rho = 0.01 has
    an error over 10x that with alpha_rho = 0.025, against the trend."""
    e_small = _tg_error(75, 1.0, 1.95, 0.01)
    e_next = _tg_error(75, 1.0, 1.95, 0.025)
    assert e_small > 10 * e_next, (e_small, e_next)
