"""FP64 reduced quantities of a lattice state.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper defines none of these; they are the plain definitions on the
periodic grid with cell volume dV = dx^d and u = q / rho:

    mass       dV sum rho
    momentum   dV sum q_j
    kinetic    1/2 dV sum |q|^2 / rho
    enstrophy  1/2 dV sum |curl_h u|^2
    div_l2     sqrt(dV sum (div_h u)^2)
    max_u      max |u|
    rho_min / rho_max
    nonfinite  number of cells holding a non-finite population

with the centred differences (D_j g)(x) = (g(x + dx e_j) - g(x - dx e_j)) / (2 dx).
"""

from __future__ import annotations

import math

import numpy as np

from . import scheme


def centred(g: np.ndarray, axis_j: int, dx: float) -> np.ndarray:
    """Periodic centred difference along direction j (j = 0 is x, the last axis)."""
    ax = g.ndim - 1 - axis_j
    return (np.roll(g, -1, axis=ax) - np.roll(g, 1, axis=ax)) / (2.0 * dx)


def vorticity(u: np.ndarray, dx: float) -> np.ndarray:
    """curl_h u: a scalar field in 2D, a (3, ...) field in 3D."""
    dim = u.shape[0]
    if dim == 2:
        return centred(u[1], 0, dx) - centred(u[0], 1, dx)
    wx = centred(u[2], 1, dx) - centred(u[1], 2, dx)
    wy = centred(u[0], 2, dx) - centred(u[2], 0, dx)
    wz = centred(u[1], 0, dx) - centred(u[0], 1, dx)
    return np.stack([wx, wy, wz])


def divergence(u: np.ndarray, dx: float) -> np.ndarray:
    return sum(centred(u[j], j, dx) for j in range(u.shape[0]))


def from_moments(rho: np.ndarray, q: np.ndarray, dx: float) -> dict:
    dim = q.shape[0]
    dV = dx ** dim
    u = q / rho[None]
    w = vorticity(u, dx)
    div = divergence(u, dx)
    return {
        "mass": dV * math.fsum(rho.ravel()),
        "mom": [dV * math.fsum(q[j].ravel()) for j in range(dim)],
        "kinetic": 0.5 * dV * math.fsum((np.sum(q * q, axis=0) / rho).ravel()),
        "enstrophy": 0.5 * dV * math.fsum((w * w).ravel()),
        "div_l2": math.sqrt(dV * math.fsum((div * div).ravel())),
        "max_u": float(np.sqrt(np.max(np.sum(u * u, axis=0)))),
        "rho_min": float(rho.min()),
        "rho_max": float(rho.max()),
    }


def of_state(f: np.ndarray, p: "scheme.Params") -> dict:
    rho, q = scheme.moments(f, p)
    d = from_moments(rho, q, p.dx)
    bad = ~np.isfinite(f)
    d["nonfinite"] = int(np.count_nonzero(bad.any(axis=(0, 1))))
    return d
