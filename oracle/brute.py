"""Scalar-loop version of the scheme for tiny grids (8x8, 4x4x4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Written independently of `scheme`: plain Python floats, one cell and one
velocity at a time, and transport written in push form (each post-relaxation
value is sent to its destination cell) rather than the pull form used by the
vectorised oracle.  Section 2 of the paper defines both phases; the two forms
are the same map.

State: nested lists f[i][l][cell] with cell = x + nx * (y + ny * z).
"""

from __future__ import annotations


def _velocities(dim):
    """Lattice velocity vectors in the order rest, +x, -x, +y, -y[, +z, -z]."""
    vel = [(0,) * dim]
    for j in range(dim):
        e = [0] * dim
        e[j] = 1
        vel.append(tuple(e))
        e[j] = -1
        vel.append(tuple(e))
    return vel


def _cell_eq(rho, q, dim, dx, mu, alpha_rho, alpha_q, gamma):
    """f^eq of one cell as nested lists [set][velocity] (Section 2)."""
    vel = _velocities(dim)
    out = []
    # density set
    row = []
    for c in vel:
        if all(v == 0 for v in c):
            row.append((1.0 - 2 * dim * alpha_rho) * rho)
        else:
            j = [k for k in range(dim) if c[k] != 0][0]
            row.append(alpha_rho * rho + c[j] * dx / (2.0 * mu) * q[j])
    out.append(row)
    P = rho ** gamma
    for i in range(dim):
        row = []
        for c in vel:
            if all(v == 0 for v in c):
                row.append(dx * (1.0 - 2 * dim * alpha_q) * q[i])
            else:
                j = [k for k in range(dim) if c[k] != 0][0]
                flux = dx * dx / (2.0 * mu) * q[i] * q[j] / rho
                if i == j:
                    flux += P / (2.0 * mu)
                row.append(dx * alpha_q * q[i] + c[j] * flux)
        out.append(row)
    return out


def step(f, shape, dx, dt, nu, omega_rho, omega_q, alpha_rho, gamma=1.0):
    """One relax + push-transport step on a periodic grid of `shape` = (nx, ny[, nz])."""
    dim = len(shape)
    mu = dx * dx / dt
    alpha_q = nu / (2.0 * mu * (1.0 / omega_q - 0.5))
    vel = _velocities(dim)
    nsets = dim + 1
    ncell = 1
    for s in shape:
        ncell *= s
    new = [[[0.0] * ncell for _ in vel] for _ in range(nsets)]
    omega = [omega_rho] + [omega_q] * dim
    for cell in range(ncell):
        coords = []
        rem = cell
        for s in shape:
            coords.append(rem % s)
            rem //= s
        rho = 0.0
        for l in range(len(vel)):
            rho += f[0][l][cell]
        q = []
        for i in range(dim):
            acc = 0.0
            for l in range(len(vel)):
                acc += f[1 + i][l][cell]
            q.append(acc / dx)
        feq = _cell_eq(rho, q, dim, dx, mu, alpha_rho, alpha_q, gamma)
        for l, c in enumerate(vel):
            dest = 0
            stride = 1
            for k in range(dim):
                dest += ((coords[k] + c[k]) % shape[k]) * stride
                stride *= shape[k]
            for i in range(nsets):
                fs = (1.0 - omega[i]) * f[i][l][cell] + omega[i] * feq[i][l]
                new[i][l][dest] = fs
    return new


def from_array(a):
    """numpy f[i, l, (z,) y, x] -> nested lists with cell = x + nx (y + ny z)."""
    sets, vels = a.shape[0], a.shape[1]
    return [[[float(v) for v in a[i, l].ravel(order="C")] for l in range(vels)]
            for i in range(sets)]


def to_nested_shape(a):
    """Grid shape (nx, ny[, nz]) of a numpy state f[i, l, (z,) y, x]."""
    return tuple(reversed(a.shape[2:]))
