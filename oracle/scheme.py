"""The vectorial D2Q5 / D3Q7 lattice Boltzmann scheme in plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Section 2 of the paper step by step, in its notation:

* one distribution set per conserved component i in {rho, q_x, q_y[, q_z]},
  each over the velocities {o, +x, -x, +y, -y[, +z, -z]} (the paper's
  circle / right / left / up / down triangles);
* moments (rho, dx q_x, dx q_y) = sum over velocities (Section 2, relaxation
  phase);
* equilibria f^eq(rho, q) exactly as printed in Section 2, with the reading
  that the rest component of each momentum set is dx (1 - 4 alpha) q (the
  printed form lacks the factor dx; only with it do the equilibria sum to
  the moments, and only with it does the checkerboard determinant of
  Lemma 1 hold);
* BGK relaxation f* = (1 - omega_i) f + omega_i f^eq, one omega per set
  (equation (LBM_scheme));
* transport: the rest population stays, +e_j populations move by +dx along
  axis j, -e_j by -dx, on a periodic lattice;
* initial distributions at equilibrium.

In 3D the rest weight becomes (1 - 6 alpha) and the z velocities follow the
same pattern as x and y (the paper states the extension is straightforward
because the scheme is Cartesian).

State layout: f[i, l, (z,) y, x] with set index i (0 = rho, 1 + j = q_j) and
velocity index l (0 = rest, 1 + 2j = +e_j, 2 + 2j = -e_j), axis j = 0 for x.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Params:
    """Scheme parameters.  mu = dx^2 / dt is the parabolic scaling (eq. 2.1);
    alpha_q follows from the viscosity relation at the end of Section 3:
    nu = 2 mu alpha_q (1/omega_q - 1/2)."""

    dim: int
    dx: float
    dt: float
    nu: float
    omega_rho: float = 6.0 / 5.0
    omega_q: float = 23.0 / 20.0
    alpha_rho: float = 3.0 / 40.0
    gamma: float = 1.0

    @property
    def mu(self) -> float:
        return self.dx * self.dx / self.dt

    @property
    def alpha_q(self) -> float:
        return self.nu / (2.0 * self.mu * (1.0 / self.omega_q - 0.5))

    @property
    def omegas(self) -> np.ndarray:
        return np.array([self.omega_rho] + [self.omega_q] * self.dim)

    @property
    def alphas(self) -> np.ndarray:
        return np.array([self.alpha_rho] + [self.alpha_q] * self.dim)

    def validate(self) -> None:
        """Reject parameters outside the admissible ranges.

        omega in (0, 2): omega = 2 gives an inviscid scheme (Section 3).
        alpha in [0, 1/(2 dim)]: Lemma 1 (checkerboard mode) gives [0, 1/4]
        in 2D; the same argument gives [0, 1/6] in 3D.
        """
        if self.dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if not (self.dx > 0 and self.dt > 0):
            raise ValueError("dx and dt must be positive")
        for w in self.omegas:
            if not (0.0 < w < 2.0):
                raise ValueError(f"relaxation parameter {w} outside (0, 2)")
        for a in self.alphas:
            if not (0.0 <= a <= 1.0 / (2 * self.dim)):
                raise ValueError(f"alpha {a} outside [0, 1/(2d)]")


def params_for_grid(dim: int, n: int, nu: float, mu: float = 8.0,
                    length: float = 2.0 * math.pi, **kw) -> Params:
    """Parameters for n cells per axis on [0, length)^dim at scaling mu."""
    dx = length / n
    return Params(dim=dim, dx=dx, dt=dx * dx / mu, nu=nu, **kw)


def n_velocities(dim: int) -> int:
    return 2 * dim + 1


def pressure(rho, gamma: float):
    """Pressure law P(rho) = rho^gamma (Section 2)."""
    return rho ** gamma


def moments(f: np.ndarray, p: Params):
    """rho = sum_l f_rho,l and q_j = (1/dx) sum_l f_qj,l."""
    rho = f[0].sum(axis=0)
    q = f[1:].sum(axis=1) / p.dx
    return rho, q


def equilibrium(rho: np.ndarray, q: np.ndarray, p: Params) -> np.ndarray:
    """f^eq(rho, q) of Section 2, extended per axis to 3D."""
    d, dx, mu = p.dim, p.dx, p.mu
    a = p.alphas
    shape = (d + 1, n_velocities(d)) + rho.shape
    feq = np.empty(shape, dtype=np.float64)
    # density set: rest (1 - 2d alpha_rho) rho, moving alpha_rho rho +- dx/(2 mu) q_j
    feq[0, 0] = (1.0 - 2 * d * a[0]) * rho
    for j in range(d):
        feq[0, 1 + 2 * j] = a[0] * rho + dx / (2.0 * mu) * q[j]
        feq[0, 2 + 2 * j] = a[0] * rho - dx / (2.0 * mu) * q[j]
    P = pressure(rho, p.gamma)
    for i in range(d):
        ai = a[1 + i]
        feq[1 + i, 0] = dx * (1.0 - 2 * d * ai) * q[i]
        for j in range(d):
            flux = dx * dx / (2.0 * mu) * q[i] * q[j] / rho
            if i == j:
                flux = flux + P / (2.0 * mu)
            feq[1 + i, 1 + 2 * j] = dx * ai * q[i] + flux
            feq[1 + i, 2 + 2 * j] = dx * ai * q[i] - flux
    return feq


def relax(f: np.ndarray, p: Params) -> np.ndarray:
    """Relaxation phase: f* = diag(1 - omega) f + diag(omega) f^eq(W(f))."""
    rho, q = moments(f, p)
    feq = equilibrium(rho, q, p)
    w = p.omegas.reshape((p.dim + 1, 1) + (1,) * p.dim)
    return (1.0 - w) * f + w * feq


def transport(fs: np.ndarray, dim: int) -> np.ndarray:
    """Transport phase on the periodic lattice.

    f_{+e_j}(t + dt, x) = f*_{+e_j}(t, x - dx e_j) and
    f_{-e_j}(t + dt, x) = f*_{-e_j}(t, x + dx e_j); the rest population stays.
    Axis j = 0 (x) is the last array axis.
    """
    out = np.empty_like(fs)
    out[:, 0] = fs[:, 0]
    for j in range(dim):
        ax = (fs.ndim - 2) - j  # axis of direction j within the (set, *grid) slice
        out[:, 1 + 2 * j] = np.roll(fs[:, 1 + 2 * j], +1, axis=ax)
        out[:, 2 + 2 * j] = np.roll(fs[:, 2 + 2 * j], -1, axis=ax)
    return out


def step(f: np.ndarray, p: Params) -> np.ndarray:
    """One time step: relax, then transport."""
    return transport(relax(f, p), p.dim)


def init(rho0: np.ndarray, u0: np.ndarray, p: Params) -> np.ndarray:
    """Distributions at equilibrium of (rho0, q0 = rho0 u0) (end of Section 2)."""
    q0 = rho0[None] * u0
    return equilibrium(rho0, q0, p)


def run(f: np.ndarray, p: Params, nsteps: int) -> np.ndarray:
    for _ in range(nsteps):
        f = step(f, p)
    return f


def velocity(f: np.ndarray, p: Params) -> np.ndarray:
    rho, q = moments(f, p)
    return q / rho[None]


def simulate(u0: np.ndarray, p: Params, nsteps: int, rho0: np.ndarray | None = None):
    """Initialise at equilibrium and advance nsteps.  Returns (rho, q, f)."""
    if rho0 is None:
        rho0 = np.ones(u0.shape[1:])
    f = run(init(rho0, u0, p), p, nsteps)
    rho, q = moments(f, p)
    return rho, q, f
