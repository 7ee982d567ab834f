"""Ghost-cell boundary conditions of the Poiseuille test (Section 5.2) for the
2D scheme, in plain numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A channel [0, L]^2 with cells centred at (i + 1/2) dx.  Before the transport
phase of each step, a ghost cell outside each side receives moments built
from the interior moments by second-order formulas (Section 5.2, "Numerical
boundary conditions"), and the post-relaxation population that the ghost
sends into the domain is the equilibrium of those moments:

* left (x = -dx/2), inlet with a prescribed velocity u_in(y):
    rho_g = 2 rho(dx/2) - rho(3dx/2),  q_g = 2 rho_bar u_in - q(dx/2);
  the +x populations of the three sets enter from it;
* right (x = L + dx/2), outlet with a prescribed pressure:
    rho_g = 2 rho_out - rho(L - dx/2),  rho_out = rho_bar (1 + dx^2 p_out)
    (the truncated relation between density and pressure of Section 3),
    q_g = 2 q(L - dx/2) - q(L - 3dx/2);
  the -x populations enter from it;
* lower (y = -dx/2) and upper (y = L + dx/2) walls moving with tangential
  velocity u_wall (0 for no-slip):
    rho_g = 2 rho(dx/2) - rho(3dx/2),  q_g = 2 rho_bar (u_wall, 0) - q(dx/2);
  the +y (lower) and -y (upper) populations enter from them, optionally plus
  the non-equilibrium part f* - f^eq(W) of the same population in the first
  interior cell (the correction of Section 5.2, needed for second order when
  the momentum sets are not relaxation schemes, omega_q != 1).

State layout and step order as in `scheme`: f[i, l, y, x], relax then
transport.  The moments a ghost uses are those of the interior at the start
of the step (relaxation does not change them).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import scheme

# velocity indices (scheme layout)
REST, XP, XM, YP, YM = 0, 1, 2, 3, 4


@dataclass(frozen=True)
class Channel:
    u_in: np.ndarray          # [2][ny] inlet velocity at x = 0 (physical units)
    rho_out: float            # outlet density target rho_bar (1 + dx^2 p_out)
    u_bottom: float = 0.0     # tangential velocity of the lower wall
    u_top: float = 0.0        # tangential velocity of the upper wall
    rho_bar: float = 1.0      # reference density
    correction: bool = False  # non-equilibrium correction on the lower and upper walls


def ghost_populations(f: np.ndarray, ch: Channel, p: scheme.Params):
    """The post-relaxation populations entering through each side, from the
    (pre-relaxation) state f at the start of a step.  Returns a dict with
    'left' [3][ny] (+x), 'right' [3][ny] (-x), 'bottom' [3][nx] (+y) and
    'top' [3][nx] (-y)."""
    rho, q = scheme.moments(f, p)                    # rho [ny][nx], q [2][ny][nx]
    rb = ch.rho_bar
    # left: inlet
    rho_g = 2 * rho[:, 0] - rho[:, 1]
    q_g = 2 * rb * ch.u_in - q[:, :, 0]
    left = scheme.equilibrium(rho_g, q_g, p)[:, XP]
    # right: outlet
    rho_g = 2 * ch.rho_out - rho[:, -1]
    q_g = 2 * q[:, :, -1] - q[:, :, -2]
    right = scheme.equilibrium(rho_g, q_g, p)[:, XM]
    # lower and upper walls
    out = {"left": left, "right": right}
    for side, row, nxt, vel, uw in (("bottom", 0, 1, YP, ch.u_bottom), ("top", -1, -2, YM, ch.u_top)):
        rho_g = 2 * rho[row] - rho[nxt]
        q_g = np.stack([2 * rb * uw - q[0, row], -q[1, row]])
        g = scheme.equilibrium(rho_g, q_g, p)[:, vel]
        if ch.correction:
            first = f[:, :, [row]]                       # the first interior row, [3][5][1][nx]
            fstar = scheme.relax(first, p)
            feq = scheme.equilibrium(rho[[row]], q[:, [row]], p)
            g = g + (fstar[:, vel, 0] - feq[:, vel, 0])
        out[side] = g
    return out


def transport(fs: np.ndarray, ghosts: dict) -> np.ndarray:
    """Transport phase on the bounded grid: interior shifts as on the torus,
    the populations entering through a side come from its ghost."""
    out = np.empty_like(fs)
    out[:, REST] = fs[:, REST]
    out[:, XP, :, 1:] = fs[:, XP, :, :-1]
    out[:, XP, :, 0] = ghosts["left"]
    out[:, XM, :, :-1] = fs[:, XM, :, 1:]
    out[:, XM, :, -1] = ghosts["right"]
    out[:, YP, 1:, :] = fs[:, YP, :-1, :]
    out[:, YP, 0, :] = ghosts["bottom"]
    out[:, YM, :-1, :] = fs[:, YM, 1:, :]
    out[:, YM, -1, :] = ghosts["top"]
    return out


def step(f: np.ndarray, ch: Channel, p: scheme.Params) -> np.ndarray:
    """One time step with the channel boundaries: ghosts from the moments at
    the start of the step, relax, transport."""
    g = ghost_populations(f, ch, p)
    return transport(scheme.relax(f, p), g)


def run(f: np.ndarray, ch: Channel, p: scheme.Params, nsteps: int) -> np.ndarray:
    for _ in range(nsteps):
        f = step(f, ch, p)
    return f


@dataclass(frozen=True)
class Poiseuille:
    """The Poiseuille test of Section 5.2 on [0, L]^2 with n cells per
    direction: u = (4U/L^2) y (L - y), v = 0, pressure p = (8 nu U / L^2)(L - x),
    nu = U L / Re; mu = dx^2/dt = 8 as in the Taylor-Green tests of Section 5.1;
    (omega_rho, alpha_rho) = (6/5, 3/40).  The run starts from the exact
    solution with the density that carries its pressure, rho = rho_bar (1 + dx^2 p)."""

    n: int
    omega_q: float
    correction: bool
    L: float = 1.0
    U: float = 1.0
    Re: float = 100.0
    mu: float = 8.0
    t_final: float = 0.05

    @property
    def nu(self) -> float:
        return self.U * self.L / self.Re

    @property
    def dx(self) -> float:
        return self.L / self.n

    def params(self) -> scheme.Params:
        return scheme.Params(dim=2, dx=self.dx, dt=self.dx * self.dx / self.mu, nu=self.nu, omega_q=self.omega_q)

    def centres(self) -> np.ndarray:
        return (np.arange(self.n) + 0.5) * self.dx

    def u_exact(self, y):
        return 4 * self.U / self.L ** 2 * y * (self.L - y)

    def p_exact(self, x):
        return 8 * self.nu * self.U / self.L ** 2 * (self.L - x)

    def steps(self) -> int:
        p = self.params()
        return int(round(self.t_final / p.dt))

    def initial(self):
        c = self.centres()
        rho0 = np.broadcast_to(1.0 + self.dx ** 2 * self.p_exact(c)[None, :], (self.n, self.n)).copy()
        u0 = np.zeros((2, self.n, self.n))
        u0[0] = self.u_exact(c)[:, None]
        return rho0, u0

    def channel(self) -> Channel:
        c = self.centres()
        u_in = np.stack([self.u_exact(c), np.zeros(self.n)])
        return Channel(u_in=u_in, rho_out=1.0 + self.dx ** 2 * self.p_exact(self.L), correction=self.correction)

    def error(self, f: np.ndarray) -> float:
        """Absolute discrete L2 error on u_x: sqrt(dx^2 sum (u_x - u_ex)^2) (reading A6)."""
        rho, q = scheme.moments(f, self.params())
        ux = q[0] / rho
        e = ux - self.u_exact(self.centres())[:, None]
        return float(np.sqrt(self.dx ** 2 * np.sum(e * e)))

    def solve(self, steps: int | None = None):
        p = self.params()
        rho0, u0 = self.initial()
        f = scheme.init(rho0, u0, p)
        f = run(f, self.channel(), p, self.steps() if steps is None else steps)
        return f
