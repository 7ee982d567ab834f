"""Linearised amplification matrix of the scheme (Section 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a reference state (rho_bar, q_bar) and a frequency theta = xi dx, a Fourier
mode f_hat e^{i xi . x} of the linearised scheme evolves as
f_hat(t + dt) = E(theta) f_hat(t) with

    E(theta) = S(theta) [ diag(1 - omega) + diag(omega) J M ]

where M maps distributions to the moments (rho, q) (q = sum / dx), J is the
Jacobian of the equilibria with respect to (rho, q) at the reference state
(written out by hand below from the formulas of Section 2, independently of
`scheme.equilibrium`), and S(theta) = diag(exp(-i theta . c_l)) is the
transport of the population with velocity c_l by one cell.

Population index: set i (0 = rho, 1 + j = q_j) times (2 dim + 1) + velocity l
(0 = rest, 1 + 2j = +e_j, 2 + 2j = -e_j).
"""

from __future__ import annotations

import numpy as np


def _vel(dim):
    v = [np.zeros(dim, dtype=int)]
    for j in range(dim):
        e = np.zeros(dim, dtype=int)
        e[j] = 1
        v.append(e.copy())
        v.append(-e)
    return v


def moment_matrix(dim: int, dx: float) -> np.ndarray:
    """M: populations -> (rho, q_1, .., q_dim); q_j = (1/dx) sum_l f_{q_j, l}."""
    nv = 2 * dim + 1
    M = np.zeros((dim + 1, (dim + 1) * nv))
    M[0, 0:nv] = 1.0
    for j in range(dim):
        M[1 + j, (1 + j) * nv:(2 + j) * nv] = 1.0 / dx
    return M


def equilibrium_jacobian(dim, dx, mu, alpha_rho, alpha_q, rho_bar, q_bar, gamma=1.0):
    """d f^eq / d(rho, q) at (rho_bar, q_bar), from the Section 2 formulas.

    density set:   rest (1 - 2d a_rho) rho           -> d/drho = 1 - 2d a_rho
                   +-e_j: a_rho rho +- dx/(2mu) q_j   -> d/drho = a_rho, d/dq_j = +-dx/(2mu)
    momentum q_i:  rest dx (1 - 2d a) q_i             -> d/dq_i = dx (1 - 2d a)
                   +-e_j: dx a q_i +- [dx^2/(2mu) q_i q_j / rho + delta_ij P(rho)/(2mu)]
    """
    nv = 2 * dim + 1
    vel = _vel(dim)
    alphas = [alpha_rho] + [alpha_q] * dim
    J = np.zeros(((dim + 1) * nv, dim + 1))
    qb = np.asarray(q_bar, dtype=float)
    dP = gamma * rho_bar ** (gamma - 1.0)
    for l, c in enumerate(vel):
        moving = np.any(c != 0)
        j = int(np.nonzero(c)[0][0]) if moving else -1
        sgn = float(c[j]) if moving else 0.0
        # density set
        r = l
        if not moving:
            J[r, 0] = 1.0 - 2 * dim * alphas[0]
        else:
            J[r, 0] = alphas[0]
            J[r, 1 + j] = sgn * dx / (2.0 * mu)
        # momentum sets
        for i in range(dim):
            r = (1 + i) * nv + l
            a = alphas[1 + i]
            if not moving:
                J[r, 1 + i] = dx * (1.0 - 2 * dim * a)
                continue
            k = dx * dx / (2.0 * mu)
            # d/dq_k of dx a q_i
            J[r, 1 + i] += dx * a
            # d of +- k q_i q_j / rho
            J[r, 1 + i] += sgn * k * qb[j] / rho_bar
            J[r, 1 + j] += sgn * k * qb[i] / rho_bar
            J[r, 0] += -sgn * k * qb[i] * qb[j] / rho_bar ** 2
            if i == j:
                J[r, 0] += sgn * dP / (2.0 * mu)
    return J


def amplification_matrix(theta, dim, dx, mu, omega_rho, omega_q, alpha_rho, alpha_q,
                         rho_bar=1.0, q_bar=None, gamma=1.0) -> np.ndarray:
    """E(theta) of Section 4, size (dim+1)(2dim+1) square, complex."""
    theta = np.asarray(theta, dtype=float)
    if q_bar is None:
        q_bar = np.zeros(dim)
    nv = 2 * dim + 1
    n = (dim + 1) * nv
    M = moment_matrix(dim, dx)
    J = equilibrium_jacobian(dim, dx, mu, alpha_rho, alpha_q, rho_bar, q_bar, gamma)
    omega = np.repeat([omega_rho] + [omega_q] * dim, nv)
    C = np.diag(1.0 - omega) + np.diag(omega) @ J @ M
    phase = np.array([np.exp(-1j * float(theta @ c)) for c in _vel(dim)] * (dim + 1))
    assert phase.shape == (n,)
    return np.diag(phase) @ C


def checkerboard_eigenvalues(dim, omegas, alphas) -> np.ndarray:
    """Roots of prod_i (z - omega_i + 1)^(2d-1) (z^2 - omega_i (1 - 4 d alpha_i) z + omega_i - 1).

    Lemma 1 gives this determinant in 2D (exponent 3, coefficient 1 - 8 alpha);
    the 3D form follows from the same computation with 2d + 1 = 7 velocities.
    """
    roots = []
    for w, a in zip(omegas, alphas):
        roots += [w - 1.0] * (2 * dim - 1)
        roots += list(np.roots([1.0, -w * (1.0 - 4 * dim * a), w - 1.0]))
    return np.array(roots, dtype=complex)


def relaxation_scheme_matrix(theta, dim, mu, alpha_rho, alpha_q) -> np.ndarray:
    """omega = 1, reference (1, 0): the (dim+1) x (dim+1) matrix acting on W.

    With omega = 1 the post-relaxation state is f^eq(W), so
    W(t+1, x) = sum_l f^eq_l(W(t, x - c_l)); linearised about (1, 0) in the
    scaled variables (rho, dx q) this is
        [[1 - 2 a_rho c, -i s_1/mu, ..], [-i s_j/mu, delta (1 - 2 a_q c), ..]]
    with c = sum_j (1 - cos theta_j) and s_j = sin theta_j.
    """
    theta = np.asarray(theta, dtype=float)
    c = float(np.sum(1.0 - np.cos(theta)))
    s = np.sin(theta)
    A = np.zeros((dim + 1, dim + 1), dtype=complex)
    A[0, 0] = 1.0 - 2.0 * alpha_rho * c
    for j in range(dim):
        A[0, 1 + j] = -1j * s[j] / mu
        A[1 + j, 0] = -1j * s[j] / mu
        A[1 + j, 1 + j] = 1.0 - 2.0 * alpha_q * c
    return A
