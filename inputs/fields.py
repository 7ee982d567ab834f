"""Seeded synthetic velocity fields sampled at cell centres (FP64).

Grid convention: a periodic box [0, L)^d with N cells per axis, spacing
dx = L / N, cell centres at (i + 1/2) dx (the half-integer grid of the
scheme's definition, Section 2).  Arrays are indexed [y, x] in 2D and
[z, y, x] in 3D, so x is the fastest (last) axis.

Every field here is an exact, divergence-free velocity sampled pointwise, so
the same continuous field exists at every resolution.  Nothing in this module
knows about distributions, equilibria or time stepping.
"""

from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def cell_centres(n: int, length: float = TWO_PI) -> np.ndarray:
    """Cell-centre coordinates (i + 1/2) * L / n for i = 0..n-1."""
    dx = length / n
    return (np.arange(n, dtype=np.float64) + 0.5) * dx


# --------------------------------------------------------------------------- #
# Closed-form flows                                                           #
# --------------------------------------------------------------------------- #

def taylor_green(n: int, amplitude: float = 1.0, length: float = TWO_PI):
    """Taylor-Green vortex u = U (sin x cos y, -cos x sin y) on [0, 2pi)^2.

    Returns u with shape (2, n, n) ([component, y, x]).  Under the
    Navier-Stokes system it decays as exp(-2 nu t) (wavenumber |k|^2 = 2).
    """
    x = cell_centres(n, length)
    y = x
    X = x[None, :]
    Y = y[:, None]
    ux = amplitude * np.sin(X) * np.cos(Y)
    uy = -amplitude * np.cos(X) * np.sin(Y)
    return np.stack([ux, uy]).astype(np.float64)


def taylor_green_pressure(n: int, amplitude: float = 1.0, length: float = TWO_PI):
    """Kinematic pressure Phi = U^2/4 (cos 2x + cos 2y) of the vortex at t=0.

    It balances the convective term: grad Phi = -(u . grad) u.
    """
    x = cell_centres(n, length)
    X = x[None, :]
    Y = x[:, None]
    return 0.25 * amplitude ** 2 * (np.cos(2 * X) + np.cos(2 * Y))


def shear_wave(ny: int, nx: int = 1, amplitude: float = 1.0, k: int = 1,
               length_y: float = TWO_PI):
    """Shear wave u = (U sin(k y), 0), an exact solution decaying as exp(-nu k^2 t).

    The field does not depend on x, so any nx (including 1) samples it; the
    grid spacing is length_y / ny in both directions.
    """
    y = cell_centres(ny, length_y)
    ux = amplitude * np.sin(k * y)[:, None] * np.ones((1, nx))
    uy = np.zeros((ny, nx))
    return np.stack([ux, uy])


def abc_flow(n: int, a: float = 1.0, b: float = 1.0, c: float = 1.0,
             length: float = TWO_PI):
    """Arnold-Beltrami-Childress flow, shape (3, n, n, n) ([comp, z, y, x]).

    u = (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x).  It is a
    Beltrami field (curl u = u), so (u . grad) u = grad(|u|^2 / 2) and it
    decays as exp(-nu t) with pressure Phi = -|u|^2 / 2.
    """
    s = cell_centres(n, length)
    Z = s[:, None, None]
    Y = s[None, :, None]
    X = s[None, None, :]
    ux = a * np.sin(Z) + c * np.cos(Y) + 0 * X
    uy = b * np.sin(X) + a * np.cos(Z) + 0 * Y
    uz = c * np.sin(Y) + b * np.cos(X) + 0 * Z
    return np.stack(np.broadcast_arrays(ux, uy, uz)).astype(np.float64)


def abc_pressure(u: np.ndarray) -> np.ndarray:
    return -0.5 * np.sum(u * u, axis=0)


def well_prepared_density(phi: np.ndarray, dx: float, rho_bar: float = 1.0,
                          gamma: float = 1.0) -> np.ndarray:
    """Density whose pressure carries the incompressible pressure field.

    Solves P(rho) = P(rho_bar) + dx^2 rho_bar Phi for P(rho) = rho^gamma, the
    assumption under which the density stays within O(dx^2) of rho_bar
    (Section 3, Proposition 1).
    """
    return (rho_bar ** gamma + dx * dx * rho_bar * phi) ** (1.0 / gamma)


# --------------------------------------------------------------------------- #
# Seeded band-limited random fields with an |k|^-3 amplitude law              #
# --------------------------------------------------------------------------- #

def _hermitian(coef: np.ndarray) -> np.ndarray:
    """Symmetrise c(k) -> (c(k) + conj(c(-k))) / 2 so the field is real."""
    flipped = coef[(slice(None, None, -1),) * coef.ndim]
    return 0.5 * (coef + np.conj(flipped))


def _coeffs(seed: int, kmax: int, dim: int, ncomp: int) -> tuple[np.ndarray, np.ndarray]:
    """Draw (a + i b) / |k|^3 for all integer k in [-kmax, kmax]^dim.

    The draw order is fixed and independent of the grid size: one call to
    default_rng(seed).standard_normal of shape (ncomp, 2, (2kmax+1)^dim).
    Modes outside 1 <= |k| <= kmax are zeroed afterwards.
    Returns (coefficients [ncomp, k...], integer wavenumbers per axis).
    """
    rng = np.random.default_rng(seed)
    side = 2 * kmax + 1
    draw = rng.standard_normal((ncomp, 2) + (side,) * dim)
    k1 = np.arange(-kmax, kmax + 1, dtype=np.float64)
    grids = np.meshgrid(*([k1] * dim), indexing="ij")
    kk = np.sqrt(sum(g * g for g in grids))
    mask = (kk >= 1.0) & (kk <= kmax)
    amp = np.zeros_like(kk)
    amp[mask] = 1.0 / kk[mask] ** 3
    coef = (draw[:, 0] + 1j * draw[:, 1]) * amp[None]
    coef = np.stack([_hermitian(c) for c in coef])
    return coef, k1


def _synth_2d(coef: np.ndarray, k1: np.ndarray, n: int, length: float) -> np.ndarray:
    """Real part of sum_k c[ky, kx] exp(i (kx x + ky y)) at cell centres -> [y, x]."""
    s = cell_centres(n, length)
    e = np.exp(1j * np.outer(k1, s))  # [k, position]
    return np.real(e.T @ coef @ e)


def _synth_3d(coef: np.ndarray, k1: np.ndarray, n: int, length: float) -> np.ndarray:
    """Real part of sum_k c[kz, ky, kx] exp(i k . x) at cell centres -> [z, y, x]."""
    s = cell_centres(n, length)
    e = np.exp(1j * np.outer(k1, s))  # [k, position]
    g = np.tensordot(coef, e, axes=([2], [0]))        # [kz, ky, x]
    g = np.tensordot(g, e, axes=([1], [0]))           # [kz, x, y]
    g = np.transpose(g, (0, 2, 1))                    # [kz, y, x]
    out = np.tensordot(e.real, g.real, axes=([0], [0])) - np.tensordot(e.imag, g.imag, axes=([0], [0]))
    return out                                         # [z, y, x]


def _velocity_2d(seed: int, n: int, kmax: int, length: float) -> np.ndarray:
    coef, k1 = _coeffs(seed, kmax, 2, 1)
    psi = coef[0]                      # indexed [ky, kx]
    ky = k1[:, None]
    kx = k1[None, :]
    ux = _synth_2d(1j * ky * psi, k1, n, length)     # d psi / dy
    uy = _synth_2d(-1j * kx * psi, k1, n, length)    # -d psi / dx
    return np.stack([ux, uy])


def random_field_2d(n: int, seed: int, umax: float = 1.0, kmax: int = 16,
                    length: float = TWO_PI, norm_n: int = 256) -> np.ndarray:
    """Divergence-free u = (d_y psi, -d_x psi) with psi_hat(k) ~ (a + ib)/|k|^3.

    Modes 1 <= |k| <= kmax (energy spectrum ~ k^-3).  The field is scaled so
    that its maximum speed over the cell centres of a norm_n^2 reference grid
    equals umax; the scale does not depend on n, so every resolution samples
    the same continuous field.  Returns shape (2, n, n).
    """
    u = _velocity_2d(seed, n, kmax, length)
    ref = u if n == norm_n else _velocity_2d(seed, norm_n, kmax, length)
    scale = umax / float(np.sqrt(np.max(np.sum(ref * ref, axis=0))))
    return u * scale


def _velocity_3d(seed: int, n: int, kmax: int, length: float) -> np.ndarray:
    coef, k1 = _coeffs(seed, kmax, 3, 3)           # vector potential A_hat[c, kz, ky, kx]
    kz = k1[:, None, None]
    ky = k1[None, :, None]
    kx = k1[None, None, :]
    ax, ay, az = coef
    # u = curl A:  (dy Az - dz Ay, dz Ax - dx Az, dx Ay - dy Ax)
    ux = _synth_3d(1j * (ky * az - kz * ay), k1, n, length)
    uy = _synth_3d(1j * (kz * ax - kx * az), k1, n, length)
    uz = _synth_3d(1j * (kx * ay - ky * ax), k1, n, length)
    return np.stack([ux, uy, uz])


def random_field_3d(n: int, seed: int, umax: float = 1.0, kmax: int = 16,
                    length: float = TWO_PI, norm_n: int = 64) -> np.ndarray:
    """Divergence-free u = curl A with each A_hat component ~ (a + ib)/|k|^3.

    Same construction and normalisation rule as random_field_2d, on a
    norm_n^3 reference grid.  Returns shape (3, n, n, n).
    """
    u = _velocity_3d(seed, n, kmax, length)
    ref = u if n == norm_n else _velocity_3d(seed, norm_n, kmax, length)
    scale = umax / float(np.sqrt(np.max(np.sum(ref * ref, axis=0))))
    return u * scale


def random_field_box(shape, dx: float, seed: int, umax: float = 1.0, mmax: int = 3) -> np.ndarray:
    """Smooth divergence-free field on a periodic box of any shape.

    shape = (ny, nx) or (nz, ny, nx) cells of spacing dx, so the box sides are
    L_a = n_a dx.  Modes exp(i k . x) with k_a = 2 pi m_a / L_a for integer
    m in [-mmax, mmax]^d, 1 <= |m| <= mmax, coefficients (a + ib)/|m|^3 from
    default_rng(seed); 2D: u = (d_y psi, -d_x psi); 3D: u = curl A.  Scaled so
    that max |u| over the grid equals umax.  Returns (d, *shape).
    """
    dim = len(shape)
    ncomp = 1 if dim == 2 else 3
    coef, m1 = _coeffs(seed, mmax, dim, ncomp)
    sizes = list(reversed(shape))                        # (nx, ny[, nz])
    # e[a][m, i] = exp(i k_a(m) x_i), axis a = 0 is x
    e = []
    kv = []
    for a in range(dim):
        L = sizes[a] * dx
        k = 2 * math.pi * m1 / L
        x = (np.arange(sizes[a]) + 0.5) * dx
        e.append(np.exp(1j * np.outer(k, x)))
        kv.append(k)

    def synth(c):                                        # c indexed [.., ky, kx] -> real field
        if dim == 2:
            return np.real(e[1].T @ c @ e[0])
        g = np.tensordot(c, e[0], axes=([2], [0]))       # [kz, ky, x]
        g = np.tensordot(g, e[1], axes=([1], [0]))       # [kz, x, y]
        g = np.transpose(g, (0, 2, 1))                   # [kz, y, x]
        return np.real(np.tensordot(e[2], g, axes=([0], [0])))

    if dim == 2:
        ky = kv[1][:, None]
        kx = kv[0][None, :]
        psi = coef[0]
        u = np.stack([synth(1j * ky * psi), synth(-1j * kx * psi)])
    else:
        kz = kv[2][:, None, None]
        ky = kv[1][None, :, None]
        kx = kv[0][None, None, :]
        ax, ay, az = coef
        u = np.stack([synth(1j * (ky * az - kz * ay)), synth(1j * (kz * ax - kx * az)),
                      synth(1j * (kx * ay - ky * ax))])
    return u * (umax / float(np.sqrt(np.max(np.sum(u * u, axis=0)))))


def pressure_coefficients(u: np.ndarray, length: float = TWO_PI):
    """Fourier coefficients of the kinematic pressure of a periodic 2D field.

    u: samples (2, m, m) at cell centres of a band-limited field whose
    products u_i u_j are resolved on the m x m grid (no aliasing).  The
    incompressible pressure solves  lap Phi = -d_i d_j (u_i u_j)  (the
    divergence of the momentum equation), i.e. Phi_hat = -k_i k_j P_ij_hat / |k|^2
    with zero mean.  Returns (c, k) with Phi(x, y) = sum c[ky, kx] exp(i (kx x + ky y)),
    k the integer-scaled wavenumbers of numpy's FFT order.
    """
    m = u.shape[-1]
    h = length / m
    k = 2 * math.pi * np.fft.fftfreq(m, d=h)
    ky = k[:, None]
    kx = k[None, :]
    shift = np.exp(-1j * (kx + ky) * h / 2)           # samples sit at (j + 1/2) h
    P = [[np.fft.fft2(u[i] * u[j]) * shift / (m * m) for j in range(2)] for i in range(2)]
    kk = [kx, ky]
    k2 = kx * kx + ky * ky
    num = sum(kk[i] * kk[j] * P[i][j] for i in range(2) for j in range(2))
    c = np.zeros_like(num)
    nz = k2 > 0
    c[nz] = -num[nz] / k2[nz]
    return c, k


def pressure_at(c: np.ndarray, k: np.ndarray, n: int, length: float = TWO_PI) -> np.ndarray:
    """Evaluate sum c[ky, kx] exp(i k . x) at the cell centres of an n x n grid."""
    x = cell_centres(n, length)
    e = np.exp(1j * np.outer(k, x))                    # [k, position]
    return np.real(e.T @ c @ e)


def random_pressure_2d(n: int, seed: int, umax: float = 1.0, kmax: int = 16,
                       length: float = TWO_PI, norm_n: int = 256) -> np.ndarray:
    """Kinematic pressure of random_field_2d(n, seed, umax, kmax) at cell centres.

    The velocity has modes |k| <= kmax, so u_i u_j has |k| <= 2 kmax and is
    resolved exactly on a 4 kmax + 4 grid; the pressure coefficients computed
    there are evaluated at the n x n cell centres.
    """
    m = 4 * kmax + 4
    u = random_field_2d(m, seed, umax, kmax, length, norm_n)
    c, k = pressure_coefficients(u, length)
    return pressure_at(c, k, n, length)


# --------------------------------------------------------------------------- #
# The batch workload: many independent runs of uneven size and viscosity      #
# --------------------------------------------------------------------------- #

BATCH_SIZES = (64, 128, 256, 512, 1024)


def batch_run_specs(n_runs: int = 512, sizes=BATCH_SIZES, log_nu=(-4.0, -2.0)):
    """Run r draws its grid size uniformly from `sizes`, nu = 10^U(log_nu),
    and uses field seed r, from numpy default_rng(r).  Returns a list of dicts."""
    specs = []
    for r in range(n_runs):
        rng = np.random.default_rng(r)
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        nu = float(10.0 ** rng.uniform(log_nu[0], log_nu[1]))
        specs.append({"run": r, "n": n, "nu": nu, "seed": r})
    return specs
