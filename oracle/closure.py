"""Coarse-grid learned correction: restriction, correction, guard (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no closure; the definitions are:

restriction (fine -> coarse, factor r = dx_c / dx_f, block averages):
    q_c   = mean of q_f over each r x r block   (physical momentum)
    rho_c = rho_ref + r^2 (mean of rho_f - rho_ref)
  The density carries the pressure, rho - rho_ref ~ dx^2 Phi (eq. (3.2)), so the
  density deviation of the same pressure field is r^2 larger on the coarse grid.

network input (per coarse cell):  ((rho - rho_ref) / s_rho, u_x / s_u, u_y / s_u)
network output:                   (d_rho / s_drho, d_q_x / s_dq, d_q_y / s_dq)

projection: each output channel minus its grid mean, so the correction leaves
total mass and momentum unchanged.

guard: with u = q / rho before and u' = (q + dq) / (rho + drho) after, accept the
correction only if it is finite and ||div_h u'||_2 <= factor * ||div_h u||_2.

correction: f <- f + f^eq(rho + drho, q + dq) - f^eq(rho, q): the moments move by
exactly (drho, dq) and the non-equilibrium part f - f^eq is unchanged.
"""

from __future__ import annotations

import numpy as np

from . import cnn, diagnostics, scheme


def restrict(rho_f: np.ndarray, q_f: np.ndarray, r: int, rho_ref: float = 1.0):
    ny, nx = rho_f.shape
    assert ny % r == 0 and nx % r == 0

    def block_mean(a):
        return a.reshape(a.shape[:-2] + (ny // r, r, nx // r, r)).mean(axis=(-3, -1))

    rho_c = rho_ref + r * r * (block_mean(rho_f) - rho_ref)
    return rho_c, block_mean(q_f)


def net_input(rho, q, scales, rho_ref=1.0):
    u = q / rho[None]
    return np.stack([(rho - rho_ref) / scales["s_rho"], u[0] / scales["s_u"], u[1] / scales["s_u"]])


def net_output_to_dw(y, scales):
    """Network output -> (d_rho, d_q) in physical units, zero-mean per channel."""
    d_rho = y[0] * scales["s_drho"]
    d_q = np.stack([y[1], y[2]]) * scales["s_dq"]
    d_rho = d_rho - d_rho.mean()
    d_q = d_q - d_q.mean(axis=(-2, -1), keepdims=True)
    return d_rho, d_q


def guard(rho, q, d_rho, d_q, dx, factor=2.0):
    u0 = q / rho[None]
    rho1 = rho + d_rho
    u1 = (q + d_q) / rho1[None]
    if not (np.all(np.isfinite(rho1)) and np.all(np.isfinite(u1))):
        return False, np.inf, np.inf
    div0 = float(np.sqrt(dx * dx * np.sum(diagnostics.divergence(u0, dx) ** 2)))
    div1 = float(np.sqrt(dx * dx * np.sum(diagnostics.divergence(u1, dx) ** 2)))
    return div1 <= factor * div0, div0, div1


def apply_correction(f, p: scheme.Params, d_rho, d_q):
    rho, q = scheme.moments(f, p)
    return f + scheme.equilibrium(rho + d_rho, q + d_q, p) - scheme.equilibrium(rho, q, p)


def closure_run(f, p: scheme.Params, params, scales, steps: int, every: int = 4,
                guard_factor: float = 2.0):
    """Advance `steps` steps; after every `every` steps apply the guarded network
    correction.  Returns (f, number of accepted corrections, number rejected)."""
    acc = rej = 0
    done = 0
    while done < steps:
        k = min(every, steps - done)
        f = scheme.run(f, p, k)
        done += k
        if k < every:
            break
        rho, q = scheme.moments(f, p)
        x = net_input(rho, q, scales)[None]
        y, _ = cnn.forward(params, x)
        d_rho, d_q = net_output_to_dw(y[0], scales)
        ok, _, _ = guard(rho, q, d_rho, d_q, p.dx, guard_factor)
        if ok:
            f = apply_correction(f, p, d_rho, d_q)
            acc += 1
        else:
            rej += 1
    return f, acc, rej


def solenoidal(u: np.ndarray) -> np.ndarray:
    """Divergence-free part of a periodic 2D field u[2][n][n] (x last): the
    spectral Helmholtz projection u^(k) - k (k . u^(k)) / |k|^2 for every
    wavenumber k != 0, with numpy's signed frequencies (fftfreq) and the mean
    kept.  The correction network is trained on the divergence-free part of
    the fine-minus-coarse momentum difference."""
    n = u.shape[-1]
    k = np.fft.fftfreq(n, 1.0 / n)
    kx, ky = k[None, :], k[:, None]
    k2 = kx * kx + ky * ky
    k2[0, 0] = 1.0
    ux, uy = np.fft.fft2(u[0]), np.fft.fft2(u[1])
    div = kx * ux + ky * uy
    return np.stack([np.fft.ifft2(ux - kx * div / k2).real, np.fft.ifft2(uy - ky * div / k2).real])


def projected_target(m_fine: np.ndarray, m_now: np.ndarray) -> np.ndarray:
    """Training target of a window: the density of the coarse state and its
    momentum plus the divergence-free part of the fine-minus-coarse momentum
    difference (moment planes [3][n][n]: rho, q_x, q_y)."""
    out = m_now.astype(np.float64).copy()
    out[1:] += solenoidal(m_fine[1:].astype(np.float64) - m_now[1:].astype(np.float64))
    return out
