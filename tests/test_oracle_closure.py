"""Pins of the coarse-grid correction reference (restriction, correction, guard)."""

import math

import numpy as np
import pytest

import inputs
from oracle import closure, cnn, scheme


def test_restriction_of_blockwise_constant_fields():
    rng = np.random.default_rng(0)
    r = 4
    rc = 1 + 0.01 * rng.standard_normal((3, 5))
    qc = rng.standard_normal((2, 3, 5))
    rho_f = 1 + (rc - 1) / r ** 2
    rho_f = np.kron(rho_f, np.ones((r, r)))
    q_f = np.stack([np.kron(qc[j], np.ones((r, r))) for j in range(2)])
    rho2, q2 = closure.restrict(rho_f, q_f, r)
    assert np.allclose(rho2, rc, atol=1e-14)
    assert np.allclose(q2, qc, atol=1e-14)


def test_restriction_conserves_momentum_integral():
    rng = np.random.default_rng(1)
    r, dxf = 8, 0.01
    q_f = rng.standard_normal((2, 32, 48))
    rho_f = 1 + 1e-4 * rng.standard_normal((32, 48))
    _, q_c = closure.restrict(rho_f, q_f, r)
    assert np.allclose(q_c.sum(axis=(1, 2)) * (r * dxf) ** 2, q_f.sum(axis=(1, 2)) * dxf ** 2)


def _state(n=16, seed=0):
    p = scheme.params_for_grid(2, n, 0.01, omega_q=1.3)
    u = inputs.random_field_2d(n, seed, umax=0.05 / p.dx)
    f = scheme.run(scheme.init(np.ones((n, n)), u, p), p, 7)  # carries a non-equilibrium part
    return f, p


def test_correction_moves_moments_exactly_and_keeps_nonequilibrium():
    f, p = _state()
    rng = np.random.default_rng(2)
    rho, q = scheme.moments(f, p)
    d_rho = 1e-4 * rng.standard_normal(rho.shape)
    d_q = 1e-2 * rng.standard_normal(q.shape)
    g = closure.apply_correction(f, p, d_rho, d_q)
    rho2, q2 = scheme.moments(g, p)
    assert np.allclose(rho2, rho + d_rho, atol=1e-14)
    assert np.allclose(q2, q + d_q, atol=1e-12)
    neq_before = f - scheme.equilibrium(rho, q, p)
    neq_after = g - scheme.equilibrium(rho2, q2, p)
    assert np.allclose(neq_after, neq_before, atol=1e-14)


def test_projection_is_zero_mean():
    rng = np.random.default_rng(3)
    y = rng.standard_normal((3, 8, 8))
    d_rho, d_q = closure.net_output_to_dw(y, {"s_drho": 1e-3, "s_dq": 0.1})
    assert abs(d_rho.sum()) < 1e-12 and np.all(np.abs(d_q.sum(axis=(1, 2))) < 1e-12)


def test_guard_trips_on_corrupted_network_and_falls_back_exactly():
    """Weights multiplied by 1e6: every correction must be rejected and the run
    must equal the plain coarse scheme bit for bit."""
    f, p = _state(16, 4)
    params = cnn.init_params(5)
    params = [(w * 1e6, b) for w, b in params]
    scales = {"s_rho": 1e-3, "s_u": 1.0, "s_drho": 1e-4, "s_dq": 1e-2}
    g, acc, rej = closure.closure_run(f, p, params, scales, 12, every=4)
    assert acc == 0 and rej == 3
    assert np.array_equal(g, scheme.run(f, p, 12))


def test_guard_accepts_a_small_divergence_free_correction():
    f, p = _state(16, 5)
    rho, q = scheme.moments(f, p)
    n = rho.shape[0]
    # a small solenoidal momentum correction reduces nothing it should not
    d_q = 1e-3 * inputs.random_field_2d(n, 9, umax=1.0)
    ok, div0, div1 = closure.guard(rho, q, np.zeros_like(rho), d_q, p.dx)
    assert ok and math.isfinite(div1)


def _spectral_div(u):
    n = u.shape[-1]
    k = np.fft.fftfreq(n, 1.0 / n)
    return np.fft.ifft2(1j * k[None, :] * np.fft.fft2(u[0]) + 1j * k[:, None] * np.fft.fft2(u[1])).real


@pytest.mark.parametrize("n", [8, 15, 64])
def test_solenoidal_projection_properties(n):
    """The Helmholtz projection keeps divergence-free fields, removes gradient
    fields, is idempotent and leaves a field of zero spectral divergence; the
    mean is kept.  Fields from a stream function and a potential sampled at
    cell centres (exact trigonometric sums, so exactly solenoidal / irrotational
    on the grid)."""
    x = (np.arange(n) + 0.5) * 2 * np.pi / n
    X, Y = np.meshgrid(x, x)
    rng = np.random.default_rng(n)
    psi_x, psi_y = np.zeros((n, n)), np.zeros((n, n))
    phi_x, phi_y = np.zeros((n, n)), np.zeros((n, n))
    for kx in range(-2, 3):
        for ky in range(-2, 3):
            a, b = rng.normal(size=2)
            # psi = a sin(kx x + ky y), phi = b cos(kx x + ky y)
            arg = kx * X + ky * Y
            psi_x += a * ky * np.cos(arg)      # u = (d_y psi, -d_x psi)
            psi_y += -a * kx * np.cos(arg)
            phi_x += -b * kx * np.sin(arg)     # grad phi
            phi_y += -b * ky * np.sin(arg)
    sol = np.stack([psi_x, psi_y]) + np.array([0.3, -0.2])[:, None, None]
    grad = np.stack([phi_x, phi_y])
    scale = np.max(np.abs(sol))
    assert np.max(np.abs(closure.solenoidal(sol) - sol)) <= 1e-13 * scale
    assert np.max(np.abs(closure.solenoidal(grad))) <= 1e-13 * np.max(np.abs(grad))
    mixed = sol + grad
    p = closure.solenoidal(mixed)
    assert np.max(np.abs(p - sol)) <= 1e-13 * scale
    assert np.max(np.abs(closure.solenoidal(p) - p)) <= 1e-13 * scale
    assert np.max(np.abs(_spectral_div(p))) <= 1e-12 * scale * n
    # a random field without content at the Nyquist frequency (n even), where
    # numpy's signed frequency -n/2 pairs a mode with itself
    r = rng.normal(size=(2, n, n))
    if n % 2 == 0:
        rh = np.fft.fft2(r)
        rh[:, n // 2, :] = 0.0
        rh[:, :, n // 2] = 0.0
        r = np.fft.ifft2(rh).real
    pr = closure.solenoidal(r)
    assert np.allclose(pr.mean(axis=(1, 2)), r.mean(axis=(1, 2)), atol=1e-14)
    assert np.max(np.abs(_spectral_div(pr))) <= 1e-12 * n


def test_projected_target_keeps_density_and_adds_projection():
    n = 16
    rng = np.random.default_rng(3)
    now = rng.normal(size=(3, n, n))
    fine = now + 1e-3 * rng.normal(size=(3, n, n))
    t = closure.projected_target(fine, now)
    assert np.array_equal(t[0], now[0])
    assert np.allclose(t[1:] - now[1:], closure.solenoidal(fine[1:] - now[1:]), atol=1e-16)
