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
