"""The seeded input fields: divergence-free, resolution-independent, and the
spectral pressure solves the pressure Poisson equation."""

import numpy as np

import inputs


def _spectral_div(u):
    n = u.shape[-1]
    k = np.fft.fftfreq(n, 1 / n)
    return np.fft.ifft2(1j * k[None, :] * np.fft.fft2(u[0]) + 1j * k[:, None] * np.fft.fft2(u[1])).real


def test_random_field_is_divergence_free_and_scaled():
    u = inputs.random_field_2d(256, 7, umax=2.0)
    assert np.abs(_spectral_div(u)).max() < 1e-10
    assert abs(np.sqrt((u ** 2).sum(0)).max() - 2.0) < 1e-12      # normalised on the 256^2 grid


def test_random_field_is_the_same_continuous_field_at_every_resolution():
    a = inputs.random_field_2d(64, 3)
    b = inputs.random_field_2d(192, 3)
    assert np.allclose(a, b[:, 1::3, 1::3], atol=1e-12)          # cell centres coincide


def test_taylor_green_pressure_closed_form():
    c, k = inputs.pressure_coefficients(inputs.taylor_green(16))
    assert np.abs(inputs.pressure_at(c, k, 40) - inputs.taylor_green_pressure(40)).max() < 1e-13


def test_random_pressure_solves_poisson():
    n = 128
    u = inputs.random_field_2d(n, 5)
    phi = inputs.random_pressure_2d(n, 5)
    k = np.fft.fftfreq(n, 1 / n)
    kx, ky = k[None, :], k[:, None]
    F = np.fft.fft2
    lap = np.fft.ifft2(-(kx ** 2 + ky ** 2) * F(phi)).real
    dd = np.fft.ifft2(-(kx * kx * F(u[0] * u[0]) + 2 * kx * ky * F(u[0] * u[1]) + ky * ky * F(u[1] * u[1]))).real
    assert np.abs(lap + dd).max() < 1e-9 * np.abs(dd).max()
    assert abs(phi.mean()) < 1e-12


def test_batch_specs_deterministic():
    a = inputs.batch_run_specs(16)
    b = inputs.batch_run_specs(16)
    assert a == b and all(s["n"] in inputs.fields.BATCH_SIZES for s in a)
    assert all(1e-4 <= s["nu"] <= 1e-2 for s in a)
