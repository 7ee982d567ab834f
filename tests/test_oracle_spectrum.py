"""Pins from Section 4 (linearised spectra) and its exact special cases.

The amplification matrix E(theta) is assembled from a hand-written Jacobian of
the equilibria (oracle.spectrum), independently of oracle.scheme; it is tied
to the paper by the checkerboard determinant of Lemma 1 and to the oracle by
evolving a small Fourier mode.
"""

import math

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import scheme, spectrum


def _match(a, b):
    """Largest distance of the best one-to-one pairing of two eigenvalue sets."""
    C = np.abs(np.asarray(a)[:, None] - np.asarray(b)[None, :])
    r, c = linear_sum_assignment(C)
    return C[r, c].max()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("trial", range(4))
def test_checkerboard_determinant(dim, trial):
    """Lemma 1: at theta = (pi, pi) the spectrum is that of
    prod_i (z - omega_i + 1)^3 (z^2 - omega_i (1 - 8 alpha_i) z + omega_i - 1),
    for any reference state (3D: exponent 5, coefficient 1 - 12 alpha)."""
    rng = np.random.default_rng(100 * dim + trial)
    w_rho, w_q = rng.uniform(0.05, 1.95, 2)
    a_rho, a_q = rng.uniform(0.0, 1.0 / (2 * dim), 2)
    dx = 10.0 ** rng.uniform(-6, -1)
    mu = rng.uniform(1, 20)
    rho_bar = rng.uniform(0.5, 2.0)
    q_bar = rng.uniform(-1, 1, dim)
    E = spectrum.amplification_matrix(np.full(dim, math.pi), dim, dx, mu, w_rho, w_q,
                                      a_rho, a_q, rho_bar, q_bar)
    expected = spectrum.checkerboard_eigenvalues(dim, [w_rho] + [w_q] * dim,
                                                 [a_rho] + [a_q] * dim)
    assert _match(np.linalg.eigvals(E), expected) <= 1e-7  # multiple roots: sqrt(eps) sensitivity


def test_checkerboard_stability_region():
    """Lemma 1: spectral radius <= 1 iff omega in [0, 2] and alpha in [0, 1/4]."""
    def radius(w, a):
        E = spectrum.amplification_matrix(np.array([math.pi, math.pi]), 2, 1e-6, 8.0,
                                          w, w, a, a)
        return np.max(np.abs(np.linalg.eigvals(E)))
    assert radius(1.5, 0.2) <= 1 + 1e-12
    assert radius(1.0, 0.25) <= 1 + 1e-12
    assert radius(1.5, 0.3) > 1 + 1e-3
    assert radius(2.2, 0.1) > 1 + 1e-3


@pytest.mark.parametrize("theta", [(0.3, 0.0), (0.7, -1.1), (2.0, 2.5), (math.pi, 0.4)])
def test_relaxation_scheme_spectrum(theta):
    """omega = 1: E = S J M has rank 3, and its non-zero eigenvalues are those of
    the 3x3 map W(t+1, x) = sum_l f^eq_l(W(t, x - c_l)) linearised about (1, 0, 0)."""
    mu, a_rho, a_q, dx = 8.0, 0.075, 0.01, 1e-3
    E = spectrum.amplification_matrix(np.array(theta), 2, dx, mu, 1.0, 1.0, a_rho, a_q)
    ev = np.linalg.eigvals(E)
    big = ev[np.abs(ev) > 1e-9]
    assert np.sum(np.abs(ev) <= 1e-9) == 12
    A = spectrum.relaxation_scheme_matrix(np.array(theta), 2, mu, a_rho, a_q)
    assert _match(big, np.linalg.eigvals(A)) <= 1e-12


def test_relaxation_scheme_acoustic_modulus():
    """Along x the acoustic pair has |z|^2 = (1 - 2 a_rho c)(1 - 2 a_q c) + sin^2(theta)/mu^2."""
    mu, a_rho, a_q = 8.0, 0.075, 0.01
    for th in (0.1, 0.5, 1.3):
        A = spectrum.relaxation_scheme_matrix(np.array([th, 0.0]), 2, mu, a_rho, a_q)
        ev = np.linalg.eigvals(A)
        c = 1 - math.cos(th)
        shear = 1 - 2 * a_q * c
        ac = np.delete(ev, np.argmin(np.abs(ev - shear)))
        want = (1 - 2 * a_rho * c) * (1 - 2 * a_q * c) + math.sin(th) ** 2 / mu ** 2
        assert np.allclose(np.abs(ac) ** 2, want, rtol=1e-12)


@pytest.mark.parametrize("omega_q", [0.8, 1.15, 1.6])
def test_small_theta_shear_decay_and_sound_speed(omega_q):
    """Small theta, reference (1, 0): the shear mode decays by
    1 - 2 alpha_q (1/omega_q - 1/2) theta^2 per step (the viscosity of Section 3,
    nu dt / dx^2 = nu / mu) and the acoustic pair rotates by +-theta/mu per step
    (sound speed 1/dx in physical units, Section 4)."""
    mu, a_rho, a_q, w_rho, dx = 8.0, 0.075, 0.01, 1.2, 1e-6
    th = 1e-3
    E = spectrum.amplification_matrix(np.array([th, 0.0]), 2, dx, mu, w_rho, omega_q,
                                      a_rho, a_q)
    ev = np.linalg.eigvals(E)
    near1 = ev[np.abs(ev - 1) < 0.05]
    assert len(near1) == 3
    shear_pred = 1 - 2 * a_q * (1 / omega_q - 0.5) * th ** 2
    k = np.argmin(np.abs(near1 - shear_pred))
    assert abs(near1[k] - shear_pred) <= 1e-3 * th ** 2 * a_q + 1e-12
    ac = np.delete(near1, k)
    assert np.allclose(np.sort(np.abs(np.angle(ac))), th / mu, rtol=1e-4)


def test_oracle_follows_the_amplification_matrix():
    """A 1e-7 Fourier perturbation of a uniform moving state, evolved by the
    nonlinear oracle, follows eps Re(E^n v e^{i theta . j}) to O(eps^2)."""
    rng = np.random.default_rng(11)
    n = 16
    p = scheme.Params(dim=2, dx=0.07, dt=0.07 ** 2 / 6.0, nu=0.03, omega_rho=1.35,
                      omega_q=1.2, alpha_rho=0.06)
    rho_bar, q_bar = 1.05, np.array([0.4, -0.25])
    k = np.array([3, 2])
    theta = 2 * math.pi * k / n
    v = rng.standard_normal(15) + 1j * rng.standard_normal(15)
    eps = 1e-7
    jx = np.arange(n)[None, :]
    jy = np.arange(n)[:, None]
    wave = np.exp(1j * (theta[0] * jx + theta[1] * jy))
    base = scheme.equilibrium(np.full((n, n), rho_bar),
                              np.stack([np.full((n, n), c) for c in q_bar]), p)
    f = base + eps * np.real(v.reshape(3, 5, 1, 1) * wave)
    E = spectrum.amplification_matrix(theta, 2, p.dx, p.mu, p.omega_rho, p.omega_q,
                                      p.alpha_rho, p.alpha_q, rho_bar, q_bar)
    steps = 40
    f = scheme.run(f, p, steps)
    vn = np.linalg.matrix_power(E, steps) @ v
    pred = base + eps * np.real(vn.reshape(3, 5, 1, 1) * wave)
    assert np.max(np.abs(f - pred)) <= 1e-5 * eps * np.max(np.abs(vn))


def _fig1_matrix(theta, mu, q_bar=(1.0, 1.0)):
    """The setting of Fig. 1: relaxation scheme (omega = 1), alpha_rho = 1/4,
    nu = pi/50, alpha_q = nu/mu, reference (1, 1, 1), dx = 1e-6."""
    nu = math.pi / 50
    return spectrum.amplification_matrix(np.asarray(theta, float), 2, 1e-6, mu, 1.0, 1.0, 0.25, nu / mu,
                                         1.0, np.array(q_bar))


@pytest.mark.parametrize("mu", [2.0, 8.0])
def test_low_frequency_acoustic_pair_on_the_diagonal(mu):
    """Lemma 2's expansion along theta = (tau, tau): the acoustic pair is
    1 +- i sqrt(2) tau/mu - c2 tau^2 + O(tau^3).  The 2x2 acoustic block of the
    omega = 1 map, [[1 - 2 a_rho c, -i sqrt(2) s/mu], [-i sqrt(2) s/mu, 1 - 2 a_q c]]
    with c = 2 (1 - cos tau), s = sin tau, gives c2 = a_rho + a_q: the damping of
    the longitudinal momentum (q_x + q_y)/sqrt(2) enters once (reading: the
    printed lemma sums a_rho + a_qx + a_qy)."""
    a_rho, a_q = 0.25, math.pi / 50 / mu
    for tau in (2e-3, 1e-3):
        ev = np.linalg.eigvals(_fig1_matrix([tau, tau], mu))
        z = ev[np.argmin(np.abs(ev - (1 + 1j * math.sqrt(2) * tau / mu)))]
        assert z.imag / tau == pytest.approx(math.sqrt(2) / mu, rel=1e-5)
        assert (1 - z.real) / tau ** 2 == pytest.approx(a_rho + a_q, rel=1e-4)
        assert abs((1 - z.real) / tau ** 2 - (a_rho + 2 * a_q)) > 0.5 * a_q


def test_stability_threshold_in_mu_on_the_diagonal():
    """|z|^2 = 1 - 2 (a_rho + a_q - 1/mu^2) tau^2 + O(tau^4) for the acoustic
    pair, so the low frequencies along the diagonal need mu^2 (a_rho + a_q) >= 1;
    with a_rho = 1/4 and a_q = nu/mu that is mu >= -2 nu + sqrt(4 nu^2 + 4)
    = 1.8783 (nu = pi/50).  The whole diagonal is stable just above it and
    unstable just below it; at mu = 1.80, above the printed bound's 1.7644, it
    is unstable, so that bound is necessary but not sufficient here."""
    nu = math.pi / 50
    mu_star = -2 * nu + math.sqrt(4 * nu * nu + 4)
    assert mu_star == pytest.approx(1.8782802469, rel=1e-9)
    ts = np.concatenate([np.linspace(-math.pi, math.pi, 401), np.geomspace(1e-4, 0.5, 60)])

    def radius(mu):
        return max(np.max(np.abs(np.linalg.eigvals(_fig1_matrix([t, t], mu)))) for t in ts)
    assert radius(1.87) > 1 + 1e-5
    assert radius(1.89) <= 1 + 1e-12
    assert radius(1.80) > 1 + 1e-3
