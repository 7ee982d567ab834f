"""Batched linear spectra on the GPU (include/lbm_spectrum.h) against the
oracle's amplification matrix (Section 4) and the closed forms that pin it.

* E(theta): element by element against oracle.spectrum.amplification_matrix
  (|difference| <= 1e-13; the two build it from the same formulas in other
  units, so they differ by rounding only).
* Eigenvalues: against LAPACK's (numpy) eigenvalues of the oracle's matrix,
  paired one to one; each pair within 64 eps ||E|| kappa + 1e-13, kappa the
  eigenvalue's condition number from the left and right eigenvectors (both
  solvers are backward stable, so their results differ by at most about
  that).  Points where an eigenvalue is too ill-conditioned for such a bound
  are covered by the closed forms instead.
* Lemma 1 (checkerboard theta = (pi, pi)), the omega = 1 reduction to a
  (d+1) x (d+1) matrix, and the low-frequency expansion of Lemma 2 and its
  threshold in mu, on the GPU's own eigenvalues.
"""

import math

import numpy as np
import pytest
import scipy.linalg
from scipy.optimize import linear_sum_assignment

from oracle import spectrum as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_24059_amd import spectrum as S  # noqa: E402

EPS = np.finfo(float).eps


def _random_points(dim, count, seed, omega_one=False):
    rng = np.random.default_rng(seed)
    states, params, thetas = [], [], []
    for _ in range(count):
        w_rho, w_q = (1.0, 1.0) if omega_one else rng.uniform(0.05, 1.95, 2)
        a_rho, a_q = rng.uniform(0.0, 1.0 / (2 * dim), 2)
        dx = 10.0 ** rng.uniform(-6, -1)
        mu = rng.uniform(1, 20)
        rho_bar = rng.uniform(0.5, 2.0)
        q_bar = rng.uniform(-1, 1, dim)
        gamma = rng.choice([1.0, 1.4])
        dp = gamma * rho_bar ** (gamma - 1.0)
        states.append(S.make_state(mu, dx, w_rho, w_q, a_rho, a_q, rho_bar, q_bar, dp))
        params.append((dx, mu, w_rho, w_q, a_rho, a_q, rho_bar, q_bar, gamma))
        thetas.append(rng.uniform(-math.pi, math.pi, dim))
    return states, params, np.array(thetas)


def _oracle_matrix(dim, prm, theta):
    dx, mu, w_rho, w_q, a_rho, a_q, rho_bar, q_bar, gamma = prm
    return O.amplification_matrix(theta, dim, dx, mu, w_rho, w_q, a_rho, a_q, rho_bar, q_bar, gamma)


def _pair(a, b):
    C = np.abs(np.asarray(a)[:, None] - np.asarray(b)[None, :])
    r, c = linear_sum_assignment(C)
    return r, c, C[r, c]


@pytest.mark.parametrize("dim", [2, 3])
def test_matrix_matches_oracle(dim):
    states, params, thetas = _random_points(dim, 40, 10 + dim)
    idx = np.arange(len(states), dtype=np.int32)
    E = S.matrix(dim, states, thetas, idx)
    n = S.lbm_spectrum_order(dim)
    assert E.shape == (len(states), n, n)
    for p, prm in enumerate(params):
        ref = _oracle_matrix(dim, prm, thetas[p])
        assert np.max(np.abs(E[p] - ref)) <= 1e-13, p


@pytest.mark.parametrize("dim", [2, 3])
def test_eigenvalues_match_lapack(dim):
    states, params, thetas = _random_points(dim, 60, 20 + dim)
    out = S.eigenvalues(dim, states, thetas, np.arange(len(states), dtype=np.int32))
    assert np.all(out["info"] >= 0)
    checked = 0
    for p, prm in enumerate(params):
        E = _oracle_matrix(dim, prm, thetas[p])
        w, vl, vr = scipy.linalg.eig(E, left=True, right=True)
        kappa = np.linalg.norm(vl, axis=0) * np.linalg.norm(vr, axis=0) / np.abs(np.sum(vl.conj() * vr, axis=0))
        r, c, d = _pair(w, out["eig"][p])
        tol = 64 * EPS * np.linalg.norm(E, 2) * kappa[r] + 1e-13
        if np.max(kappa) > 1e8:
            continue
        assert np.all(d <= tol), (p, d.max(), tol[np.argmax(d - tol)])
        assert out["radius"][p] == pytest.approx(np.max(np.abs(out["eig"][p])), rel=1e-15)
        checked += 1
    assert checked >= 50
    print(f"[spectrum] {dim}D: {checked} points within the perturbation bound; "
          f"sweeps {out['info'].mean():.1f} mean, flops {out['flops'].mean():.3g} mean", flush=True)


@pytest.mark.parametrize("dim", [2, 3])
def test_checkerboard_lemma1(dim):
    """Lemma 1: at theta = (pi, .., pi) the eigenvalues are omega_i - 1
    (2d - 1 times per set) and the roots of z^2 - omega_i (1 - 4 d alpha_i) z + omega_i - 1."""
    states, params, _ = _random_points(dim, 24, 30 + dim)
    th = np.full((len(states), dim), math.pi)
    out = S.eigenvalues(dim, states, th, np.arange(len(states), dtype=np.int32))
    for p, prm in enumerate(params):
        _, _, w_rho, w_q, a_rho, a_q, *_ = prm
        want = O.checkerboard_eigenvalues(dim, [w_rho] + [w_q] * dim, [a_rho] + [a_q] * dim)
        _, _, d = _pair(want, out["eig"][p])
        assert d.max() <= 1e-7, (p, d.max())       # multiple roots: sqrt(eps) sensitivity


@pytest.mark.parametrize("dim", [2, 3])
def test_relaxation_scheme_reduction(dim):
    """omega = 1 about (1, 0): n - (d+1) zero eigenvalues, the others those of
    the (d+1) x (d+1) matrix of W(t+1, x) = sum_l f^eq_l(W(t, x - c_l))."""
    rng = np.random.default_rng(40 + dim)
    mu, a_rho, a_q = 8.0, 0.075, 0.01
    thetas = rng.uniform(-math.pi, math.pi, (32, dim))
    st = S.make_state(mu, 1e-3, 1.0, 1.0, a_rho, a_q)
    out = S.eigenvalues(dim, [st], thetas)
    n = S.lbm_spectrum_order(dim)
    for p in range(len(thetas)):
        ev = out["eig"][p]
        order = np.argsort(np.abs(ev))
        zeros, big = ev[order[: n - dim - 1]], ev[order[n - dim - 1:]]
        assert np.max(np.abs(zeros)) <= 1e-12
        A = O.relaxation_scheme_matrix(thetas[p], dim, mu, a_rho, a_q)
        _, _, d = _pair(big, np.linalg.eigvals(A))
        assert d.max() <= 1e-12


def test_lemma2_expansion_and_threshold_fig1_setting():
    """Fig. 1 setting (omega = 1, alpha_rho = 1/4, nu = pi/50, alpha_q = nu/mu,
    reference (1, 1, 1), dx = 1e-6): on the diagonal theta = (tau, tau) the
    acoustic pair is 1 +- i sqrt(2) tau/mu - (alpha_rho + alpha_q) tau^2
    + O(tau^3), and the diagonal is stable for mu above
    -2 nu + sqrt(4 nu^2 + 4) = 1.8783 and unstable below it."""
    nu = math.pi / 50
    mus = np.array([1.80, 1.87, 1.89, 2.0, 8.0])
    taus = np.concatenate([np.linspace(-math.pi, math.pi, 2001), np.geomspace(1e-4, 0.5, 100), [1e-3, 2e-3]])
    states = [S.make_state(mu, 1e-6, 1.0, 1.0, 0.25, nu / mu, 1.0, (1.0, 1.0)) for mu in mus]
    idx = np.repeat(np.arange(len(mus), dtype=np.int32), len(taus))
    th = np.tile(np.stack([taus, taus], axis=1), (len(mus), 1))
    out = S.eigenvalues(2, states, th, idx)
    assert np.all(out["info"] >= 0)
    rad = out["radius"].reshape(len(mus), len(taus)).max(axis=1)
    print(f"[spectrum] Fig. 1 diagonal radius by mu: {dict(zip(mus.tolist(), rad.tolist()))}", flush=True)
    assert rad[0] > 1 + 1e-3 and rad[1] > 1 + 1e-5
    assert np.all(rad[2:] <= 1 + 1e-12)
    eig = out["eig"].reshape(len(mus), len(taus), -1)
    for m, mu in enumerate(mus[3:], start=3):
        for k, tau in ((len(taus) - 2, 1e-3), (len(taus) - 1, 2e-3)):
            ev = eig[m, k]
            z = ev[np.argmin(np.abs(ev - (1 + 1j * math.sqrt(2) * tau / mu)))]
            assert z.imag / tau == pytest.approx(math.sqrt(2) / mu, rel=1e-5)
            assert (1 - z.real) / tau ** 2 == pytest.approx(0.25 + nu / mu, rel=1e-4)


def test_state_index_errors_and_empty():
    st = S.make_state(8.0, 1e-3, 1.2, 1.15, 0.075, 0.01)
    th = np.array([[0.3, 0.2], [0.1, -0.4], [1.0, 1.0]])
    out = S.eigenvalues(2, [st], th, np.array([0, 5, -1], dtype=np.int32))
    assert out["info"].tolist()[1:] == [-2, -2] and out["info"][0] >= 0
    assert np.all(np.isnan(out["eig"][1:])) and np.all(np.isnan(out["radius"][1:]))
    assert np.isfinite(out["radius"][0])
    E = S.matrix(2, [st], th, np.array([0, 1, 0], dtype=np.int32))
    assert np.all(np.isnan(E[1])) and np.all(np.isfinite(E[[0, 2]]))
    empty = S.eigenvalues(2, [st], np.zeros((0, 2)))
    assert empty["eig"].shape == (0, 15)


def test_large_batch_sampled_parity():
    """The benchmark's launch: a (mu, theta) map of the Fig. 1 setting in 2D
    (64 mu x 4096 diagonal theta) and a general-omega 3D map (16 states x
    4096 theta); sampled points against LAPACK on the oracle's matrix."""
    nu = math.pi / 50
    mus = np.linspace(0.5, 16.0, 64)
    taus = np.linspace(-math.pi, math.pi, 4096)
    states = [S.make_state(mu, 1e-6, 1.0, 1.0, 0.25, nu / mu, 1.0, (1.0, 1.0)) for mu in mus]
    idx = np.repeat(np.arange(len(mus), dtype=np.int32), len(taus))
    th = np.tile(np.stack([taus, taus], axis=1), (len(mus), 1))
    out = S.eigenvalues(2, states, th, idx)
    assert np.all(out["info"] >= 0)
    rng = np.random.default_rng(5)
    for p in rng.choice(len(idx), 40, replace=False):
        mu = mus[idx[p]]
        E = O.amplification_matrix(th[p], 2, 1e-6, mu, 1.0, 1.0, 0.25, nu / mu, 1.0, np.array([1.0, 1.0]))
        assert abs(out["radius"][p] - np.max(np.abs(np.linalg.eigvals(E)))) <= 1e-10
    states3, params3, _ = _random_points(3, 16, 77)
    th3 = np.random.default_rng(6).uniform(-math.pi, math.pi, (16 * 4096, 3))
    idx3 = np.repeat(np.arange(16, dtype=np.int32), 4096)
    out3 = S.eigenvalues(3, states3, th3, idx3)
    assert np.all(out3["info"] >= 0)
    for p in rng.choice(len(idx3), 20, replace=False):
        E = _oracle_matrix(3, params3[idx3[p]], th3[p])
        w, vl, vr = scipy.linalg.eig(E, left=True, right=True)
        kappa = np.linalg.norm(vl, axis=0) * np.linalg.norm(vr, axis=0) / np.abs(np.sum(vl.conj() * vr, axis=0))
        r, c, d = _pair(w, out3["eig"][p])
        if np.max(kappa) <= 1e8:
            assert np.all(d <= 64 * EPS * np.linalg.norm(E, 2) * kappa[r] + 1e-13)
