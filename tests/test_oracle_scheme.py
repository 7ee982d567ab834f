"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a conservation law,
a symmetry, an independent implementation (scalar loops, push transport), a
closed form from the paper, or an exact solution of the Navier-Stokes system.
"""

import math

import numpy as np
import pytest

import inputs
from oracle import brute, diagnostics, scheme

PI = math.pi


def _random_state(p, shape, rng, noise=1e-3):
    """f^eq of random moments near (1, +-0.05/dx) plus a non-equilibrium part."""
    d = p.dim
    rho = 1.0 + 0.02 * rng.standard_normal(shape)
    q = 0.05 / p.dx * rng.uniform(-1, 1, (d,) + shape)
    f = scheme.equilibrium(rho, q, p)
    return f + noise * rng.standard_normal(f.shape)


# --------------------------------------------------------------------------- #
# 1. independent scalar-loop implementation                                   #
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("dim,shape,steps", [(2, (8, 8), 20), (2, (6, 5), 7), (3, (4, 4, 4), 5),
                                             (3, (3, 4, 5), 3)])
def test_brute_force_matches(dim, shape, steps):
    rng = np.random.default_rng(7 + dim)
    p = scheme.Params(dim=dim, dx=0.2, dt=0.2 ** 2 / 8.0, nu=0.013, omega_rho=1.3,
                      omega_q=1.1, alpha_rho=0.07)
    f = _random_state(p, shape, rng)
    b = brute.from_array(f)
    nested_shape = brute.to_nested_shape(f)
    for _ in range(steps):
        f = scheme.step(f, p)
        b = brute.step(b, nested_shape, p.dx, p.dt, p.nu, p.omega_rho, p.omega_q, p.alpha_rho)
    fb = np.array(b).reshape(f.shape)
    assert np.max(np.abs(fb - f)) <= 1e-14 * np.max(np.abs(f))


# --------------------------------------------------------------------------- #
# 2. conservation                                                             #
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_has_the_moments(dim):
    """sum_l f^eq_l(rho, q) = (rho, dx q): holds only with dx on the rest q-component."""
    rng = np.random.default_rng(3)
    p = scheme.Params(dim=dim, dx=0.05, dt=0.05 ** 2 / 8, nu=0.01)
    shape = (5,) * dim
    rho = 1 + 0.1 * rng.standard_normal(shape)
    q = rng.standard_normal((dim,) + shape)
    feq = scheme.equilibrium(rho, q, p)
    r2, q2 = scheme.moments(feq, p)
    assert np.allclose(r2, rho, rtol=0, atol=1e-14)
    assert np.allclose(q2, q, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_relaxation_conserves_moments_and_fixes_equilibrium(dim):
    rng = np.random.default_rng(4)
    p = scheme.Params(dim=dim, dx=0.05, dt=0.05 ** 2 / 8, nu=0.01, omega_rho=1.5, omega_q=0.7)
    shape = (6,) * dim
    f = _random_state(p, shape, rng, noise=1e-2)
    fs = scheme.relax(f, p)
    r0, q0 = scheme.moments(f, p)
    r1, q1 = scheme.moments(fs, p)
    scale = np.max(np.abs(f))
    assert np.max(np.abs(r1 - r0)) <= 8 * np.finfo(float).eps * scale
    assert np.max(np.abs(q1 - q0)) * p.dx <= 8 * np.finfo(float).eps * scale
    feq = scheme.equilibrium(r0, q0, p)
    assert np.max(np.abs(scheme.relax(feq, p) - feq)) <= 4 * np.finfo(float).eps * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_transport_is_a_permutation(dim):
    rng = np.random.default_rng(5)
    shape = (7, 6, 5)[:dim]
    fs = rng.standard_normal((dim + 1, 2 * dim + 1) + shape)
    out = scheme.transport(fs, dim)
    for i in range(dim + 1):
        for l in range(2 * dim + 1):
            assert np.array_equal(np.sort(out[i, l].ravel()), np.sort(fs[i, l].ravel()))
    # direction: f_{+x}(x) = f*_{+x}(x - dx)
    assert np.array_equal(out[0, 1][..., 3], fs[0, 1][..., 2])
    assert np.array_equal(out[0, 2][..., 2], fs[0, 2][..., 3])


def test_global_sums_conserved_1000_steps():
    """Taylor-Green 64^2, nu = 0.01, 1000 steps: mass and momentum are invariants."""
    n = 64
    p = scheme.params_for_grid(2, n, 0.01)
    f = scheme.init(np.ones((n, n)), inputs.taylor_green(n), p)
    d0 = diagnostics.of_state(f, p)
    f = scheme.run(f, p, 1000)
    d1 = diagnostics.of_state(f, p)
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["mass"]
    for j in range(2):
        assert abs(d1["mom"][j] - d0["mom"][j]) <= 1e-12 * d0["max_u"] * (2 * PI) ** 2


# --------------------------------------------------------------------------- #
# 3. symmetries                                                               #
# --------------------------------------------------------------------------- #

def test_translation_equivariance_is_exact():
    rng = np.random.default_rng(6)
    p = scheme.Params(dim=2, dx=0.1, dt=0.1 ** 2 / 8, nu=0.02)
    f = _random_state(p, (9, 10), rng)
    a = scheme.run(np.roll(f, (2, -3), axis=(2, 3)), p, 5)
    b = np.roll(scheme.run(f, p, 5), (2, -3), axis=(2, 3))
    assert np.array_equal(a, b)


def _transpose_xy(f):
    """Swap the x and y axes: grid transpose, sets q_x <-> q_y, velocities +-x <-> +-y."""
    g = np.swapaxes(f, 2, 3).copy()
    g = g[[0, 2, 1]]
    return g[:, [0, 3, 4, 1, 2]]


def _reflect_x(f):
    """x -> -x: cell i -> n-1-i, +x <-> -x, q_x -> -q_x."""
    g = f[..., ::-1].copy()
    g = g[:, [0, 2, 1, 3, 4]]
    g[1] = -g[1]
    return g


def test_transpose_and_reflection_equivariance():
    rng = np.random.default_rng(8)
    p = scheme.Params(dim=2, dx=0.1, dt=0.1 ** 2 / 8, nu=0.02, omega_q=1.4)
    f = _random_state(p, (8, 8), rng)
    ref = scheme.run(f, p, 6)
    for op in (_transpose_xy, _reflect_x):
        got = scheme.run(op(f), p, 6)
        assert np.max(np.abs(got - op(ref))) <= 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_uniform_state_is_steady(dim):
    p = scheme.Params(dim=dim, dx=0.1, dt=0.1 ** 2 / 8, nu=0.02)
    shape = (4,) * dim
    rho = np.full(shape, 1.1)
    q = np.stack([np.full(shape, 0.3 * (j + 1)) for j in range(dim)])
    f = scheme.equilibrium(rho, q, p)
    g = scheme.run(f, p, 10)
    assert np.max(np.abs(g - f)) <= 1e-15


def test_3d_reduces_to_2d_for_z_invariant_flow():
    """z-invariant data with q_z = 0: the +-z populations never move and, with
    the rest population, act as the 2D rest population of weight 1 - 4 alpha."""
    rng = np.random.default_rng(9)
    p2 = scheme.Params(dim=2, dx=0.1, dt=0.1 ** 2 / 8, nu=0.02, omega_q=1.3)
    p3 = scheme.Params(dim=3, dx=0.1, dt=0.1 ** 2 / 8, nu=0.02, omega_q=1.3)
    rho = 1 + 0.01 * rng.standard_normal((8, 8))
    u = 0.3 * rng.standard_normal((2, 8, 8))
    f2 = scheme.run(scheme.init(rho, u, p2), p2, 12)
    rho3 = np.broadcast_to(rho, (3, 8, 8)).copy()
    u3 = np.zeros((3, 3, 8, 8))
    u3[0] = u[0]
    u3[1] = u[1]
    f3 = scheme.run(scheme.init(rho3, u3, p3), p3, 12)
    r2, q2 = scheme.moments(f2, p2)
    r3, q3 = scheme.moments(f3, p3)
    for z in range(3):
        assert np.max(np.abs(r3[z] - r2)) <= 1e-13
        assert np.max(np.abs(q3[:2, z] - q2)) <= 1e-12
        assert np.max(np.abs(q3[2, z])) <= 1e-12


# --------------------------------------------------------------------------- #
# 4. parameters                                                               #
# --------------------------------------------------------------------------- #

def test_viscosity_relation_and_validation():
    p = scheme.params_for_grid(2, 64, 0.01)
    assert p.mu == pytest.approx(8.0)
    # nu = 2 mu alpha_q (1/omega_q - 1/2) (end of Section 3)
    assert 2 * p.mu * p.alpha_q * (1 / p.omega_q - 0.5) == pytest.approx(0.01, rel=1e-15)
    p.validate()
    for bad in (dict(omega_q=2.0), dict(omega_rho=0.0), dict(alpha_rho=0.3),
                dict(alpha_rho=-0.01)):
        with pytest.raises(ValueError):
            scheme.Params(dim=2, dx=0.1, dt=0.01, nu=0.01, **bad).validate()
    with pytest.raises(ValueError):  # 3D alpha bound is 1/6
        scheme.Params(dim=3, dx=0.1, dt=0.01, nu=0.01, alpha_rho=0.2).validate()
