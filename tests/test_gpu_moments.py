"""Moment-only storage (LBM_F32_MOMENTS): the relaxation scheme omega = 1 on
every set, advanced as a stencil on the moments alone.

Parity: against the FP64 oracle of the full scheme (15 / 28 populations) run
with omega_rho = omega_q = 1, where every post-relaxation population is its
cell's equilibrium, so both compute the same W(t) up to rounding (relative L2
of u <= 1e-5 after 1000 steps in 2D); the multi-step kernels (2D: 2 to 6 steps per launch, 3D: two) are
bit-identical to single steps; and the population storage (LBM_F32) at
omega = 1 agrees to FP32 rounding.
"""

import math

import numpy as np
import pytest

import inputs
from oracle import scheme

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_24059_amd import lbm  # noqa: E402


def _params(dim, n, nu):
    dx = 2 * math.pi / n
    return scheme.Params(dim=dim, dx=dx, dt=dx * dx / 8, nu=nu, omega_rho=1.0, omega_q=1.0)


def _engine(p, u0, storage="f32_moments", rho0=None):
    n = tuple(reversed(u0.shape[1:]))
    prm = lbm.make_params(p.dim, n, p.dx, p.dt, p.nu, p.omega_rho, p.omega_q, p.alpha_rho, storage=storage)
    return lbm.Engine.create(prm, u0, rho0)


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("dim,n,steps", [(2, 256, 1000), (2, 75, 300), (3, 24, 200)])
def test_moments_match_full_oracle_at_omega_one(dim, n, steps):
    p = _params(dim, n, 1e-3 if dim == 2 else 1e-2)
    u0 = inputs.random_field_2d(n, 3, umax=0.05 / p.dx) if dim == 2 else inputs.random_field_3d(n, 3, umax=0.05 / p.dx)
    shape = u0.shape[1:]
    rho0 = 1 + 1e-3 * np.cos(np.arange(shape[-1]) * p.dx)[None] * np.ones(shape)
    print(f"[moments] dim={dim} n={n} steps={steps}", flush=True)
    eng = _engine(p, u0, rho0=rho0)
    eng.step(steps)
    rho, q = eng.moments()
    eng.close()
    r_ref, q_ref, _ = scheme.simulate(u0, p, steps, rho0)
    err = _rel(q / rho, q_ref / r_ref)
    print(f"[moments] rel-L2(u) = {err:.3e}", flush=True)
    assert err <= 1e-5
    assert np.max(np.abs(rho - r_ref)) <= 1e-6


@pytest.mark.parametrize("shape,steps", [((64, 64), 10), ((75, 75), 11), ((9, 130), 7), ((1, 1), 4), ((300, 600), 5),
                                         ((70, 33), 13), ((129, 257), 23)])
def test_moments_fusion_is_bitwise(shape, steps):
    """Every fusion depth (1 .. 6 steps per launch) gives the single-step state."""
    ny, nx = shape
    dx = 2 * math.pi / max(shape)
    p = scheme.Params(dim=2, dx=dx, dt=dx * dx / 8, nu=0.02, omega_rho=1.0, omega_q=1.0)
    u = inputs.random_field_box(shape, dx, seed=12, umax=0.05 / dx)
    blobs = []
    for fuse in (1, 2, 3, 4, 5, 6):
        eng = _engine(p, u)
        eng.set_fusion(fuse)
        eng.step(steps)
        blobs.append(eng.save_state())
        eng.close()
    for fuse, b in zip((2, 3, 4, 5, 6), blobs[1:]):
        assert np.array_equal(blobs[0], b), f"{fuse} steps per launch differ from single steps"


@pytest.mark.parametrize("shape,steps", [((40, 20, 33), 60), ((70, 9, 66), 40), ((10, 12, 14), 80), ((1, 1, 1), 5),
                                         ((3, 70, 5), 30), ((65, 17, 129), 12)])
def test_moments_3d_ragged_and_z_segments(shape, steps):
    """3D moment-only storage at its default fusion (one step per launch on
    these grids, by the cell-parallel kernel: the z-marching launches would
    have fewer than 128 blocks) against the full-population oracle at
    omega = 1 on grids ragged in every direction, tiny grids and a y extent
    below the tile."""
    nz, ny, nx = shape
    dx = 2 * math.pi / max(shape)
    p = scheme.Params(dim=3, dx=dx, dt=dx * dx / 8, nu=0.02, omega_rho=1.0, omega_q=1.0)
    u0 = inputs.random_field_box(shape, dx, seed=21, umax=0.05 / dx)
    rho0 = 1 + 1e-3 * inputs.random_field_box(shape, dx, seed=22)[0]
    print(f"[moments] 3D shape={shape} steps={steps}", flush=True)
    eng = _engine(p, u0, rho0=rho0)
    eng.step(steps)
    rho, q = eng.moments()
    eng.close()
    r_ref, q_ref, _ = scheme.simulate(u0, p, steps, rho0)
    err = _rel(q / rho, q_ref / r_ref)
    cell = float(np.max(np.abs(q / rho - q_ref / r_ref)) / np.max(np.abs(q_ref / r_ref)))
    print(f"[moments] rel-L2(u) = {err:.3e}, max cell {cell:.3e}", flush=True)
    assert err <= 1e-5 and cell <= 1e-4
    assert np.max(np.abs(rho - r_ref)) <= 1e-6


@pytest.mark.parametrize("shape,steps", [((40, 20, 33), 9), ((70, 9, 66), 8), ((10, 12, 14), 11), ((1, 1, 1), 5),
                                         ((3, 70, 5), 6), ((65, 17, 129), 7), ((33, 7, 130), 4), ((17, 13, 64), 10)])
def test_moments_3d_two_step_is_bitwise(shape, steps):
    """3D moment-only storage, two steps per launch (the z-marching kernel on
    64 x 11 column tiles, segments of at least 8 planes): the single-step state
    bit for bit on grids ragged in every direction, with several segments
    along z, tiny grids whose border wraps several times, and odd step counts
    (the last step runs alone)."""
    nz, ny, nx = shape
    dx = 2 * math.pi / max(shape)
    p = scheme.Params(dim=3, dx=dx, dt=dx * dx / 8, nu=0.02, omega_rho=1.0, omega_q=1.0)
    u = inputs.random_field_box(shape, dx, seed=23, umax=0.05 / dx)
    print(f"[moments] 3D two-step shape={shape} steps={steps}", flush=True)
    blobs = []
    for fuse in (1, 2):
        eng = _engine(p, u)
        eng.set_fusion(fuse)
        assert eng.fusion() == fuse
        eng.step(steps)
        blobs.append(eng.save_state())
        eng.close()
    assert np.array_equal(blobs[0], blobs[1])


def test_moments_3d_default_two_steps_large_grid():
    """A 3D grid whose two-step launch has enough blocks (130 x 200 x 96:
    3 x 19 column tiles, 12-plane segments, 456 blocks) runs two steps per
    launch by default, bit for bit the single-step state after 7 steps; three
    steps per launch are refused, and small grids keep one step per launch."""
    shape = (96, 200, 130)
    dx = 2 * math.pi / 200
    p = scheme.Params(dim=3, dx=dx, dt=dx * dx / 8, nu=1e-3, omega_rho=1.0, omega_q=1.0)
    u = inputs.random_field_box(shape, dx, seed=24, umax=0.05 / dx)
    blobs = []
    for fuse in (1, None):
        eng = _engine(p, u)
        if fuse is None:
            assert eng.fusion() == 2
            with pytest.raises(lbm.LbmError):
                eng.set_fusion(3)
        else:
            eng.set_fusion(fuse)
        eng.step(7)
        blobs.append(eng.save_state())
        eng.close()
    assert np.array_equal(blobs[0], blobs[1])
    small = _engine(p, inputs.random_field_box((24, 24, 24), dx, seed=25, umax=0.05 / dx))
    assert small.fusion() == 1
    small.close()


def test_moments_3d_z_marching_single_step_oracle():
    """The z-marching single step runs where its launch has at least 128
    blocks (smaller grids take the cell-parallel kernel): 130 x 260 x 100 is
    3 x 17 column tiles by 4 segments, ragged in every direction.  Against
    the full-population oracle at omega = 1 after 4 steps, and bit for bit
    the two-step kernel's state."""
    shape = (100, 260, 130)
    dx = 2 * math.pi / 260
    p = scheme.Params(dim=3, dx=dx, dt=dx * dx / 8, nu=0.02, omega_rho=1.0, omega_q=1.0)
    u0 = inputs.random_field_box(shape, dx, seed=26, umax=0.05 / dx)
    states = []
    for fuse in (1, 2):
        print(f"[moments] 3D {shape} fusion {fuse}", flush=True)
        eng = _engine(p, u0)
        eng.set_fusion(fuse)
        eng.step(4)
        states.append(eng.save_state())
        if fuse == 1:
            rho, q = eng.moments()
        eng.close()
    assert np.array_equal(states[0], states[1])
    r_ref, q_ref, _ = scheme.simulate(u0, p, 4)
    err = _rel(q / rho, q_ref / r_ref)
    cell = float(np.max(np.abs(q / rho - q_ref / r_ref)) / np.max(np.abs(q_ref / r_ref)))
    print(f"[moments] rel-L2(u) = {err:.3e}, max cell {cell:.3e}", flush=True)
    assert err <= 1e-5 and cell <= 1e-4
    assert np.max(np.abs(rho - r_ref)) <= 1e-6


def _patch_reference(u0_full, p, centre, steps):
    """Oracle value at `centre` after `steps` steps, from a periodic patch of
    side 2*steps + 2 around it (information moves one cell per step)."""
    half = steps + 1
    idx = [np.arange(c - half, c + half) % s for c, s in zip(centre, u0_full.shape[1:])]
    patch = u0_full[(slice(None),) + np.ix_(*idx)]
    rho, q, _ = scheme.simulate(np.ascontiguousarray(patch), p, steps)
    mid = (half,) * p.dim
    return rho[mid], q[(slice(None),) + mid]


def test_moments_3d_256_default_sampled():
    """256^3 at the default fusion (two steps per launch: the z-marching
    two-step kernel, 64 x 11 column tiles, one block per tile and segment):
    sampled cells against the full-population oracle at omega = 1 on
    domain-of-dependence patches."""
    n, steps = 256, 16
    p = _params(3, n, 1e-3)
    u0 = inputs.random_field_3d(n, 0, umax=0.05 / p.dx)
    eng = _engine(p, u0)
    assert eng.fusion() == 2
    eng.step(steps)
    rho, q = eng.moments()
    eng.close()
    rng = np.random.default_rng(2)
    for centre in [(0, 0, 0), (255, 3, 128), (17, 200, 63)] + [tuple(rng.integers(0, n, 3)) for _ in range(2)]:
        r_ref, q_ref = _patch_reference(u0, p, centre, steps)
        assert abs(rho[centre] - r_ref) <= 1e-6, centre
        assert np.max(np.abs(q[(slice(None),) + centre] - q_ref)) <= 1e-5 * 0.05 / p.dx, centre


def test_moments_default_fusion_large_grid_bitwise():
    """From 2^20 cells the moment-only storage runs four steps per launch by
    default: a 1100 x 1000 grid (ragged against the 64 x 32 tiles), 19 steps."""
    import hashlib
    p = scheme.Params(dim=2, dx=2 * math.pi / 1100, dt=(2 * math.pi / 1100) ** 2 / 8, nu=1e-3,
                      omega_rho=1.0, omega_q=1.0)
    u = inputs.random_field_box((1000, 1100), p.dx, seed=4, umax=0.05 / p.dx)
    digests = []
    for fuse in (1, None):
        eng = _engine(p, u)
        if fuse is None:
            assert eng.fusion() == 4
        else:
            eng.set_fusion(fuse)
        eng.step(19)
        digests.append(hashlib.sha256(eng.save_state().tobytes()).hexdigest())
        eng.close()
    assert digests[0] == digests[1]


def test_population_storage_agrees_at_omega_one():
    n = 128
    p = _params(2, n, 1e-3)
    u0 = inputs.random_field_2d(n, 5, umax=0.05 / p.dx)
    out = []
    for storage in ("f32_moments", "f32"):
        eng = _engine(p, u0, storage)
        eng.step(500)
        out.append(eng.moments())
        eng.close()
    err = _rel(out[0][1] / out[0][0], out[1][1] / out[1][0])
    print(f"[moments] moments vs populations rel-L2(u) = {err:.3e}", flush=True)
    assert err <= 5e-6


def test_moments_storage_requires_omega_one():
    p = scheme.params_for_grid(2, 16, 0.01)     # omega_q = 23/20
    with pytest.raises(lbm.LbmError):
        lbm.Engine.create(lbm.make_params(2, (16, 16), p.dx, p.dt, p.nu, storage="f32_moments"),
                          np.zeros((2, 16, 16)))
