"""Parity of the HIP engine (through the C ABI) with the FP64 oracle.

Bar: plain FP32 storage must stay within relative L2 1e-5 of the oracle on
the velocity after up to 1000 steps; the FP64 diagnostics must agree with the
oracle's definitions evaluated on the same moments to ~1e-12.
"""

import math

import numpy as np
import pytest

import inputs
from oracle import diagnostics as odiag
from oracle import scheme

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_24059_amd import lbm  # noqa: E402

FP32_TOL = 1e-5


def _engine(p: scheme.Params, u0, rho0=None, storage="f32"):
    shape = u0.shape[1:]
    n = tuple(reversed(shape))
    prm = lbm.make_params(p.dim, n, p.dx, p.dt, p.nu, p.omega_rho, p.omega_q, p.alpha_rho,
                          storage=storage)
    return lbm.Engine.create(prm, u0, rho0)


def _rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _compare(p, u0, steps, rho0=None, tol=FP32_TOL, storage="f32"):
    print(f"[gpu parity] dim={p.dim} shape={u0.shape[1:]} steps={steps} storage={storage}", flush=True)
    eng = _engine(p, u0, rho0, storage=storage)
    eng.step(steps)
    rho, q = eng.moments()
    eng.close()
    r_ref, q_ref, _ = scheme.simulate(u0, p, steps, rho0)
    u, u_ref = q / rho, q_ref / r_ref
    err = _rel_l2(u, u_ref)
    cell = float(np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)))
    print(f"[gpu parity] rel-L2(u) = {err:.3e}, max cell |du| / max |u| = {cell:.3e}", flush=True)
    assert err <= tol, err
    # cell by cell as well: one wrong cell cannot hide inside the global norm
    assert cell <= 10 * tol, cell
    assert np.max(np.abs(rho - r_ref)) <= 1e-5
    return err


def test_taylor_green_64_1000_steps():
    """64^2 Taylor-Green, nu = 0.01, mu = 8, 1000 steps (the oracle-sized case)."""
    n = 64
    p = scheme.params_for_grid(2, n, 0.01)
    _compare(p, inputs.taylor_green(n), 1000)


def test_random_field_256_1000_steps():
    """The benchmark field (k^-3, Mach 0.05, nu = 1e-3) at 256^2 for 1000 steps."""
    n = 256
    p = scheme.params_for_grid(2, n, 1e-3)
    _compare(p, inputs.random_field_2d(n, 0, umax=0.05 / p.dx), 1000)


def test_raw_fp32_storage_runs_close():
    """LBM_F32_RAW (populations themselves in FP32) on the same case: correct to
    FP32 precision, but its large constant parts make it the less accurate mode."""
    n = 64
    p = scheme.params_for_grid(2, n, 0.01)
    u0 = inputs.taylor_green(n)
    eng = _engine(p, u0, storage="f32_raw")
    eng.step(1000)
    rho, q = eng.moments()
    eng.close()
    r_ref, q_ref, _ = scheme.simulate(u0, p, 1000)
    err = _rel_l2(q / rho, q_ref / r_ref)
    print(f"[gpu parity] f32_raw rel-L2(u) = {err:.3e}", flush=True)
    assert err <= 5e-5


FP64_TOL = 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_fp64_storage_matches_oracle_to_rounding(dim):
    """LBM_F64 (deviations in FP64, FP64 arithmetic) agrees with the FP64 oracle
    to accumulated FP64 rounding after 1000 steps (2D) / 200 steps (3D)."""
    if dim == 2:
        n, steps = 96, 1000
        p = scheme.params_for_grid(2, n, 1e-3)
        u0 = inputs.random_field_2d(n, 4, umax=0.05 / p.dx)
    else:
        n, steps = 24, 200
        p = scheme.params_for_grid(3, n, 1e-2)
        u0 = inputs.abc_flow(n)
    print(f"[gpu parity] f64 dim={dim} n={n} steps={steps}", flush=True)
    eng = _engine(p, u0, storage="f64")
    eng.step(steps)
    rho, q = eng.moments()
    with pytest.raises(lbm.LbmError):
        eng.set_fusion(2)   # one step per launch in the FP64 mode
    eng.close()
    r_ref, q_ref, _ = scheme.simulate(u0, p, steps)
    err = _rel_l2(q / rho, q_ref / r_ref)
    print(f"[gpu parity] f64 rel-L2(u) = {err:.3e}", flush=True)
    assert err <= FP64_TOL, err
    assert np.max(np.abs(rho - r_ref)) <= 1e-13


@pytest.mark.parametrize("storage", ["f32", "f16_neq"])
@pytest.mark.parametrize("shape", [(8, 8), (75, 75), (40, 96), (3, 130), (129, 1)])
def test_random_field_2d_ragged(shape, storage):
    """Non power-of-two and ragged grids: wrap-around and partial blocks."""
    ny, nx = shape
    dx = 2 * math.pi / max(nx, ny)
    p = scheme.Params(dim=2, dx=dx, dt=dx * dx / 8, nu=0.02)
    u = inputs.random_field_box(shape, dx, seed=3, umax=0.05 / dx)
    rho0 = 1 + 1e-3 * inputs.random_field_box(shape, dx, seed=4)[0]  # smooth density bump
    _compare(p, u, 300, rho0, storage=storage)


def test_zero_steps_is_the_equilibrium():
    n = 32
    p = scheme.params_for_grid(2, n, 0.01)
    u0 = inputs.random_field_2d(n, 0, umax=0.05 / p.dx)
    eng = _engine(p, u0)
    rho, q = eng.moments()
    eng.close()
    assert np.max(np.abs(rho - 1)) <= 1e-6
    assert _rel_l2(q, u0) <= 1e-6


@pytest.mark.parametrize("storage", ["f32", "f16_neq"])
@pytest.mark.parametrize("shape,steps", [((16, 16, 16), 200), ((10, 12, 14), 100), ((32, 32, 32), 100)])
def test_random_field_3d(shape, steps, storage):
    dx = 2 * math.pi / max(shape)
    p = scheme.Params(dim=3, dx=dx, dt=dx * dx / 8, nu=0.02)
    if len(set(shape)) == 1:
        u = inputs.random_field_3d(shape[0], seed=5, umax=0.05 / dx)
    else:
        u = inputs.random_field_box(shape, dx, seed=5, umax=0.05 / dx)
    _compare(p, u, steps, storage=storage)


def test_abc_3d():
    n = 24
    p = scheme.params_for_grid(3, n, 0.05)
    u0 = inputs.abc_flow(n, 0.25, 0.25, 0.25)
    rho0 = inputs.well_prepared_density(inputs.abc_pressure(u0), p.dx)
    _compare(p, u0, 150, rho0)


@pytest.mark.parametrize("dim", [2, 3])
def test_diagnostics_match_definitions(dim):
    n = 48 if dim == 2 else 20
    p = scheme.params_for_grid(dim, n, 0.02)
    if dim == 2:
        u0 = inputs.random_field_2d(n, 2, umax=0.05 / p.dx)
    else:
        u0 = inputs.random_field_3d(n, 2, umax=0.05 / p.dx)
    eng = _engine(p, u0)
    eng.step(50)
    rho, q = eng.moments()
    d = eng.diagnostics()
    eng.close()
    ref = odiag.from_moments(rho, q, p.dx)
    for key in ("mass", "kinetic", "enstrophy", "div_l2", "max_u", "rho_min", "rho_max"):
        assert d[key] == pytest.approx(ref[key], rel=1e-12, abs=1e-300), key
    for j in range(dim):
        assert d["mom"][j] == pytest.approx(ref["mom"][j], abs=1e-12 * ref["kinetic"])
    assert d["nonfinite"] == 0 and d["status"] == lbm.LBM_OK
    assert d["step"] == 50 and d["time"] == pytest.approx(50 * p.dt)


def test_mass_momentum_conserved_and_deterministic():
    n = 96
    p = scheme.params_for_grid(2, n, 0.01)
    u0 = inputs.random_field_2d(n, 4, umax=0.05 / p.dx)
    blobs = []
    for _ in range(2):
        eng = _engine(p, u0)
        d0 = eng.diagnostics()
        eng.step(500)
        d1 = eng.diagnostics()
        blobs.append(eng.save_state())
        eng.close()
        assert d1["mass"] == pytest.approx(d0["mass"], rel=1e-6)
    assert np.array_equal(blobs[0], blobs[1])


@pytest.mark.parametrize("storage", ["f32", "f16_neq"])
def test_save_load_continuation_is_bitwise(storage):
    """A snapshot continues bit for bit in a context created from another
    initial state (for the split storage the snapshot carries its scales)."""
    n = 40
    p = scheme.params_for_grid(2, n, 0.01)
    u0 = inputs.random_field_2d(n, 6, umax=0.05 / p.dx)
    a = _engine(p, u0, storage=storage)
    a.step(60)
    blob_full = None
    mid = a.save_state()
    a.step(60)
    blob_full = a.save_state()
    a.close()
    b = _engine(p, 3.0 * inputs.taylor_green(n), storage=storage)  # other initial state (and scales)
    b.load_state(mid)
    assert b.steps == 60
    b.step(60)
    assert np.array_equal(b.save_state(), blob_full)
    b.close()


def test_nonfinite_reported():
    n = 16
    p = scheme.params_for_grid(2, n, 0.01)
    u0 = inputs.taylor_green(n)
    eng = _engine(p, u0)
    blob = eng.save_state()
    f = blob[:-8].view(np.float32)
    f[5] = np.nan          # rho rest plane, cell 5
    f[n * n + 7] = np.inf  # q_x rest plane (the snapshot holds cells x planes, no padding), cell 7
    eng.load_state(blob)
    d = eng.diagnostics()
    eng.close()
    assert d["status"] == lbm.LBM_ENONFINITE and d["nonfinite"] == 2


def test_invalid_workspace_rejected():
    n = 16
    p = scheme.params_for_grid(2, n, 0.01)
    prm = lbm.make_params(2, (n, n), p.dx, p.dt, p.nu)
    nb = lbm.lbm_workspace_bytes(prm)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_init(prm, inputs.taylor_green(n), None, ws.data_ptr(), nb - 256,
                     torch.cuda.current_stream().cuda_stream)
    assert e.value.status == lbm.LBM_ENOMEM


# --------------------------------------------------------------------------- #
# full-size cases, in the launch configuration the benchmark times            #
# --------------------------------------------------------------------------- #

def _patch_reference(u0_full, p, centre, steps):
    """Oracle value at `centre` after `steps` steps, from a periodic patch of
    side 2*steps + 2 around it: information moves at most one cell per step,
    so the wrapped patch edges cannot reach the centre in time."""
    dim = p.dim
    half = steps + 1
    idx = [np.arange(c - half, c + half) % s for c, s in zip(centre, u0_full.shape[1:])]
    patch = u0_full[(slice(None),) + np.ix_(*idx)]
    rho, q, _ = scheme.simulate(np.ascontiguousarray(patch), p, steps)
    mid = (half,) * dim
    return rho[mid], q[(slice(None),) + mid]


def test_full_size_2d_4096_sampled():
    """4096^2, nu = 1e-3, k^-3 field at Mach 0.05, 64 steps: sampled cells
    against the oracle on domain-of-dependence patches."""
    n, steps = 4096, 64
    p = scheme.params_for_grid(2, n, 1e-3)
    u0 = inputs.random_field_2d(n, 0, umax=0.05 / p.dx)
    eng = _engine(p, u0)
    eng.step(steps)
    rho, q = eng.moments()
    d = eng.diagnostics()
    eng.close()
    assert d["nonfinite"] == 0
    rng = np.random.default_rng(0)
    for centre in [(0, 0), (n - 1, 17), (2048, 4095)] + [tuple(rng.integers(0, n, 2)) for _ in range(3)]:
        r_ref, q_ref = _patch_reference(u0, p, centre, steps)
        assert abs(rho[centre] - r_ref) <= 1e-6
        assert np.max(np.abs(q[(slice(None),) + centre] - q_ref)) <= 1e-5 * 0.05 / p.dx


def test_full_size_3d_256_sampled():
    n, steps = 256, 16
    p = scheme.params_for_grid(3, n, 1e-3)
    u0 = inputs.random_field_3d(n, 0, umax=0.05 / p.dx)
    eng = _engine(p, u0)
    eng.step(steps)
    rho, q = eng.moments()
    eng.close()
    rng = np.random.default_rng(1)
    for centre in [(0, 0, 0), (255, 3, 128)] + [tuple(rng.integers(0, n, 3)) for _ in range(2)]:
        r_ref, q_ref = _patch_reference(u0, p, centre, steps)
        assert abs(rho[centre] - r_ref) <= 1e-6
        assert np.max(np.abs(q[(slice(None),) + centre] - q_ref)) <= 1e-5 * 0.05 / p.dx


# --------------------------------------------------------------------------- #
# two steps per launch (2D): bit-identical to single-step launches            #
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("storage", ["f32", "f16_dev", "bf16_dev", "f16_dev_r32", "f32_raw", "f16_neq"])
@pytest.mark.parametrize("shape,steps", [((64, 64), 10), ((75, 75), 11), ((9, 130), 7), ((200, 3), 8),
                                         ((1, 1), 4), ((300, 257), 5)])
def test_two_step_fusion_is_bitwise(storage, shape, steps):
    ny, nx = shape
    dx = 2 * math.pi / max(shape)
    p = scheme.Params(dim=2, dx=dx, dt=dx * dx / 8, nu=0.02)
    u = inputs.random_field_box(shape, dx, seed=11, umax=0.05 / dx)
    blobs = []
    for fuse in (1, 2):
        eng = _engine(p, u, storage=storage)
        eng.set_fusion(fuse)
        eng.step(steps)
        blobs.append(eng.save_state())
        eng.close()
    assert np.array_equal(blobs[0], blobs[1])


@pytest.mark.parametrize("storage", ["f32", "f32_raw"])
def test_two_step_fusion_bitwise_large_tile(storage):
    """From 2^23 cells on, the two-step kernel runs 256x8 tiles on 1024
    threads for 4-byte planes: a 2900^2 grid (ragged against both tile
    edges), 5 steps."""
    import hashlib
    n = 2900
    p = scheme.params_for_grid(2, n, 1e-3)
    u = inputs.random_field_2d(n, 2, umax=0.05 / p.dx)
    digests = []
    for fuse in (1, 2):
        eng = _engine(p, u, storage=storage)
        eng.set_fusion(fuse)
        eng.step(5)
        digests.append(hashlib.sha256(eng.save_state().tobytes()).hexdigest())
        eng.close()
    assert digests[0] == digests[1]


# --------------------------------------------------------------------------- #
# 3 .. 6 steps per launch (2D population storages): bit-identical as well     #
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("storage", ["f32", "f16_dev", "bf16_dev", "f16_dev_r32", "bf16_dev_r32", "f32_raw",
                                     "f16_neq"])
@pytest.mark.parametrize("shape,steps", [((64, 64), 13), ((75, 75), 17), ((17, 130), 11), ((3, 200), 9),
                                         ((1, 1), 7), ((300, 257), 12)])
def test_deep_fusion_is_bitwise(storage, shape, steps):
    """Every fusion depth gives the single-step state; the step counts leave
    remainders that run as two-step and single-step launches."""
    ny, nx = shape
    dx = 2 * math.pi / max(shape)
    p = scheme.Params(dim=2, dx=dx, dt=dx * dx / 8, nu=0.02)
    u = inputs.random_field_box(shape, dx, seed=13, umax=0.05 / dx)
    blobs = []
    for fuse in (1, 3, 4, 5, 6):
        eng = _engine(p, u, storage=storage)
        eng.set_fusion(fuse)
        assert eng.fusion() == fuse
        eng.step(steps)
        assert eng.steps == steps
        blobs.append(eng.save_state())
        eng.close()
    for b in blobs[1:]:
        assert np.array_equal(blobs[0], b)


@pytest.mark.parametrize("storage", ["f32", "f16_dev", "bf16_dev", "f16_dev_r32", "bf16_dev_r32", "f16_neq"])
def test_deep_fusion_bitwise_large_grid(storage):
    """The default depth from 2^20 cells on (6 steps per launch for FP32 and
    the 16-bit storages with FP32 rest planes, 5 for the all-16-bit and split
    storages) on a 2900^2 grid, ragged against the tile edges, 23 steps."""
    import hashlib
    n = 2900
    p = scheme.params_for_grid(2, n, 1e-3)
    u = inputs.random_field_2d(n, 2, umax=0.05 / p.dx)
    digests = []
    for fuse in (1, None):
        eng = _engine(p, u, storage=storage)
        if fuse is not None:
            eng.set_fusion(fuse)
        else:
            assert eng.fusion() == (6 if storage in ("f32", "f16_dev_r32", "bf16_dev_r32") else 5)
        eng.step(23)
        digests.append(hashlib.sha256(eng.save_state().tobytes()).hexdigest())
        eng.close()
    assert digests[0] == digests[1]


def test_fusion_settings_and_defaults():
    small = scheme.params_for_grid(2, 64, 0.01)
    u = inputs.random_field_box((64, 64), small.dx, seed=3, umax=0.05 / small.dx)
    eng = _engine(small, u)
    assert eng.fusion() == 2                     # below 2^20 cells: two steps per launch
    for bad in (0, 7, -1):
        with pytest.raises(lbm.LbmError):
            eng.set_fusion(bad)
    eng.set_fusion(6)
    assert eng.fusion() == 6
    eng.close()
    neq = _engine(small, u, storage="f16_neq")
    assert neq.fusion() == 2
    neq.set_fusion(3)
    with pytest.raises(lbm.LbmError):
        neq.set_fusion(7)
    neq.close()
    f64 = _engine(small, u, storage="f64")
    assert f64.fusion() == 1
    for bad in (2, 3):
        with pytest.raises(lbm.LbmError):
            f64.set_fusion(bad)
    f64.close()
    big = scheme.params_for_grid(2, 1024, 1e-3)
    u_big = inputs.random_field_2d(1024, 0, umax=0.05 / big.dx)
    for storage, depth in (("f32", 6), ("f32_raw", 6), ("f16_dev_r32", 6), ("bf16_dev_r32", 6), ("bf16_dev", 5),
                           ("f16_dev", 5), ("f16_neq", 5)):
        eng = _engine(big, u_big, storage=storage)
        assert eng.fusion() == depth, storage
        eng.close()
    p3 = scheme.params_for_grid(3, 8, 0.01)
    e3 = _engine(p3, inputs.abc_flow(8, 0.1, 0.1, 0.1))
    assert e3.fusion() == 1                      # 3D: too few column tiles to fuse
    e3.set_fusion(3)
    with pytest.raises(lbm.LbmError):
        e3.set_fusion(4)
    e3.close()


@pytest.mark.parametrize("storage", ["f32", "f32_raw", "f16_dev", "bf16_dev", "f16_dev_r32", "bf16_dev_r32"])
@pytest.mark.parametrize("shape,steps", [((8, 8, 8), 6), ((17, 13, 9), 7), ((40, 20, 33), 5), ((1, 1, 1), 4),
                                         ((3, 70, 5), 9), ((64, 64, 64), 3), ((70, 9, 66), 4), ((33, 7, 130), 8)])
def test_multi_step_fusion_3d_is_bitwise(storage, shape, steps):
    """3D population storages: the z-marching two-step kernel (64 x 8
    columns, 32-plane segments) and three-step kernel (64 x 8 columns,
    segments of 8 planes on these grids) give
    the single-step state bit for bit, ragged in every direction, over several
    segments along z, and with remainders that run as shorter launches."""
    nz, ny, nx = shape
    dx = 2 * math.pi / max(shape)
    p = scheme.Params(dim=3, dx=dx, dt=dx * dx / 8, nu=0.02)
    u = inputs.random_field_box(shape, dx, seed=5, umax=0.05 / dx)
    blobs = []
    for fuse in (1, 2, 3):
        eng = _engine(p, u, storage=storage)
        eng.set_fusion(fuse)
        eng.step(steps)
        blobs.append(eng.save_state())
        eng.close()
    assert np.array_equal(blobs[0], blobs[1])
    assert np.array_equal(blobs[0], blobs[2])


def test_two_step_fusion_3d_defaults_and_limits():
    """3D defaults: the z-marching kernels only where their launch has at
    least 128 blocks (64^3: 64 blocks, one step per launch; 128^3: 256 blocks,
    three steps per launch)."""
    for n, expect in ((64, 1), (128, 3)):
        pn = scheme.params_for_grid(3, n, 0.01)
        for storage in ("f32", "f16_dev_r32"):
            e = _engine(pn, np.zeros((3, n, n, n)), storage=storage)
            assert e.fusion() == expect, (n, storage)
            e.close()
    p = scheme.params_for_grid(3, 8, 0.01)
    u = inputs.abc_flow(8, 0.1, 0.1, 0.1)
    eng = _engine(p, u)
    assert eng.fusion() == 1
    eng.set_fusion(2)
    assert eng.fusion() == 2
    for bad in (4, 5, 7):
        with pytest.raises(lbm.LbmError):
            eng.set_fusion(bad)
    eng.close()
    for storage in ("f16_neq", "f64"):
        e = _engine(p, u, storage=storage)
        assert e.fusion() == 1
        with pytest.raises(lbm.LbmError):
            e.set_fusion(2)
        e.close()
    for storage in ("f16_dev", "f16_dev_r32"):
        e = _engine(p, u, storage=storage)
        assert e.fusion() == 1
        e.set_fusion(2)
        e.set_fusion(3)
        with pytest.raises(lbm.LbmError):
            e.set_fusion(4)
        e.close()
