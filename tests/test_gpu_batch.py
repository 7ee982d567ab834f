"""Batched engine: every run of a batch must be bit-identical to the same run
advanced alone by the single-run engine (same per-cell device code), and the
autotuner must not change the state."""

import math
import os

import numpy as np
import pytest

import inputs
from oracle import scheme

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_24059_amd import batch as B  # noqa: E402
from paper_2607_24059_amd import lbm  # noqa: E402


def _mixed_runs(dim=2):
    """Uneven sizes (incl. ragged and non-square) and viscosities."""
    rng = np.random.default_rng(42)
    shapes = [(64, 64), (128, 128), (75, 75), (256, 256), (40, 96), (8, 8), (130, 3), (512, 512)]
    if dim == 3:
        shapes = [(16, 16, 16), (12, 10, 8), (32, 32, 32), (5, 40, 20)]
    runs, u0s = [], []
    for i, shp in enumerate(shapes):
        dx = 2 * math.pi / max(shp)
        nu = float(10 ** rng.uniform(-4, -2))
        dt = dx * dx / 8
        runs.append(B.make_run(tuple(reversed(shp)), dx, dt, nu))
        u0s.append(inputs.random_field_box(shp, dx, seed=i, umax=0.05 / dx))
    return runs, u0s


def _single(dim, storage, run, u0, steps):
    prm = lbm.make_params(dim, tuple(run.n)[:dim], run.dx, run.dt, run.nu, run.omega_rho,
                          run.omega_q, run.alpha_rho, rho_ref=run.rho_ref, storage=storage)
    eng = lbm.Engine.create(prm, u0)
    eng.step(steps)
    out = eng.moments()
    eng.close()
    return out


@pytest.mark.parametrize("fuse", [5, 2, 1])
@pytest.mark.parametrize("storage,steps", [("f32", 73), ("f16_dev_r32", 120), ("bf16_dev", 51), ("f16_dev", 8),
                                           ("bf16_dev_r32", 17), ("f32_raw", 126)])
def test_batch_bitwise_equals_single_runs_2d(storage, steps, fuse):
    """Every kernel (five steps per launch, the 2D default for batches of
    small runs, two or one) gives each run's single-run state bit for bit; the
    step counts end on shorter launches (73 = 14 x 5 + 2 + 1) or use the
    graphs of 24 launches (120, 126)."""
    runs, u0s = _mixed_runs(2)
    print(f"[batch] 2D {storage} {len(runs)} runs {steps} steps fuse={fuse}", flush=True)
    b = B.Batch.create(2, storage, runs, u0s)
    assert b.fusion() == 5
    assert b.fused_grid() > 0
    b.set_fusion(fuse)
    assert b.fusion() == fuse
    b.step(steps)
    cells, tiles, done = b.info()
    assert done == steps
    assert cells == sum(int(r.n[0] * r.n[1]) for r in runs)
    for r, (run, u0) in enumerate(zip(runs, u0s)):
        rho, q = b.moments(r)
        rho1, q1 = _single(2, storage, run, u0, steps)
        assert np.array_equal(rho, rho1) and np.array_equal(q, q1), r
    b.close()


@pytest.mark.parametrize("storage", ["f32", "f16_dev_r32", "bf16_dev"])
@pytest.mark.parametrize("shape", [0, 1, 2])
def test_every_fused_tile_shape_is_bitwise(storage, shape):
    """Each of the three five-step tile shapes the autotuner chooses from
    gives the single-run states bit for bit (ragged, tiny and non-square runs;
    52 = 10 x 5 + 2 steps)."""
    runs, u0s = _mixed_runs(2)
    b = B.Batch.create(2, storage, runs, u0s)
    b.set_fused_shape(shape)
    tiles = {b.fused_tile(r) for r in range(len(runs))}
    assert len(tiles) == 1
    expect = {"f32": [(32, 32), (32, 16), (16, 16)]}.get(storage, [(64, 16), (32, 32), (32, 16)])[shape]
    assert tiles == {expect}
    print(f"[batch] {storage} fused tile {expect}", flush=True)
    b.step(52)
    for r, (run, u0) in enumerate(zip(runs, u0s)):
        rho, q = b.moments(r)
        rho1, q1 = _single(2, storage, run, u0, 52)
        assert np.array_equal(rho, rho1) and np.array_equal(q, q1), r
    with pytest.raises(lbm.LbmError):
        b.set_fused_shape(3)
    b.close()


@pytest.mark.parametrize("per_cu", [0, 1, 3])
def test_every_fused_grid_is_bitwise(per_cu):
    """The five-step launches give the single-run states bit for bit with one
    block per tile (0) and with persistent grids of 1 and 3 blocks per compute
    unit (each block then walks several tiles); 27 = 5 x 5 + 2 steps."""
    runs, u0s = _mixed_runs(2)
    b = B.Batch.create(2, "f32", runs, u0s)
    b.set_fused_grid(per_cu)
    print(f"[batch] f32 fused grid {per_cu} per CU: {b.fused_grid()} blocks", flush=True)
    tiles_k = sum(-(-int(r.n[0]) // b.fused_tile(i)[0]) * -(-int(r.n[1]) // b.fused_tile(i)[1])
                  for i, r in enumerate(runs))
    assert b.fused_grid() <= tiles_k if per_cu else b.fused_grid() == tiles_k
    b.step(27)
    for r, (run, u0) in enumerate(zip(runs, u0s)):
        rho, q = b.moments(r)
        rho1, q1 = _single(2, "f32", run, u0, 27)
        assert np.array_equal(rho, rho1) and np.array_equal(q, q1), r
    for bad in (-1, 65):
        with pytest.raises(lbm.LbmError):
            b.set_fused_grid(bad)
    b.close()


@pytest.mark.parametrize("storage,depth", [("f32", 6), ("f32_raw", 6), ("f16_dev_r32", 5)])
def test_batch_depth_follows_run_sizes(storage, depth):
    """A batch whose cells are mostly in runs of at least 2^20 cells (one
    1024^2 run beside small ones) runs six steps per launch in the 4-byte
    storages (32x28 tiles for the large run), five in the 16-bit ones; bit for
    bit the single runs after 151 = 24 x 6 + 6 + 1 steps, and only 1, 2 and
    that depth are accepted."""
    shapes = [(1024, 1024), (64, 64), (75, 75), (130, 3)]
    runs, u0s = [], []
    for i, (ny, nx) in enumerate(shapes):
        dx = 2 * math.pi / max(nx, ny)
        runs.append(B.make_run((nx, ny), dx, dx * dx / 8, 0.01 * (1 + i)))
        u0s.append(inputs.random_field_box((ny, nx), dx, seed=40 + i, umax=0.05 / dx))
    print(f"[batch] depth {storage}", flush=True)
    b = B.Batch.create(2, storage, runs, u0s)
    assert b.fusion() == depth
    assert b.fused_tile(0) == ((32, 28) if depth == 6 else (64, 16))
    for bad in (3, 4, 11 - depth, 7):
        with pytest.raises(lbm.LbmError):
            b.set_fusion(bad)
    b.set_fusion(depth)
    b.step(151)
    for r, (run, u0) in enumerate(zip(runs, u0s)):
        rho, q = b.moments(r)
        rho1, q1 = _single(2, storage, run, u0, 151)
        assert np.array_equal(rho, rho1) and np.array_equal(q, q1), r
    b.close()


def test_batch_bitwise_equals_single_runs_3d():
    runs, u0s = _mixed_runs(3)
    b = B.Batch.create(3, "f32", runs, u0s)
    assert b.fused_grid() == 0 and b.fusion() == 1
    for bad in (2, 5, 3, 0):
        with pytest.raises(lbm.LbmError):
            b.set_fusion(bad)
    with pytest.raises(lbm.LbmError):
        b.set_fused_grid(0)
    b.step(37)
    for r, (run, u0) in enumerate(zip(runs, u0s)):
        rho, q = b.moments(r)
        rho1, q1 = _single(3, "f32", run, u0, 37)
        assert np.array_equal(rho, rho1) and np.array_equal(q, q1), r
    b.close()


def test_switching_fusion_mid_run_is_bitwise():
    """Alternating one-, two- and five-step launches (buffer parity changes)
    keeps the single-run states."""
    runs, u0s = _mixed_runs(2)
    b = B.Batch.create(2, "f32", runs, u0s)
    for bad in (3, 4, 6):
        with pytest.raises(lbm.LbmError):
            b.set_fusion(bad)
    total = 0
    for fuse, n in ((2, 5), (5, 7), (1, 3), (2, 50), (5, 121), (1, 1), (5, 10), (2, 2)):
        b.set_fusion(fuse)
        b.step(n)
        total += n
    for r in (0, 2, 5, 7):
        rho, q = b.moments(r)
        rho1, q1 = _single(2, "f32", runs[r], u0s[r], total)
        assert np.array_equal(rho, rho1) and np.array_equal(q, q1), r
    b.close()


def test_batch_matches_oracle():
    n = 64
    p = scheme.params_for_grid(2, n, 0.01)
    u0 = inputs.taylor_green(n)
    run = B.make_run((n, n), p.dx, p.dt, p.nu)
    b = B.Batch.create(2, "f32", [run, run], [u0, 0.5 * u0])
    b.step(200)
    rho, q = b.moments(0)
    b.close()
    r_ref, q_ref, _ = scheme.simulate(u0, p, 200)
    err = np.linalg.norm(q / rho - q_ref / r_ref) / np.linalg.norm(q_ref / r_ref)
    assert err <= 1e-5, err


def test_autotune_keeps_state_and_caches(tmp_path):
    runs, u0s = _mixed_runs(2)
    b = B.Batch.create(2, "f32", runs, u0s)
    b.step(10)
    before = [b.moments(r) for r in range(len(runs))]
    cache = str(tmp_path / "tune.txt")
    b.autotune(cache)
    for r in range(len(runs)):
        rho, q = b.moments(r)
        assert np.array_equal(rho, before[r][0]) and np.array_equal(q, before[r][1])
        w = b.tile_width(r)
        assert w in (64, 128, 256)
        assert b.fused_tile(r) in ((32, 32), (32, 16), (16, 16))
    assert os.path.exists(cache) and open(cache).read().strip()
    lines_first = open(cache).read()
    assert b.fused_grid() > 0
    b.step(25)
    for r in (0, 3, 7):
        rho, q = b.moments(r)
        rho1, q1 = _single(2, "f32", runs[r], u0s[r], 35)
        assert np.array_equal(rho, rho1) and np.array_equal(q, q1), r
    b.close()
    # a second batch reads the cache and appends nothing new
    b2 = B.Batch.create(2, "f32", runs, u0s)
    b2.autotune(cache)
    assert open(cache).read() == lines_first
    b2.close()


def test_invalid_run_reported():
    runs, u0s = _mixed_runs(2)
    bad = B.make_run((64, 64), 0.1, 0.1 ** 2 / 8, 0.01, omega_q=2.5)
    with pytest.raises(lbm.LbmError) as e:
        B.Batch.create(2, "f32", runs[:2] + [bad], u0s[:2] + [u0s[0]])
    assert e.value.status == lbm.LBM_EUNSTABLE and "run 2" in str(e.value)


def test_full_batch_workload_sampled():
    """The 512-run workload (sizes 64^2..1024^2, nu log-uniform; most cells in
    the 1024^2 runs, so six steps per launch in FP32): a few steps, then
    sampled runs against the single-run engine, bitwise."""
    specs = inputs.batch_run_specs(512)
    runs, u0s = [], []
    for s in specs:
        n = s["n"]
        dx = 2 * math.pi / n
        runs.append(B.make_run((n, n), dx, dx * dx / 8, s["nu"]))
        u0s.append(inputs.random_field_2d(n, s["seed"], umax=0.05 / dx))
    b = B.Batch.create(2, "f32", runs, u0s)
    assert b.fusion() == 6
    b.autotune(None)
    b.step(23)
    for r in (0, 1, 255, 511) + tuple(i for i, s in enumerate(specs) if s["n"] == 1024)[:1]:
        rho, q = b.moments(r)
        rho1, q1 = _single(2, "f32", runs[r], u0s[r], 23)
        assert np.array_equal(rho, rho1) and np.array_equal(q, q1), r
    b.close()
