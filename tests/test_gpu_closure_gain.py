"""What the trained correction network gains over the scheme without it.

The network shipped in paper_2607_24059_amd/closure_weights.npz (trained on
seeds 0..199, 64 pairs each, 25 epochs, by `python -m
paper_2607_24059_amd.closure`; the file's metadata records the configuration)
corrects a 256^2 run
every 4 steps; the reference is the plain scheme at 2048^2 in FP64 storage,
restricted to 256^2.  On held-out seeds the corrected run must beat the plain
256^2 run by at least 2x on the divergence-free velocity error after 256
coarse steps, must not be worse on the full velocity error, and must reach
the plain scheme's resolution-limited error of a resolution between 512^2
and 1024^2 faster than the plain FP32 run at that resolution.
"""

import math

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2607_24059_amd import closure as cl  # noqa: E402
from paper_2607_24059_amd import cnn  # noqa: E402

HELD_OUT = [1010, 1011]


def test_trained_network_beats_plain_coarse():
    params, meta = cl.load_model(cl.WEIGHTS)
    cfg = cl.Config(**{k: v for k, v in meta["config"].items()
                       if k in ("coarse_n", "factor", "nu", "mach", "mu", "every", "guard", "horizon")})
    assert not set(HELD_OUT) & set(meta["config"]["train_seeds"])
    net = cnn.Net(params=params)
    print(f"[gain] seeds {HELD_OUT}, coarse {cfg.coarse_n}^2, reference FP64 {cfg.fine_n}^2", flush=True)
    ev = cl.evaluate(cfg, net, meta["scales"], seeds=HELD_OUT, levels=(256, 512, 1024), plain_storages=("f32", "f64"),
                     log=lambda *a: print(*a, flush=True))
    ps = ev["per_seed"]
    for i, seed in enumerate(HELD_OUT):
        plain, corr = ps["plain_coarse_u_sol"][i], ps["closure_u_sol"][i]
        print(f"[gain] seed {seed}: plain {plain:.3e} corrected {corr:.3e} gain {plain / corr:.2f}x", flush=True)
        assert corr <= 0.5 * plain
        assert ps["closure_u"][i] <= ps["plain_coarse_u"][i]
    assert ev["closure"]["rejected"] == 0
    # equal error on the scheme's resolution-limited error (the FP64 plain
    # levels, which converge at second order) with the FP32 run times
    sp = ev["speedup_equal_error"]["u_sol"]["closure_resolution_limited"]
    print(f"[gain] equal-error speedup over plain FP32: {sp}", flush=True)
    assert math.isfinite(sp["N_star"]) and 512 < sp["N_star"] < 1024 and sp["speedup"] > 1
