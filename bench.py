#!/usr/bin/env python3
"""Throughput of the fused relax-and-transport step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-variants] [--no-cpu]

Workload (the headline line): 2D vectorial D2Q5, 4096 x 4096 periodic grid on
[0, 2pi)^2, nu = 1e-3, mu = dx^2/dt = 8, seeded divergence-free random field
(|k|^-3 amplitudes, 1 <= |k| <= 16) scaled to Mach dx*max|u| = 0.05, FP32
storage and arithmetic, 2000 steps.  Inputs are resident in HBM before the
timed region; a launch of the fused kernel advances the grid by two steps.

Printed: one JSON line on stdout with MLUPS, the HBM roofline of the step
kernel (algorithmic bytes / measured average launch time, against the 8 TB/s
published peak and against the measured copy-probe bandwidth), and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0                 # MI355X published HBM3E bandwidth
METRIC = "MLUPS & % HBM peak; fp16-store / learned closure vs plain fp32 at fixed error"
BYTES_PER_LUP = {("f32", 2): 120, ("f16_dev", 2): 60, ("bf16_dev", 2): 60, ("f16_dev_r32", 2): 72,
                 ("bf16_dev_r32", 2): 72, ("f32_raw", 2): 120, ("f32", 3): 224, ("f16_dev", 3): 112, ("bf16_dev", 3): 112,
                 ("f16_dev_r32", 3): 128, ("bf16_dev_r32", 3): 128, ("f16_neq", 2): 72, ("f16_neq", 3): 128}
KERNEL_SOURCES = ("paper_2607_24059_amd/csrc/lbm_kernels.hip", "paper_2607_24059_amd/csrc/lbm_device.hpp",
                  "paper_2607_24059_amd/csrc/lbm_fused.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stepK_2d_f32_4096_traffic.json")
VARIANT_WARMUP = 50   # untimed steps before each variant's timed steps (clocks settle)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_workload(n: int, dim: int, nu: float, seed: int = 0, mach: float = 0.05):
    import inputs
    from paper_2607_24059_amd import lbm
    dx = 2 * math.pi / n
    dt = dx * dx / 8.0
    if dim == 2:
        u0 = inputs.random_field_2d(n, seed, umax=mach / dx)
    else:
        u0 = inputs.random_field_3d(n, seed, umax=mach / dx)
    return u0, dx, dt, lbm


def time_engine(n, dim, storage, steps, warmup, nu=1e-3, u0=None, fuse=None):
    """Run `warmup` untimed steps then `steps` timed steps; returns (ms per step, engine).
    fuse: time steps per launch (None = the library default)."""
    import torch
    from paper_2607_24059_amd import lbm
    dx = 2 * math.pi / n
    dt = dx * dx / 8.0
    if u0 is None:
        u0, *_ = make_workload(n, dim, nu)
    grid = (n,) * dim
    prm = lbm.make_params(dim, grid, dx, dt, nu, storage=storage)
    eng = lbm.Engine.create(prm, u0)
    if fuse is not None:
        eng.set_fusion(fuse)
    eng.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(eng.stream)
    eng.step(steps)
    ev1.record(eng.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / max(steps, 1)
    return ms, eng


def copy_probe_gbs(nbytes: int = 1 << 30, reps: int = 20) -> float:
    """Read + write bandwidth of the library's copy kernel on a 1 GiB buffer."""
    import torch
    from paper_2607_24059_amd import lbm
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    s = torch.cuda.current_stream()
    for _ in range(3):
        lbm.lbm_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, s.cuda_stream)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s)
    for _ in range(reps):
        lbm.lbm_copy_probe(dst.data_ptr(), src.data_ptr(), nbytes, s.cuda_stream)
    ev1.record(s)
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) / 1e3 / reps
    del src, dst
    return 2 * nbytes / sec / 1e9


def cpu_baseline(n: int = 4096, steps: int = 10, nu: float = 1e-3) -> dict:
    """The FP64 numpy oracle on `steps` steps of the same 4096^2 workload."""
    from oracle import scheme
    u0, dx, dt, _ = make_workload(n, 2, nu)
    p = scheme.Params(dim=2, dx=dx, dt=dt, nu=nu)
    f = scheme.init(np.ones((n, n)), u0, p)
    f = scheme.step(f, p)  # warm-up
    t0 = time.perf_counter()
    for _ in range(steps):
        f = scheme.step(f, p)
    sec = time.perf_counter() - t0
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), cpu)
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": n * n * steps / sec / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"numpy FP64 oracle, {n}x{n} k^-3 field, {steps} steps after 1 warm-up step "
                      f"({sec:.1f} s); numpy {np.__version__} element-wise kernels run on one thread "
                      f"of {avail} available ({cpu})"}


def headline_kernel(fuse: int) -> str:
    """The step kernel instantiation the 4096^2 FP32 engine launches at `fuse`
    steps per launch (tiles as chosen in the library)."""
    tile = {3: "32,16,256", 4: "64,16,512", 5: "32,32,768", 6: "32,28,768"}
    if fuse >= 3:
        return f"k_stepKr_2d<float,float,{tile[fuse]},{fuse},true>"
    return "k_step2_2d<float,float,256,8,1024>" if fuse == 2 else "k_step<2,float,float>"


def traffic_entry(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel source and on this kernel instantiation; else
    None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or t.get("kernel") != kernel:
        return None
    return t.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variant-steps", type=int, default=1000)
    ap.add_argument("--no-equal-error", action="store_true")
    ap.add_argument("--equal-error-seeds", type=int, default=2)
    ap.add_argument("--only", choices=sorted(ONLY),
                    help="run one secondary workload alone and print its JSON (for profiling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design, not a build).", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.only:
        print(json.dumps({"only": args.only, **ONLY[args.only](args)}), flush=True)
        return

    n = args.n
    log(f"[bench] generating {n}^2 workload")
    u0, dx, dt, lbm = make_workload(n, 2, 1e-3)
    log("[bench] copy probe")
    probe = copy_probe_gbs()
    log(f"[bench] probe {probe:.0f} GB/s; timing {args.steps} steps after {args.warmup} warm-up")
    ms, eng = time_engine(n, 2, "f32", args.steps, args.warmup, u0=u0)
    fuse = eng.fusion()                      # steps per launch (the library default)
    d = eng.diagnostics()
    eng.close()
    del eng
    cells = n * n
    mlups = cells / (ms * 1e-3) / 1e6
    lup_bytes = BYTES_PER_LUP[("f32", 2)]
    launch_ms = fuse * ms                    # one launch advances `fuse` steps
    # The unit of the roofline is one cell per launch: a launch must read each
    # cell's state (15 FP32 values) once and write it once, 120 B, however
    # many steps it fuses (the intermediate steps stay on chip).
    unit_bytes = lup_bytes
    bytes_launch = unit_bytes * cells
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    single = lup_bytes * fuse * cells        # the same updates as `fuse` single-step launches
    kname = headline_kernel(fuse)
    traffic = traffic_entry(kname)
    result = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"vectorial D2Q5, {n}x{n} periodic, nu=1e-3, mu=8, k^-3 random "
                               f"field at Mach 0.05, FP32 storage+math, {fuse} fused steps per launch",
                   "grid": [n, n], "storage": "f32", "nu": 1e-3, "mu": 8.0,
                   "omega_rho": 1.2, "omega_q": 1.15, "alpha_rho": 0.075, "steps_per_launch": fuse},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "kernel": f"{kname} ({fuse} lattice updates per cell per launch)",
                     "unit_bytes": unit_bytes, "units_per_launch": cells,
                     "bytes_per_launch": bytes_launch, "launch_us": round(launch_ms * 1e3, 2),
                     "note": "achieved = the state read once and written once per launch "
                             "(120 B per cell) / the average launch time from HIP events on the "
                             "engine's stream; traffic = HBM bytes per launch from the committed "
                             "rocprofv3 FETCH_SIZE / WRITE_SIZE summary (null if the kernel source "
                             "changed since)",
                     "traffic_gbs": round(traffic / (launch_ms * 1e-3) / 1e9, 1) if traffic else None,
                     "probe_gbs": round(probe, 1), "frac_of_probe": round(achieved / probe, 4),
                     "equivalent_single_steps": {
                         "bytes_per_launch": single,
                         "gbs": round(single / (launch_ms * 1e-3) / 1e9, 1),
                         "frac_of_peak": round(single / (launch_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                         "note": f"the {fuse} updates per cell priced as {fuse} single-step launches "
                                 "(120 B per lattice update); above 1 because the fused launch moves "
                                 "fewer bytes"}},
        "health": {"nonfinite": d["nonfinite"], "mass": d["mass"], "kinetic": d["kinetic"]},
    }

    if not args.no_variants:
        variants = {}
        vs = args.variant_steps
        log("[bench] variant 2D f32 single step per launch")
        ms_v, e = time_engine(n, 2, "f32", vs, VARIANT_WARMUP, u0=u0, fuse=1)
        e.close()
        variants[f"2d_{n}_f32_one_step_per_launch"] = _variant(cells, ms_v, BYTES_PER_LUP[("f32", 2)], probe)
        log("[bench] variant 2D f32 two steps per launch")
        ms_v, e = time_engine(n, 2, "f32", vs, VARIANT_WARMUP, u0=u0, fuse=2)
        e.close()
        variants[f"2d_{n}_f32_two_steps_per_launch"] = _variant(cells, ms_v, BYTES_PER_LUP[("f32", 2)], probe)
        for storage in ("f16_dev", "bf16_dev", "f16_dev_r32", "f16_neq"):
            log(f"[bench] variant 2D {storage}")
            ms_v, e = time_engine(n, 2, storage, vs, VARIANT_WARMUP, u0=u0)
            fuse_v = e.fusion()
            e.close()
            variants[f"2d_{n}_{storage}"] = _variant(cells, ms_v, BYTES_PER_LUP[(storage, 2)], probe)
            variants[f"2d_{n}_{storage}"]["steps_per_launch"] = fuse_v
        del u0
        n3 = 256
        u3, *_ = make_workload(n3, 3, 1e-3)
        for storage, fuse_3 in (("f32", None), ("f32", 2), ("f32", 1), ("f16_dev", None), ("bf16_dev", None),
                                ("f16_dev_r32", None), ("bf16_dev_r32", None), ("f16_neq", None)):
            name = f"3d_{n3}_{storage}" + {1: "_one_step_per_launch", 2: "_two_steps_per_launch"}.get(fuse_3, "")
            log(f"[bench] variant {name}")
            ms_v, e = time_engine(n3, 3, storage, vs, VARIANT_WARMUP, u0=u3, fuse=fuse_3)
            fuse_v = e.fusion()
            e.close()
            variants[name] = _variant(n3 ** 3, ms_v, BYTES_PER_LUP[(storage, 3)], probe)
            variants[name]["steps_per_launch"] = fuse_v
        for dim_m, n_m in ((2, n), (3, 256)):
            log(f"[bench] variant {dim_m}D moment-only storage, relaxation scheme omega = 1")
            variants[f"{dim_m}d_{n_m}_f32_moments_omega1"] = moments_variant(dim_m, n_m, vs, probe)
        log("[bench] variant 2D 4096^2 channel boundaries (one step per launch)")
        variants[f"2d_{n}_f32_channel_walls"] = walls_variant(n, vs, probe)
        log("[bench] Poiseuille 253^2 to t = 0.05 in FP64 storage (Table 2 case)")
        variants["poiseuille_253_f64"] = poiseuille_variant()
        for storage in ("f32", "f16_dev_r32"):
            log(f"[bench] batch 512 runs {storage}")
            variants[f"batch512_{storage}"] = batch_variant(storage, 1000, probe)
        log("[bench] batch 512 runs f32, one and two steps per launch")
        variants["batch512_f32_one_step_per_launch"] = batch_variant("f32", 1000, probe, fuse=1)
        variants["batch512_f32_two_steps_per_launch"] = batch_variant("f32", 1000, probe, fuse=2)
        log("[bench] Taylor-Green parameter sweep (Fig. 2 plane + Fig. 3 curves) as one batch")
        variants["sweep_tg75_fig2_fig3"] = sweep_variant()
        for dim_s in (2, 3):
            log(f"[bench] batched linear spectra, {dim_s}D")
            variants[f"spectrum_{dim_s}d"] = spectrum_variant(dim_s)
        result["variants"] = variants

    if not args.no_equal_error:
        log("[bench] equal-error comparison (FP64 2048^2 reference, plain FP32 / FP16 levels, learned closure)")
        result["equal_error"] = equal_error_section(args.equal_error_seeds)

    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(result), flush=True)


def _finite(v):
    """JSON-safe copy: NaN / inf become null."""
    if isinstance(v, dict):
        return {k: _finite(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_finite(x) for x in v]
    if isinstance(v, float) and not math.isfinite(v):
        return None
    return v


def equal_error_section(n_seeds: int) -> dict:
    """Speedups over the plain FP32 scheme at equal error against the fine-grid
    reference, on the closure workload: k^-3 fields (held-out seeds 1000...),
    nu = 5e-4, coarse 256^2, reference = the plain scheme at 2048^2 in FP64
    storage restricted to 256^2, 256 coarse steps.  Plain levels 256^2, 512^2,
    1024^2, 2048^2 in FP32, FP64, split FP16, FP16 + FP32-rest and all-FP16
    deviation storage; the
    corrected 256^2 run uses the committed trained network.  Errors: relative
    L2 of u and of its divergence-free part, each with its own equal-error
    speedups.  Times: HIP events around each run's steps."""
    from paper_2607_24059_amd import closure, cnn
    params, meta = closure.load_model(closure.WEIGHTS)
    cfg = closure.Config(**{k: v for k, v in meta["config"].items()
                            if k in ("coarse_n", "factor", "nu", "mach", "mu", "every", "guard")})
    cfg.test_seeds = list(range(1000, 1000 + n_seeds))
    net = cnn.Net(params=params)
    ev = closure.evaluate(cfg, net, meta["scales"], log=log, levels=(256, 512, 1024, 2048),
                          plain_storages=("f32", "f64", "f16_neq", "f16_dev_r32", "f16_dev"))
    return _finite({"workload": f"k^-3 field, nu={cfg.nu}, coarse {cfg.coarse_n}^2, reference FP64 "
                        f"{cfg.fine_n}^2 restricted, {cfg.horizon} coarse steps, "
                        f"seeds {cfg.test_seeds[0]}..{cfg.test_seeds[-1]}",
            "error_metrics": {"u": "relative L2 of u on the coarse grid",
                              "u_sol": "relative L2 of the divergence-free part of u"},
            "plain": ev["plain"], "closure": ev["closure"], "speedup": ev["speedup_equal_error"]})


def _restrict_3d(a: np.ndarray, r: int) -> np.ndarray:
    """Block averages over r^3 cells of the last three axes (host arrays)."""
    if r == 1:
        return a
    m = a.shape[-1] // r
    return a.reshape(a.shape[:-3] + (m, r, m, r, m, r)).mean(axis=(-5, -3, -1))


def _solenoidal_3d(u: np.ndarray) -> np.ndarray:
    """Divergence-free part of a periodic field u[3][z][y][x] (spectral
    Helmholtz projection; the same operator on both sides of a comparison)."""
    n = u.shape[-1]
    k = np.fft.fftfreq(n, 1.0 / n)
    kv = (k[None, None, :], k[None, :, None], k[:, None, None])   # kx, ky, kz
    k2 = kv[0] ** 2 + kv[1] ** 2 + kv[2] ** 2
    k2[0, 0, 0] = 1.0
    uh = [np.fft.fftn(c) for c in u]
    div = sum(kk * c for kk, c in zip(kv, uh))
    return np.stack([np.fft.ifftn(c - kk * div / k2).real for kk, c in zip(kv, uh)])


def _rel(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def precision_3d_variant(levels=(64, 128, 256), fine_n: int = 512, horizon: int = 64, seed: int = 1000,
                         storages=("f32", "f64", "f16_neq", "f16_dev_r32", "bf16_dev_r32", "f16_dev")) -> dict:
    """Storage precision at equal error in 3D: a k^-3 divergence-free field
    (Mach 0.05 on the coarsest grid, nu = 5e-4, dt = dx^2/8) run for `horizon`
    steps of the coarsest grid (levels[0]^3, the comparison grid) at each level
    in each storage, every run started from the block average of the fine
    initial field; reference = the FP64 run on fine_n^3, block-averaged to the
    comparison grid.  Errors are relative L2 of u and of its divergence-free
    part; times are HIP events around each run's steps.  Equal-error speedups
    against plain FP32 interpolate its error and time between levels."""
    import torch
    import inputs
    from paper_2607_24059_amd import lbm
    from paper_2607_24059_amd.closure import equal_error_speedup
    nc, mu, nu = levels[0], 8.0, 5e-4
    for n in levels:
        if fine_n % n or n % nc:
            raise ValueError(f"level {n} must divide {fine_n} and be a multiple of {nc}")
    u0f = inputs.random_field_3d(fine_n, seed, umax=0.05 / (2 * math.pi / nc))
    starts = {n: _restrict_3d(u0f, fine_n // n) for n in levels}

    def run(n, storage, u0):
        dx = 2 * math.pi / n
        eng = lbm.Engine.create(lbm.make_params(3, (n, n, n), dx, dx * dx / mu, nu, storage=storage), u0)
        steps = horizon * (n // nc) ** 2
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(eng.stream)
        eng.step(steps)
        e1.record(eng.stream)
        torch.cuda.synchronize()
        rho, q = eng.moments()
        fuse = eng.fusion()
        eng.close()
        r = n // nc
        u = _restrict_3d(q, r) / _restrict_3d(rho, r)[None]
        return u, e0.elapsed_time(e1), steps, fuse

    log(f"[precision 3d] FP64 reference {fine_n}^3, {horizon * (fine_n // nc) ** 2} steps")
    ref, t_ref, _, _ = run(fine_n, "f64", u0f)
    del u0f
    ref_sol = _solenoidal_3d(ref)
    err = {st: {"u": {}, "u_sol": {}} for st in storages}
    tim = {st: {} for st in storages}
    fuse_of = {}
    for st in storages:
        for n in levels:
            u, ms, steps, fuse = run(n, st, starts[n])
            err[st]["u"][str(n)] = _rel(u, ref)
            err[st]["u_sol"][str(n)] = _rel(_solenoidal_3d(u), ref_sol)
            tim[st][str(n)] = ms
            fuse_of[st] = fuse
            log(f"[precision 3d] {st} {n}^3: u {err[st]['u'][str(n)]:.3e} u_sol {err[st]['u_sol'][str(n)]:.3e} "
                f"{ms:.1f} ms ({n ** 3 * steps / (ms * 1e-3) / 1e9:.1f} GLUPS)")
    speed = {}
    for st in storages:
        if st == "f32":
            continue
        speed[st] = {}
        for metric in ("u_sol", "u"):
            speed[st][metric] = {}
            for n in levels:
                k = str(n)
                sp = equal_error_speedup(levels, err["f32"][metric], tim["f32"], err[st][metric][k], tim[st][k])
                sp["speedup_same_resolution"] = tim["f32"][k] / tim[st][k]
                sp["error_ratio_same_resolution"] = err[st][metric][k] / err["f32"][metric][k]
                speed[st][metric][k] = {a: (None if isinstance(b, float) and math.isnan(b) else b)
                                        for a, b in sp.items()}
    return {"workload": f"3D k^-3 field, nu={nu}, Mach 0.05 on {nc}^3, dt = dx^2/{mu:g}, {horizon} steps of "
                        f"the {nc}^3 grid, reference FP64 {fine_n}^3 block-averaged, seed {seed}",
            "reference_ms": t_ref, "steps_per_launch": fuse_of, "errors": err, "time_ms": tim,
            "speedup_vs_f32": speed}


def moments_variant(dim: int, n: int, steps: int, probe: float) -> dict:
    """The relaxation scheme (omega_rho = omega_q = 1) on the same k^-3 field,
    in moment-only storage: (1 + dim) FP32 planes, 24 B (2D) / 32 B (3D) per
    lattice update; the library's default fusion (four steps per launch in 2D
    from 2^20 cells on, two in 3D where that launch has at least 128 blocks)."""
    import torch
    from paper_2607_24059_amd import lbm
    u0, dx, dt, _ = make_workload(n, dim, 1e-3)
    prm = lbm.make_params(dim, (n,) * dim, dx, dt, 1e-3, omega_rho=1.0, omega_q=1.0, alpha_rho=0.05,
                          storage="f32_moments")   # (omega_rho, alpha_rho) = (1, 1/20) of Section 5.1
    eng = lbm.Engine.create(prm, u0)
    eng.step(VARIANT_WARMUP)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(eng.stream)
    eng.step(steps)
    ev1.record(eng.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    fuse = eng.fusion()
    eng.close()
    out = _variant(n ** dim, ms, 4 * 2 * (dim + 1), probe)
    out["steps_per_launch"] = fuse
    return out


def walls_variant(n: int, steps: int, probe: float) -> dict:
    """The 4096^2 FP32 workload with the channel boundaries set (inlet profile,
    outlet density, corrected walls): one step per launch with the boundary
    cells' ghost values computed in the step kernel."""
    import torch
    from paper_2607_24059_amd import lbm
    u0, dx, dt, _ = make_workload(n, 2, 1e-3)
    eng = lbm.Engine.create(lbm.make_params(2, (n, n), dx, dt, 1e-3), u0)
    eng.set_walls(np.stack([np.full(n, 0.05 / dx), np.zeros(n)]), 1.0, correction=True)
    eng.step(VARIANT_WARMUP)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(eng.stream)
    eng.step(steps)
    ev1.record(eng.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    eng.close()
    return _variant(n * n, ms, BYTES_PER_LUP[("f32", 2)], probe)


def poiseuille_variant(n: int = 253) -> dict:
    """The Poiseuille test of Table 2 (omega_q = 1.15, corrected walls) at
    n^2 to t = 0.05 in FP64 storage: wall time and the L2 error on u_x."""
    import torch
    from paper_2607_24059_amd import lbm
    dx = 1.0 / n
    dt = dx * dx / 8.0
    nu = 0.01
    c = (np.arange(n) + 0.5) * dx                      # cell centres along x and along y
    u_ex = 4 * c * (1 - c)                             # u(y) = 4 U y (L - y) / L^2, U = L = 1
    rho0 = np.broadcast_to(1.0 + dx * dx * 8 * nu * (1 - c)[None, :], (n, n)).copy()  # 1 + dx^2 p(x)
    u0 = np.zeros((2, n, n))
    u0[0] = u_ex[:, None]
    eng = lbm.Engine.create(lbm.make_params(2, (n, n), dx, dt, nu, omega_q=1.15, storage="f64"), u0, rho0)
    eng.set_walls(np.stack([u_ex, np.zeros(n)]), 1.0, correction=True)
    steps = int(round(0.05 / dt))
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(eng.stream)
    eng.step(steps)
    ev1.record(eng.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    rho, q = eng.moments()
    eng.close()
    e = q[0] / rho - u_ex[:, None]
    err = float(np.sqrt(dx * dx * np.sum(e * e)))
    return {"MLUPS": round(n * n * steps / (ms * 1e-3) / 1e6, 1), "steps": steps, "ms": round(ms, 2),
            "l2_error_ux": err, "table2_value": 1.368e-06}


def batch_variant(storage: str, steps: int, probe: float, n_runs: int = 512, fuse: int | None = None) -> dict:
    """The batch workload: n_runs independent 2D runs, sizes 64^2..1024^2,
    nu log-uniform in [1e-4, 1e-2], k^-3 fields at Mach 0.05, all advanced
    `steps` steps by persistent launches replayed from graphs: the batch's
    multi-step default (fuse = None: six steps per launch in FP32, where most
    cells are in the 1024^2 runs, five in the 16-bit storages), two or one."""
    import torch
    import inputs
    from paper_2607_24059_amd import batch as B
    specs = inputs.batch_run_specs(n_runs)
    runs, u0s = [], []
    for s in specs:
        n = s["n"]
        dx = 2 * math.pi / n
        runs.append(B.make_run((n, n), dx, dx * dx / 8, s["nu"]))
        u0s.append(inputs.random_field_2d(n, s["seed"], umax=0.05 / dx))
    b = B.Batch.create(2, storage, runs, u0s)
    del u0s
    b.autotune(None)
    if fuse is not None:
        b.set_fusion(fuse)
    fuse = b.fusion()
    b.step(10)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(b.stream)
    b.step(steps)
    ev1.record(b.stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    cells, tiles, _ = b.info()
    widths = sorted({(int(r.n[0]), b.tile_width(i)) for i, r in enumerate(runs)})
    shapes = sorted({(int(r.n[0]), "x".join(map(str, b.fused_tile(i)))) for i, r in enumerate(runs)}) \
        if fuse > 2 else []
    grid, grid2 = b.grid(), b.fused_grid()
    b.close()
    out = _variant(cells, ms, BYTES_PER_LUP[(storage, 2)], probe)
    out.update({"runs": n_runs, "cells": cells, "tiles": tiles, "steps": steps, "steps_per_launch": fuse,
                "grid": grid, "fused_grid": grid2,
                "tile_width_by_n": {str(n): w for n, w in widths},
                "fused_tile_by_n": {str(n): t for n, t in shapes}})
    return out


def sweep_variant() -> dict:
    """The parameter sweeps of Section 5.1 at 75 cells to t = 1: the Fig. 2
    plane (omega_rho in 1..1.95, alpha_rho in 0.01..0.25, omega_q = 1) and
    the Fig. 3 curves (omega_q in 1..1.6 for the three isoline pairs), one
    batch, FP32, tiles autotuned; wall time of the time stepping."""
    from paper_2607_24059_amd import sweep
    tg = sweep.TaylorGreen()
    pts2, pts3 = sweep.figure2_points(), sweep.figure3_points()
    res = sweep.run(pts2 + pts3, tg, autotune=True)
    e2 = res.errors[:len(pts2)]
    i = int(np.argmin(e2))
    iso = {f"{wr:g},{ar:g}": float(res.errors[len(pts2) + pts3.index((wr, ar, 1.15))])
           for wr, ar in sweep.PAIRS}
    return _finite({"runs": len(res.points), "cells_per_run": tg.n ** 2, "steps": res.steps,
                    "ms": round(res.seconds * 1e3, 2), "MLUPS": round(res.glups * 1e3, 1),
                    "fig2_min_error": float(e2[i]), "fig2_min_at": list(pts2[i][:2]),
                    "fig2_nonfinite_runs": int(np.sum(~np.isfinite(e2))),
                    "isoline_errors_omega_q_1.15": iso, "nu": tg.nu})


def spectrum_variant(dim: int, reps: int = 3, cpu_points: int = 1000) -> dict:
    """Eigenvalues of E(theta) (Section 4) for a map of points: in 2D the
    Fig. 1 setting (omega = 1, alpha_rho = 1/4, nu = pi/50, alpha_q = nu/mu,
    reference (1, 1, 1), dx = 1e-6) for 64 values of mu in [0.5, 16] x 4096
    frequencies on the diagonal; in 3D 16 general-omega states x 4096 random
    frequencies.  Time: HIP events around the launch on its stream; work:
    the flops the kernel counts (reflections and rotations).  CPU: LAPACK
    (numpy) on the oracle's matrices for a sample of the points, one core."""
    import time
    import torch
    from paper_2607_24059_amd import spectrum as S
    from oracle import spectrum as O
    nth = 4096
    if dim == 2:
        nu = math.pi / 50
        mus = np.linspace(0.5, 16.0, 64)
        states = [S.make_state(mu, 1e-6, 1.0, 1.0, 0.25, nu / mu, 1.0, (1.0, 1.0)) for mu in mus]
        prm = [(1e-6, mu, 1.0, 1.0, 0.25, nu / mu, 1.0, np.array([1.0, 1.0])) for mu in mus]
        taus = np.linspace(-math.pi, math.pi, nth)
        th = np.tile(np.stack([taus, taus], axis=1), (len(mus), 1))
    else:
        rng = np.random.default_rng(3)
        states, prm = [], []
        for _ in range(16):
            w = rng.uniform(1.0, 1.9, 2)
            a = rng.uniform(0.0, 1.0 / 6.0, 2)
            mu = rng.uniform(4.0, 12.0)
            qb = rng.uniform(-1, 1, 3)
            states.append(S.make_state(mu, 1e-3, w[0], w[1], a[0], a[1], 1.0, qb))
            prm.append((1e-3, mu, w[0], w[1], a[0], a[1], 1.0, qb))
        th = rng.uniform(-math.pi, math.pi, (16 * nth, 3))
    idx = np.repeat(np.arange(len(states), dtype=np.int32), nth)
    pb = S.Problem(dim, states, th, idx)
    stream = torch.cuda.current_stream()
    pb.launch(stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        pb.launch(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    res = pb.results()
    flops = float(np.sum(res["flops"]))
    gflops = flops / (ms * 1e-3) / 1e9
    sample = np.linspace(0, len(idx) - 1, cpu_points).astype(int)
    t0 = time.perf_counter()
    for p in sample:
        dx, mu, wr, wq, ar, aq, rb, qb = prm[idx[p]]
        np.linalg.eigvals(O.amplification_matrix(th[p], dim, dx, mu, wr, wq, ar, aq, rb, qb))
    cpu_s = time.perf_counter() - t0
    return {"points": int(len(idx)), "order": S.lbm_spectrum_order(dim), "ms": round(ms, 3),
            "points_per_s": round(len(idx) / (ms * 1e-3), 1), "mean_qr_sweeps": round(float(res["info"].mean()), 2),
            "unconverged": int(np.sum(res["info"] < 0)), "counted_gflops": round(gflops, 2),
            "frac_fp64_vector_peak": round(gflops / 78600.0, 5),
            "cpu_lapack_points_per_s": round(cpu_points / cpu_s, 1), "cpu_sample_points": cpu_points}


def _variant(cells, ms, bytes_per_lup, probe):
    gbs = bytes_per_lup * cells / (ms * 1e-3) / 1e9
    return {"MLUPS": round(cells / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5),
            "GBs": round(gbs, 1), "frac_peak": round(gbs / PEAK_HBM_GBS, 4),
            "frac_probe": round(gbs / probe, 4)}


def engine_variant(dim: int, n: int, storage: str, steps: int, probe: float) -> dict:
    """One run of the step engine on the k^-3 field at the library's default
    fusion: the rate priced at the scheme's bytes per lattice update."""
    u0, *_ = make_workload(n, dim, 1e-3)
    ms, e = time_engine(n, dim, storage, steps, VARIANT_WARMUP, u0=u0)
    fuse = e.fusion()
    e.close()
    out = _variant(n ** dim, ms, BYTES_PER_LUP[(storage, dim)], probe)
    out["steps_per_launch"] = fuse
    return out


# secondary workloads that `--only` runs alone (each as in the variants section)
ONLY = {
    "engine_3d": lambda a: engine_variant(3, 256, "f32", a.variant_steps, copy_probe_gbs()),
    "spectrum_2d": lambda a: spectrum_variant(2, cpu_points=10),
    "spectrum_3d": lambda a: spectrum_variant(3, cpu_points=10),
    "moments_2d": lambda a: moments_variant(2, a.n, a.variant_steps, copy_probe_gbs()),
    "moments_3d": lambda a: moments_variant(3, 256, a.variant_steps, copy_probe_gbs()),
    "sweep": lambda a: sweep_variant(),
    "batch_f32": lambda a: batch_variant("f32", 1000, copy_probe_gbs()),
    "precision_3d": lambda a: precision_3d_variant(),
    "batch_f16_dev_r32": lambda a: batch_variant("f16_dev_r32", 1000, copy_probe_gbs()),
}

if __name__ == "__main__":
    main()
