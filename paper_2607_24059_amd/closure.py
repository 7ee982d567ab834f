"""Learned coarse-grid correction: bindings of include/lbm_closure.h and the
driver that generates data, trains the network and evaluates it.

Workload (defaults): coarse 256^2 runs of the D2Q5 scheme corrected every 4
coarse steps by the four-layer 3x3 network of `cnn`; training data from 2048^2
fine runs of the same scheme (nu = 5e-4, k^-3 random fields at coarse Mach
0.05, mu = 8 on both grids so one coarse step is 64 fine steps), restricted
8x to the coarse grid; compared with held-out fine runs; the guard falls back
to the plain coarse step when the correction would more than double the
discrete divergence norm.

Every numerical step runs in liblbm.so; this module sequences calls and keeps
device buffers (torch tensors) and a few host scalars (normalisation scales,
errors).

    python -m paper_2607_24059_amd.closure --train-seeds 200 --test-seeds 20 --out model.npz
"""

from __future__ import annotations

import argparse
import ctypes as C
import json
import math
import os
import sys
import time
from dataclasses import asdict, dataclass, field

import numpy as np

from . import cnn
from .lbm import Engine, _ok, lib, make_params


class lbm_closure_report(C.Structure):
    _fields_ = [("n_accepted", C.c_int64), ("n_rejected", C.c_int64), ("accepted", C.c_int32), ("div_before", C.c_double), ("div_after", C.c_double),
                ("mean", C.c_double * 3)]


SIGNATURES = {
    "lbm_restrict": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_double, C.c_void_p, C.c_void_p]),
    "lbm_closure_features": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float, C.c_float,
                                       C.c_void_p, C.c_void_p]),
    "lbm_closure_target": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_float, C.c_void_p,
                                     C.c_void_p]),
    "lbm_set_equilibrium_device": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_closure_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_float, C.c_float]),
    "lbm_closure_correct": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_float,
                                      C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p, C.c_void_p]),
    "lbm_closure_report_get": (C.c_int, [C.c_void_p, C.POINTER(lbm_closure_report)]),
    "lbm_closure_project_scratch_bytes": (C.c_size_t, [C.c_int32]),
    "lbm_closure_project": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
}

_bound = False


def xlib():
    global _bound
    L = lib()
    if not _bound:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _p(t):
    return C.c_void_p(t.data_ptr())


def lbm_restrict(fine, nfx, nfy, r, rho_ref, coarse, stream):
    # the C entry point writes 3 (nfx/r)(nfy/r) values: check the buffers against that
    if r < 1 or nfx % r or nfy % r or fine.numel() < 3 * nfx * nfy or coarse.numel() != 3 * (nfx // r) * (nfy // r):
        raise ValueError(f"lbm_restrict: {nfx}x{nfy} by {r} does not match the buffers")
    _ok(xlib().lbm_restrict(_p(fine), nfx, nfy, r, rho_ref, _p(coarse), C.c_void_p(stream.cuda_stream)),
        "lbm_restrict")


def lbm_closure_features(moments, dim, cells, rho_ref, s_rho, s_u, x, stream):
    _ok(xlib().lbm_closure_features(_p(moments), dim, cells, rho_ref, s_rho, s_u, _p(x),
                                    C.c_void_p(stream.cuda_stream)), "lbm_closure_features")


def lbm_closure_target(m_next, m_now, cells, s_drho, s_dq, t, stream):
    _ok(xlib().lbm_closure_target(_p(m_next), _p(m_now), cells, s_drho, s_dq, _p(t),
                                  C.c_void_p(stream.cuda_stream)), "lbm_closure_target")


def lbm_closure_project_scratch_bytes(n):
    return int(xlib().lbm_closure_project_scratch_bytes(int(n)))


def lbm_closure_project(m_fine, m_now, n, out, scratch, stream):
    _ok(xlib().lbm_closure_project(_p(m_fine), _p(m_now), int(n), _p(out), _p(scratch),
                                   C.c_void_p(stream.cuda_stream)), "lbm_closure_project")


def lbm_set_equilibrium_device(ctx, moments):
    _ok(xlib().lbm_set_equilibrium_device(C.c_void_p(ctx), _p(moments)), "lbm_set_equilibrium_device")


def lbm_closure_apply(ctx, moments, y, s_drho, s_dq, guard_factor):
    _ok(xlib().lbm_closure_apply(C.c_void_p(ctx), _p(moments), _p(y), s_drho, s_dq, guard_factor),
        "lbm_closure_apply")


def lbm_closure_correct(ctx, net, s_rho, s_u, s_drho, s_dq, guard_factor, moments, y):
    packed, bias = net.layer_pointers()
    _ok(xlib().lbm_closure_correct(C.c_void_p(ctx), packed, bias, s_rho, s_u, s_drho, s_dq, guard_factor,
                                   _p(moments), _p(y)), "lbm_closure_correct")


def lbm_closure_report_get(ctx):
    r = lbm_closure_report()
    _ok(xlib().lbm_closure_report_get(C.c_void_p(ctx), C.byref(r)), "lbm_closure_report_get")
    return {"n_accepted": r.n_accepted, "n_rejected": r.n_rejected, "accepted": bool(r.accepted), "div_before": r.div_before, "div_after": r.div_after,
            "mean": list(r.mean)}


# --------------------------------------------------------------------------- #
# driver                                                                      #
# --------------------------------------------------------------------------- #

@dataclass
class Config:
    coarse_n: int = 256
    factor: int = 8
    nu: float = 5e-4
    mach: float = 0.05
    mu: float = 8.0
    every: int = 4                 # coarse steps between corrections
    pairs_per_seed: int = 16       # training pairs (4-coarse-step windows) per fine run
    train_seeds: list = field(default_factory=lambda: list(range(200)))
    test_seeds: list = field(default_factory=lambda: list(range(1000, 1020)))
    horizon: int = 256             # coarse steps of each evaluation run (and training span)
    batch: int = 8
    epochs: int = 20
    lr: float = 1e-3
    guard: float = 2.0
    eval_levels: tuple = (256, 512, 1024, 2048)
    project_targets: bool = True   # correct the divergence-free momentum only (else rho and q)
    fine_storage: str = "f64"      # the fine reference runs: FP32 rounding accumulates over their
                                   # factor^2 more steps to well above the coarse error

    @property
    def fine_n(self):
        return self.coarse_n * self.factor

    def dx(self, n):
        return 2 * math.pi / n

    def umax(self):
        """Physical speed bound: Mach 0.05 on the coarse grid (dx_c max|u| = 0.05)."""
        return self.mach / self.dx(self.coarse_n)


def _engine(cfg: Config, n: int, u0=None, storage="f32", rho0=None):
    dx = cfg.dx(n)
    prm = make_params(2, (n, n), dx, dx * dx / cfg.mu, cfg.nu, storage=storage)
    if u0 is None:
        u0 = np.zeros((2, n, n))
    return Engine.create(prm, u0, rho0)


def _field(cfg: Config, n: int, seed: int):
    """Velocity of seed `seed` and a well-prepared density carrying its pressure:
    P(rho0) = 1 + dx^2 Phi (eq. (3.2)); starting from rho = 1 instead would
    launch O(dx) acoustic waves whose phase no coarse model can predict."""
    import inputs
    u = inputs.random_field_2d(n, seed, umax=cfg.umax())
    phi = inputs.random_pressure_2d(n, seed, umax=cfg.umax())
    return u, inputs.well_prepared_density(phi, cfg.dx(n))


class FineRun:
    """One fine run of the scheme; its moments restricted to coarser grids on request."""

    def __init__(self, cfg: Config, seed: int, stream):
        import torch
        self.cfg = cfg
        self.nf = cfg.fine_n
        self.stream = stream
        u0, rho0 = _field(cfg, self.nf, seed)
        self.eng = _engine(cfg, self.nf, u0, storage=cfg.fine_storage, rho0=rho0)
        self.m = torch.empty((3, self.nf, self.nf), dtype=torch.float32, device="cuda")

    def advance(self, coarse_steps: int) -> None:
        # mu fixed on both grids: one coarse step is factor^2 fine steps
        self.eng.step(coarse_steps * self.cfg.factor ** 2)

    def restricted(self, n: int, out) -> None:
        self.eng.moments_device(self.m)
        lbm_restrict(self.m, self.nf, self.nf, self.nf // n, 1.0, out, self.stream)

    def close(self):
        self.eng.close()


def _projected_next(m_c, m_f, out, scratch, stream, project=True):
    """out = m_c + P(m_f - m_c) on the device (lbm_closure_project), with P
    keeping the divergence-free part of the momentum difference and no
    density difference.  The fine and coarse grids carry acoustic waves at
    different speeds (1/dx) whose relative phase no coarse-grid model can
    predict; the solenoidal part is the incompressible dynamics the
    correction can learn."""
    if not project:
        out.copy_(m_f)
        return
    lbm_closure_project(m_f, m_c, m_c.shape[-1], out, scratch, stream)


def build_dataset(cfg: Config, log=print):
    """Training pairs along a shadow coarse trajectory.

    For each training seed a fine run (FP64 storage) and a coarse run start
    from the same restricted state.  After every window of `every` coarse
    steps the pair (coarse moments, restricted fine moments) is formed, and
    the coarse run is nudged onto the fine one by the same guarded correction
    the corrected run applies (its populations keep their non-equilibrium
    part), with the projected difference as the correction.  So the network
    sees coarse states exactly as the corrected run produces them, not states
    freshly set to equilibrium (whose first step lacks the viscous flux of the
    non-equilibrium part).  pairs_per_seed windows, evenly spread over the
    horizon, are kept; returns the network inputs, targets and scales."""
    import torch
    s = torch.cuda.current_stream()
    nc = cfg.coarse_n
    cells = nc * nc
    windows = max(1, cfg.horizon // cfg.every)
    keep_every = max(1, windows // cfg.pairs_per_seed)
    P = len(cfg.train_seeds) * cfg.pairs_per_seed
    mc = torch.empty((P, 3, nc, nc), dtype=torch.float32, device="cuda")
    mn = torch.empty_like(mc)
    m_c = torch.empty((3, nc, nc), dtype=torch.float32, device="cuda")
    m_f = torch.empty_like(m_c)
    m_next = torch.empty_like(m_c)
    y = torch.empty_like(m_c)
    proj = torch.empty(lbm_closure_project_scratch_bytes(nc), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(12345)
    perm = rng.permutation(P)  # shuffled storage order: minibatches are contiguous slices
    t0 = time.time()
    for si, seed in enumerate(cfg.train_seeds):
        fine = FineRun(cfg, seed, s)
        ceng = _engine(cfg, nc)
        fine.restricted(nc, m_f)
        lbm_set_equilibrium_device(ceng.ctx, m_f)
        k = 0
        for w in range(windows):
            ceng.step(cfg.every)
            ceng.moments_device(m_c)
            fine.advance(cfg.every)
            fine.restricted(nc, m_f)
            _projected_next(m_c, m_f, m_next, proj, s, cfg.project_targets)
            if w % keep_every == keep_every - 1 and k < cfg.pairs_per_seed:
                j = int(perm[si * cfg.pairs_per_seed + k])
                mc[j].copy_(m_c)
                mn[j].copy_(m_next)
                k += 1
            # nudge: g += f^eq(W + dW) - f^eq(W), dW = projected difference
            lbm_closure_target(m_next, m_c, cells, 1.0, 1.0, y, s)
            lbm_closure_apply(ceng.ctx, m_c, y, 1.0, 1.0, 1e30)
        ceng.close()
        fine.close()
        if si % 20 == 0:
            torch.cuda.synchronize()
            log(f"[closure] data seed {seed} ({si + 1}/{len(cfg.train_seeds)}) {time.time() - t0:.1f}s")
    # scales: rms of the raw features and of the raw moment differences
    x = torch.empty_like(mc)
    t = torch.empty_like(mc)
    for i in range(P):
        lbm_closure_features(mc[i], 2, cells, 1.0, 1.0, 1.0, x[i], s)
        lbm_closure_target(mn[i], mc[i], cells, 1.0, 1.0, t[i], s)
    picks = range(0, P, max(1, P // 64))
    raw = np.zeros(3)
    rawd = np.zeros(3)
    for i in picks:
        raw += cnn.channel_rms(x[i], 3, s).cpu().numpy() ** 2
        rawd += cnn.channel_rms(t[i], 3, s).cpu().numpy() ** 2
    raw = np.sqrt(raw / len(picks))
    rawd = np.sqrt(rawd / len(picks))
    scales = {"s_rho": float(raw[0]), "s_u": float(math.sqrt((raw[1] ** 2 + raw[2] ** 2) / 2)),
              "s_drho": float(rawd[0]) if rawd[0] > 0 else 1.0,
              "s_dq": float(math.sqrt((rawd[1] ** 2 + rawd[2] ** 2) / 2))}
    for i in range(P):
        lbm_closure_features(mc[i], 2, cells, 1.0, scales["s_rho"], scales["s_u"], x[i], s)
        lbm_closure_target(mn[i], mc[i], cells, scales["s_drho"], scales["s_dq"], t[i], s)
    if cfg.project_targets:
        scales["s_drho"] = 0.0  # the correction moves momentum only
    torch.cuda.synchronize()
    log(f"[closure] dataset: {P} pairs, scales {scales}, {time.time() - t0:.1f}s")
    return x, t, scales


def train(cfg: Config, x, t, log=print, seed: int = 0):
    import torch
    net = cnn.Net(seed=seed)
    P = x.shape[0]
    B = cfg.batch
    nb = P // B
    grad = torch.empty((B,) + tuple(x.shape[1:]), dtype=torch.float32, device="cuda")
    scratch = torch.empty(cnn.lbm_reduce_scratch_bytes(grad.numel()) // 4, dtype=torch.float32, device="cuda")
    losses = torch.zeros(nb, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(seed)
    history = []
    t0 = time.time()
    step = 0
    total = cfg.epochs * nb
    for ep in range(cfg.epochs):
        order = rng.permutation(nb)
        for bi in order:
            lr = cfg.lr * 0.5 * (1 + math.cos(math.pi * step / total))  # cosine schedule
            xb = x[bi * B:(bi + 1) * B]
            tb = t[bi * B:(bi + 1) * B]
            out = net.forward(xb)
            cnn.mse(out, tb, grad, net.stream, scratch, losses[bi:bi + 1])
            net.backward(grad)
            net.adam_step(lr=lr)
            step += 1
        mean_loss = float(losses.mean().item())
        history.append(mean_loss)
        log(f"[closure] epoch {ep + 1}/{cfg.epochs} mean batch loss {mean_loss:.4e} ({time.time() - t0:.1f}s)")
    return net, history


class CorrectedRun:
    """A coarse run with the guarded network correction after every `every`
    steps.  One window = `every` steps, moments, features, network forward,
    guarded correction; with use_graph the window is captured once in a HIP
    graph (every launch of the window goes to one private stream, the guard
    decides on the device, so nothing in the window needs the host) and
    replayed.  The context's host-side step counter does not advance during
    replays."""

    def __init__(self, cfg: Config, net, scales, m0, storage="f32", use_graph=True, fused=True):
        import torch
        self.torch = torch
        self.cfg, self.net, self.scales = cfg, net, scales
        nc = cfg.coarse_n
        self.cells = nc * nc
        self.stream = torch.cuda.Stream()
        self.graph = None
        self.use_graph = use_graph and cfg.every % 2 == 0  # even steps: the state returns to its buffer
        with torch.cuda.stream(self.stream):
            dx = cfg.dx(nc)
            prm = make_params(2, (nc, nc), dx, dx * dx / cfg.mu, cfg.nu, storage=storage)
            self.eng = Engine.create(prm, np.zeros((2, nc, nc)), stream=self.stream)
            lbm_set_equilibrium_device(self.eng.ctx, m0)
            self.m = torch.empty((3, nc, nc), dtype=torch.float32, device="cuda")
            self.x = torch.empty((1, 3, nc, nc), dtype=torch.float32, device="cuda")
            self.y = torch.empty((3, nc, nc), dtype=torch.float32, device="cuda")
            self.fused = fused
            self.net.forward(self.x.zero_())  # allocates the activation buffers outside any capture

    def _window(self):
        sc = self.scales
        self.eng.step(self.cfg.every)
        if self.fused:
            lbm_closure_correct(self.eng.ctx, self.net, sc["s_rho"], sc["s_u"], sc["s_drho"], sc["s_dq"],
                                self.cfg.guard, self.m, self.y)
            return
        self.eng.moments_device(self.m)
        lbm_closure_features(self.m, 2, self.cells, 1.0, sc["s_rho"], sc["s_u"], self.x, self.stream)
        y = self.net.forward(self.x)
        lbm_closure_apply(self.eng.ctx, self.m, y, sc["s_drho"], sc["s_dq"], self.cfg.guard)

    def run(self, windows: int):
        torch = self.torch
        with torch.cuda.stream(self.stream):
            if not self.use_graph:
                for _ in range(windows):
                    self._window()
                return
            if self.graph is None:
                self.stream.synchronize()
                self.graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(self.graph, stream=self.stream):
                    self._window()
            for _ in range(windows):
                self.graph.replay()

    def moments(self, out):
        with self.torch.cuda.stream(self.stream):
            self.eng.moments_device(out)

    def report(self):
        return lbm_closure_report_get(self.eng.ctx)

    def close(self):
        self.graph = None
        self.eng.close()


def _host(m):
    return m.double().cpu().numpy()


def rel_u(m, ref):
    """Relative L2 error of u = q/rho on the coarse grid (host arrays [3][n][n])."""
    u = m[1:] / m[0:1]
    ur = ref[1:] / ref[0:1]
    return float(np.linalg.norm((u - ur).ravel()) / np.linalg.norm(ur.ravel()))


def solenoidal(u):
    """Divergence-free part of a periodic 2D field (spectral Helmholtz projection)."""
    n = u.shape[-1]
    k = np.fft.fftfreq(n, 1.0 / n)
    kx, ky = k[None, :], k[:, None]
    k2 = kx * kx + ky * ky
    k2[0, 0] = 1.0
    ux, uy = np.fft.fft2(u[0]), np.fft.fft2(u[1])
    div = kx * ux + ky * uy
    return np.stack([np.fft.ifft2(ux - kx * div / k2).real, np.fft.ifft2(uy - ky * div / k2).real])


def rel_u_sol(m, ref):
    """Relative L2 error of the divergence-free part of u.  The scheme's
    artificial compressibility carries acoustic waves whose speed 1/dx differs
    on every grid; the incompressible solution the scheme approximates is the
    divergence-free part, so the comparison across grids is made on it."""
    u = solenoidal(m[1:] / m[0:1])
    ur = solenoidal(ref[1:] / ref[0:1])
    return float(np.linalg.norm((u - ur).ravel()) / np.linalg.norm(ur.ravel()))


def evaluate(cfg: Config, net, scales, log=print, seeds=None, levels=None, plain_storages=("f32", "f16_neq", "f16_dev_r32"),
             use_graph=True):
    """Errors against the restricted fine reference after `horizon` coarse steps,
    for the plain scheme at each level in each storage and for the corrected
    coarse run (FP32 storage), with the wall time of each run (HIP events
    around the steps only).  Every run starts from the restriction of the fine
    initial state to its own grid.  Errors are relative L2 over the coarse grid
    of u (`u`) and of its divergence-free part (`u_sol`, the primary metric:
    the acoustic waves of the artificial compressibility travel at speed ~1/dx
    and differ on every grid)."""
    import torch
    s = torch.cuda.current_stream()
    nc = cfg.coarse_n
    seeds = cfg.test_seeds if seeds is None else seeds
    levels = cfg.eval_levels if levels is None else levels
    chunks = cfg.horizon // cfg.every
    for n in levels:  # every level restricts the fine state and is restricted to the coarse grid
        if cfg.fine_n % n or n % nc:
            raise ValueError(f"level {n} must divide {cfg.fine_n} and be a multiple of {nc}")
    err = {st: {n: {"u_sol": [], "u": []} for n in levels} for st in plain_storages}
    tim = {st: {n: [] for n in levels} for st in plain_storages}
    cerr = {"u_sol": [], "u": []}
    ctim = []
    acc = rej = 0
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    mbuf = torch.empty((3, nc, nc), dtype=torch.float32, device="cuda")
    for seed in seeds:
        fine = FineRun(cfg, seed, s)
        starts = {}
        for n in levels:
            starts[n] = torch.empty((3, n, n), dtype=torch.float32, device="cuda")
            fine.restricted(n, starts[n])
        fine.advance(cfg.horizon)
        ref_c = torch.empty((3, nc, nc), dtype=torch.float32, device="cuda")
        fine.restricted(nc, ref_c)
        fine.close()
        ref_h = _host(ref_c)
        for st in plain_storages:
            for n in levels:
                eng = _engine(cfg, n, storage=st)
                lbm_set_equilibrium_device(eng.ctx, starts[n])
                torch.cuda.synchronize()
                ev0.record(s)
                eng.step(cfg.horizon * (n // nc) ** 2)
                ev1.record(s)
                mm = torch.empty((3, n, n), dtype=torch.float32, device="cuda")
                eng.moments_device(mm)
                lbm_restrict(mm, n, n, n // nc, 1.0, mbuf, s)
                torch.cuda.synchronize()
                tim[st][n].append(ev0.elapsed_time(ev1))
                mh = _host(mbuf)
                err[st][n]["u_sol"].append(rel_u_sol(mh, ref_h))
                err[st][n]["u"].append(rel_u(mh, ref_h))
                eng.close()
        run = CorrectedRun(cfg, net, scales, starts[nc], use_graph=use_graph)
        if use_graph:
            run.run(0)  # capture the window graph outside the timed region
        torch.cuda.synchronize()
        ev0.record(run.stream)
        run.run(chunks)
        ev1.record(run.stream)
        torch.cuda.synchronize()
        ctim.append(ev0.elapsed_time(ev1))
        rep = run.report()
        acc += rep["n_accepted"]
        rej += rep["n_rejected"]
        run.moments(mbuf)
        torch.cuda.synchronize()
        mh = _host(mbuf)
        cerr["u_sol"].append(rel_u_sol(mh, ref_h))
        cerr["u"].append(rel_u(mh, ref_h))
        run.close()
        st0 = plain_storages[0]
        log(f"[closure] seed {seed}: u_sol plain {st0} " +
            ", ".join(f"{n}: {err[st0][n]['u_sol'][-1]:.3e}" for n in levels) +
            f"; corrected {nc}: {cerr['u_sol'][-1]:.3e} | u plain " +
            ", ".join(f"{n}: {err[st0][n]['u'][-1]:.3e}" for n in levels) +
            f"; corrected {cerr['u'][-1]:.3e} (accepted {rep['n_accepted']}, rejected {rep['n_rejected']})")
    mean = lambda v: float(np.mean(v))
    out = {"levels": list(levels), "seeds": list(seeds), "horizon": cfg.horizon, "every": cfg.every,
           "plain": {st: {"u_sol": {str(n): mean(err[st][n]["u_sol"]) for n in levels},
                          "u": {str(n): mean(err[st][n]["u"]) for n in levels},
                          "time_ms": {str(n): mean(tim[st][n]) for n in levels}} for st in plain_storages},
           "closure": {"u_sol": mean(cerr["u_sol"]), "u": mean(cerr["u"]), "time_ms": mean(ctim),
                       "accepted": acc, "rejected": rej},
           "per_seed": {"plain_coarse_u_sol": err[plain_storages[0]][nc]["u_sol"],
                        "closure_u_sol": cerr["u_sol"],
                        "plain_coarse_u": err[plain_storages[0]][nc]["u"], "closure_u": cerr["u"]}}
    # equal-error speedups over the plain FP32 scheme, on both error metrics
    ref = out["plain"][plain_storages[0]]
    out["speedup_equal_error"] = {}
    for metric in ("u_sol", "u"):
        sp = {"closure": equal_error_speedup(levels, ref[metric], ref["time_ms"], out["closure"][metric],
                                             out["closure"]["time_ms"])}
        last_dec = last_decreasing_level(levels, ref[metric])
        for st in plain_storages[1:]:
            sp[st] = {}
            for n in levels:
                if int(n) > last_dec:
                    # the plain FP32 curve is rounding-limited here: no resolution
                    # has the same error on its resolution-limited part
                    r = {"N_star": float("nan"), "speedup": float("nan"),
                         "note": "plain FP32 error rounding-limited at this level (above the previous level's): "
                                 "compare at the same resolution"}
                else:
                    r = equal_error_speedup(levels, ref[metric], ref["time_ms"], out["plain"][st][metric][str(n)],
                                            out["plain"][st]["time_ms"][str(n)])
                r["speedup_same_resolution"] = ref["time_ms"][str(n)] / out["plain"][st]["time_ms"][str(n)]
                r["error_ratio_same_resolution"] = out["plain"][st][metric][str(n)] / ref[metric][str(n)]
                sp[st][str(n)] = r
        if "f64" in out["plain"]:
            # the same comparison on the scheme's resolution-limited error
            # (the FP64 levels, free of FP32 rounding) with the FP32 run times
            r = equal_error_speedup(levels, out["plain"]["f64"][metric], ref["time_ms"], out["closure"][metric],
                                    out["closure"]["time_ms"])
            r["note"] = ("errors of the FP64 plain levels, times of the FP32 ones; " + r["note"])
            sp["closure_resolution_limited"] = r
        out["speedup_equal_error"][metric] = sp
    return out


def last_decreasing_level(levels, err) -> int:
    """The finest level up to which err(N) decreases from level to level."""
    lv = sorted(int(n) for n in levels)
    k = 1
    while k < len(lv) and float(err[str(lv[k])]) < float(err[str(lv[k - 1])]):
        k += 1
    return lv[k - 1]


def equal_error_speedup(levels, err, time_ms, e_target, t_target):
    """Speedup of a run with error e_target and wall time t_target over the
    plain FP32 scheme at equal error.  N* is the resolution at which the plain
    scheme's error equals e_target, by log-log interpolation of err(N) between
    two levels over which it still decreases (FP32 rounding, which grows with
    the N^2 steps of a run, ends the second-order decrease at fine levels);
    T_plain(N*) is interpolated log-log the same way; speedup = T_plain(N*) /
    t_target.  No extrapolation: a target error above the coarsest level's or
    below the finest decreasing level's has no equal-error point (NaN)."""
    lv = sorted(int(n) for n in levels)
    e = [float(err[str(n)]) for n in lv]
    t = [float(time_ms[str(n)]) for n in lv]
    k = 1
    while k < len(lv) and e[k] < e[k - 1]:
        k += 1
    lv, e, t = lv[:k], e[:k], t[:k]
    if not e_target < e[0]:
        return {"N_star": float("nan"), "speedup": float("nan"),
                "note": "error above the plain scheme's at the coarsest level: no equal-error point"}
    if not e_target >= e[-1]:
        return {"N_star": float("nan"), "speedup": float("nan"),
                "note": f"error below the plain scheme's at every level up to {lv[-1]} (the finest level "
                        "where its error still decreases): no equal-error point without extrapolation"}
    ln, le, lt = np.log(lv), np.log(e), np.log(t)
    lc = math.log(e_target)
    i = next(j for j in range(len(lv) - 1) if le[j + 1] <= lc)
    f = (lc - le[i]) / (le[i + 1] - le[i])
    nstar = math.exp(ln[i] + f * (ln[i + 1] - ln[i]))
    tstar = math.exp(lt[i] + f * (lt[i + 1] - lt[i]))
    return {"N_star": nstar, "speedup": tstar / t_target, "note": "interpolated"}


# trained correction network shipped with the package (written by main())
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closure_weights.npz")


def save_model(path, net, scales, cfg, history, evaluation=None):
    flat = net.p.double().cpu().numpy()
    meta = {"scales": scales, "config": {k: (list(v) if isinstance(v, tuple) else v)
                                         for k, v in asdict(cfg).items()},
            "history": history, "evaluation": evaluation}
    np.savez(path, params=flat, meta=json.dumps(meta))


def load_model(path):
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    flat = z["params"]
    params, off = [], 0
    for cin, cout in cnn.LAYERS:
        nw = cout * cin * 9
        params.append((flat[off:off + nw].reshape(cout, cin, 3, 3), flat[off + nw:off + nw + cout]))
        off += nw + cout
    return params, meta


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-seeds", type=int, default=200)
    ap.add_argument("--test-seeds", type=int, default=20)
    ap.add_argument("--pairs", type=int, default=16)
    ap.add_argument("--horizon", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--every", type=int, default=4)
    ap.add_argument("--full-targets", action="store_true",
                    help="correct rho and the whole momentum, not only its divergence-free part")
    ap.add_argument("--out", default="closure_model.npz")
    ap.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    cfg = Config(train_seeds=list(range(args.train_seeds)),
                 test_seeds=list(range(1000, 1000 + args.test_seeds)),
                 pairs_per_seed=args.pairs, horizon=args.horizon, epochs=args.epochs, lr=args.lr,
                 every=args.every, project_targets=not args.full_targets)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    x, t, scales = build_dataset(cfg, log)
    net, hist = train(cfg, x, t, log)
    del x, t
    ev = evaluate(cfg, net, scales, log)
    save_model(args.out, net, scales, cfg, hist, ev)
    out = {"scales": scales, "loss_history": hist, "evaluation": ev}
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(out, fh, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
